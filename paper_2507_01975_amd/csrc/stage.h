// Host-side interface of the fused RK stage kernels.
#pragma once

#include "internal.h"

// One Runge-Kutta stage, fused with the finite-volume residual R(us):
//   out   = alpha * un + beta * us + delta * acc + eps * R(us) [+ tc]
//   acc'  = gamma * acc + wacc * R(us)
// (delta and eps include the time step).  Pointers marked nullable are
// skipped when their coefficient is zero / when absent.
struct StageArgs {
  const void* us = nullptr;
  const void* vs = nullptr;
  const void* un = nullptr;   // nullable when alpha == 0
  const void* vn = nullptr;
  const void* accu = nullptr; // nullable when delta == 0 and gamma == 0
  const void* accv = nullptr;
  void* ou = nullptr;
  void* ov = nullptr;
  void* oaccu = nullptr;      // nullable: no accumulator output
  void* oaccv = nullptr;
  const float* coef = nullptr;  // raw learned stencil values, planar, nullable
  size_t coef_bstride = 0;      // elements between trajectories
  const uint16_t* coef16 = nullptr;  // the same in bf16 [B][8][Ny][Nx][8] (used when set)
  size_t coef16_bstride = 0;
  // per-cell learned derivative values, raw, with the layout and batch
  // stride of coef (dcoef) or coef16 (dcoef16); used only together with them
  const float* dcoef = nullptr;
  const uint16_t* dcoef16 = nullptr;
  const float* tcu = nullptr;   // temporal correction added to out, nullable
  const float* tcv = nullptr;
  size_t tc_bstride = 0;
  // flux block (used when fbw is set): uniform kernels [2][4][20] (interp,
  // deriv) and optional fields [B][8][Ny][Nx]
  const float* fbw = nullptr;
  const float* fbf = nullptr;
  size_t fb_bstride = 0;
  double alpha = 0, beta = 0, delta = 0, eps = 0, gamma = 0, wacc = 0;
  // per-trajectory mask (int [B], nullable; MAC only): the workgroups of a
  // trajectory whose entry is 0 return at once and write nothing
  const int* active = nullptr;
};

// Flux-block operands of a step (Sec. 3.4, Eqs. 5-8): uniform kernels
// w [2][4][20] (interp, deriv; FP32, device) and per-cell fields
// f [B][8][Ny][Nx] (FP32, nullable; batch stride fbs).  The adjoint
// accumulates dL/dw into gw [160] and dL/df into gf (same layout, batch
// stride gfbs); both nullable.
struct FluxBlockArgs {
  const float* w = nullptr;
  const float* f = nullptr;
  size_t fbs = 0;
  float* gw = nullptr;
  float* gf = nullptr;
  size_t gfbs = 0;
};

// Per-cell learned derivative stencils (Sec. 3.4, the m = d operator in
// per-cell form): raw values r [B][64][Ny][Nx] (channel 16K + s), float (d)
// or bf16 (d16, [B][8][Ny][Nx][8]), with the batch stride of the interpolation
// coefficients they accompany.  Per kind and cell the weights are
//   w = w_P + r - mean(r) - x (x . r)/16 - b (b . r)/24
// (x_s = a_s - 1/2 along the face normal, b_s across, w_P the fourth-order
// kernel), and the face derivative is (1/h) sum_s w_s q_s.  The adjoint
// accumulates dL/dr into gd (float, nullable, the gradient batch stride).
struct DerivCoef {
  const float* d = nullptr;
  const uint16_t* d16 = nullptr;
  float* gd = nullptr;
};

int ldsv_launch_stage(ldsv_handle* h, const ldsv_params* prm, const StageArgs& a,
                      hipStream_t st);
// active (int [B], nullable): only trajectories whose entry is nonzero are
// projected and written; the others' outputs are left untouched
int ldsv_launch_project(ldsv_handle* h, const void* us, const void* vs, void* uo, void* vo,
                        void* po, hipStream_t st, const int* active = nullptr);
