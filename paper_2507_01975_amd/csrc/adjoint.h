// Host-side interface of the adjoint kernels.
#pragma once

#include "internal.h"
#include "stage.h"

int ldsv_ensure_adjoint(ldsv_handle* h);
int ldsv_launch_adj_rhs(ldsv_handle* h, const ldsv_params* prm, const float* coef, size_t cbs,
                        float* gcoef, size_t gcbs, const void* us, const void* vs, const void* Au,
                        const void* Av, const void* Gu, const void* Gv, double aA, double aG,
                        const void* addu, const void* addv, void* ou, void* ov, hipStream_t st,
                        const FluxBlockArgs* fb = nullptr, const DerivCoef* dc = nullptr);
int ldsv_launch_axpy2(ldsv_handle* h, void* yu, void* yv, const void* xu, const void* xv, double a,
                      hipStream_t st);
// VJP of one RK4 step at (su, sv) with fixed coefficients; gcoef accumulates
// dL/dr (nullable); with dc the step also used per-cell derivative values
// dc->d (float, stride cbs) and dc->gd accumulates their gradient (stride
// gcbs, nullable).
int ldsv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const float* coef, size_t cbs,
                  float* gcoef, size_t gcbs, const void* su, const void* sv, const void* gu_out,
                  const void* gv_out, void* gu_in, void* gv_in, hipStream_t st,
                  const FluxBlockArgs* fb = nullptr, const DerivCoef* dc = nullptr);
