/*
 * ldsv.h -- C ABI of libldsv.so, an MI355X (gfx950) implementation of the
 * hot path of the learnable-differentiable finite-volume solver (Yan et al.,
 * KDD 2025): the batched time step on a periodic 2D grid (face interpolation
 * and flux stencils, viscous fluxes, Runge-Kutta stages, a spectral pressure
 * projection), with fixed or network-produced stencil coefficients, its
 * rollout and its adjoint.
 *
 * Conventions for every call
 * --------------------------
 * - Return value: LDSV_OK (0) or a negative status.  Nothing aborts or
 *   throws across the ABI.  ldsv_last_error() returns a thread-local message
 *   describing the last failure on the calling thread.
 * - Buffers: every array argument is a caller-owned DEVICE pointer (unless
 *   documented as host), valid for the duration of the stream-ordered work.
 *   The library never frees or retains caller buffers.  The handle owns its
 *   workspace (stage buffers, spectra, twiddle tables, activations).
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  All work is enqueued asynchronously on it; no call synchronises
 *   the device unless documented.  One handle must not be used from two
 *   streams at once (the workspace is shared).
 * - Layout: fields are [B][Ny][Nx] row-major, x fastest, in the grid's dtype
 *   (float for LDSV_F32, double for LDSV_F64).  MAC layout: u[b][j][i] is the
 *   x-velocity on the west face of cell (i, j), at (i dx, (j+1/2) dy);
 *   v[b][j][i] the y-velocity on its south face, at ((i+1/2) dx, j dy);
 *   pressure at cell centres (App. B.1, staggered grid, Fig. S1).
 *   COLLOCATED layout: u, v at cell centres.  Boundaries are periodic.
 * - Sizes: Nx and Ny are powers of two in [8, 4096]; MAC grids (which carry
 *   the spectral projection) are limited to 2048 (FP32) or 1024 (FP64) per
 *   axis; batch >= 1.
 */
#ifndef LDSV_H
#define LDSV_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(LDSV_BUILDING)
#define LDSV_API __attribute__((visibility("default")))
#else
#define LDSV_API
#endif

/* ---- status codes ---- */
#define LDSV_OK 0
#define LDSV_EINVAL (-1)      /* null pointer or out-of-range argument */
#define LDSV_ESHAPE (-2)      /* unsupported grid size */
#define LDSV_EDTYPE (-3)      /* call not available for the grid's dtype/layout */
#define LDSV_EHIP (-4)        /* HIP runtime error; message has the HIP code */
#define LDSV_ENONFINITE (-5)  /* guard tripped and fallback disabled */
#define LDSV_ENOMEM (-6)      /* workspace allocation failed */

/* ---- enums ---- */
#define LDSV_F32 0
#define LDSV_F64 1
#define LDSV_MAC 0           /* incompressible NS on the staggered grid */
#define LDSV_COLLOCATED 1    /* 2D viscous Burgers on cell centres */
#define LDSV_RK4 0           /* App. B.5 S15-S20, projection per sub-step */
#define LDSV_SSPRK3 1        /* Shu-Osher SSP-RK3 (Burgers configuration) */
#define LDSV_ADVECTION 1     /* physics_mask bits */
#define LDSV_VISCOSITY 2
#define LDSV_FORCING 4       /* forcing A sin(k y) and linear drag */
#define LDSV_ALL_PHYSICS 7
#define LDSV_IC_FOURIER_MODES 0
#define LDSV_IC_GRF_PEAK 1
#define LDSV_IC_TGV 2
#define LDSV_IC_SHEAR_LAYER 3

/* Number of raw network channels: 4 interpolation kinds x 16 footprint
 * points (stencil coefficients) + 2 temporal-correction channels. */
#define LDSV_NCOEF 64
#define LDSV_NOUT 66
#define LDSV_NLAYERS 6

typedef struct ldsv_handle ldsv_handle;

/* Grid: Nx x Ny cells on [0,lx) x [0,ly), `batch` independent trajectories. */
typedef struct {
  int nx, ny;
  double lx, ly;
  int batch;
  int dtype;   /* LDSV_F32 | LDSV_F64 */
  int layout;  /* LDSV_MAC | LDSV_COLLOCATED */
} ldsv_grid;

/* Physics and time-step parameters (Eq. 1 flux parameters mu, source S). */
typedef struct {
  double nu;            /* kinematic viscosity (1/Re) */
  double forcing_amp;   /* A in f_x = A sin(k y)       (App. C.1 forced flow) */
  double forcing_k;     /* k in f_x = A sin(k y)                               */
  double drag;          /* d in f = -d u                                       */
  double dt;            /* time step                                           */
  int rk;               /* LDSV_RK4 | LDSV_SSPRK3                              */
  int physics_mask;     /* LDSV_ADVECTION | LDSV_VISCOSITY | LDSV_FORCING      */
  int k_c;              /* temporal-correction interval (Eq. 2); <= 0: never  */
  double guard_threshold; /* rollout guard: max|u| bound (<= 0: finite check only) */
  int fallback_enable;  /* rollout: redo a failed learned step with plain FV   */
} ldsv_params;

/* Initial-condition shape parameters; NULL selects the defaults in (). */
typedef struct {
  double amp;        /* TGV amplitude (1)                                      */
  double k;          /* TGV wavenumber in units of 2 pi / L (1)                */
  double delta;      /* shear-layer thickness (1/30)                           */
  double pert;       /* shear-layer v perturbation amplitude (0.05)            */
  double noise_rms;  /* shear-layer noise rms (1e-3)                           */
  double kpeak;      /* GRF spectral peak (4)                                  */
} ldsv_ic_args;

/* The coefficient network: 6 conv3x3 layers 2->64->64->64->64->64->66, with
 * bias, circular padding, exact GELU after layers 0..4.  Weights are bfloat16
 * bit patterns laid out [Cout][3][3][Cin] (tap (dy,dx) row-major, Cin
 * fastest); biases float [Cout]. */
typedef struct {
  const uint16_t* w[LDSV_NLAYERS];
  const float* b[LDSV_NLAYERS];
} ldsv_net;

/* Gradient of the network parameters, float, same layouts as ldsv_net. */
typedef struct {
  float* w[LDSV_NLAYERS];
  float* b[LDSV_NLAYERS];
} ldsv_net_grad;

/* ---- lifecycle ---- */
LDSV_API int ldsv_version(void);
LDSV_API const char* ldsv_last_error(void);
/* Creates a handle for grid *g on the current HIP device and allocates its
 * workspace (about 8 state-sized arrays plus network activations when the
 * grid is LDSV_F32/LDSV_MAC).  Errors: EINVAL, ESHAPE, ENOMEM, EHIP. */
LDSV_API int ldsv_create(ldsv_handle** h, const ldsv_grid* g);
LDSV_API int ldsv_destroy(ldsv_handle* h);
/* Bytes of device workspace the handle holds. */
LDSV_API int ldsv_workspace_bytes(const ldsv_handle* h, size_t* bytes);

/* ---- a0: seeded initial conditions (App. C.1; S30-S31) ----
 * kind: LDSV_IC_FOURIER_MODES (collocated; 24 half-plane modes |k| <= 4,
 * N(0,1) cos/sin amplitudes, max|u| = 1), LDSV_IC_GRF_PEAK (MAC; Gaussian
 * random streamfunction with energy spectrum k^4 exp(-2 (k/kpeak)^2), unit
 * energy), LDSV_IC_TGV (MAC Taylor-Green vortex), LDSV_IC_SHEAR_LAYER (MAC
 * tanh shear layers + v perturbation + divergence-free noise).  Random draws:
 * SplitMix64 stream seeded seed + b * 0xD1B54A32D192ED03 for trajectory b,
 * Box-Muller normals.  Writes u, v ([B][Ny][Nx]). */
LDSV_API int ldsv_init_state(ldsv_handle* h, int kind, uint64_t seed, const ldsv_ic_args* args,
                    void* u, void* v, void* stream);

/* ---- a1-a7: the FV residual R(u) without pressure (Eq. 4; S1-S7) ----
 * coef: NULL for the physics stencil, else raw network values r, float
 * [B][64][Ny][Nx] (channel 16K+s: kind K, footprint point s), constrained on
 * the fly to c = c_P + r - mean(r) per kind and cell.  MAC/F32 only for coef.
 * Writes ru, rv. */
LDSV_API int ldsv_rhs(ldsv_handle* h, const ldsv_params* prm, const float* coef,
             const void* u, const void* v, void* ru, void* rv, void* stream);

/* ---- a1-a11: the FV module, nsteps time steps (Sec. 3.2; S15-S20) ----
 * RK4 with a projection after every sub-step (MAC) or SSP-RK3 (collocated,
 * no pressure).  coef as in ldsv_rhs (same coefficients every step).
 * In-place (u_out == u_in) is allowed.  nsteps >= 1. */
LDSV_API int ldsv_fv_step(ldsv_handle* h, const ldsv_params* prm, const float* coef,
                 const void* u_in, const void* v_in, void* u_out, void* v_out,
                 int nsteps, void* stream);

/* ---- ldsv_fv_step without a handle, allocating nothing ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * exactly what ldsv_fv_step computes on grid *g (the same kernels, arguments
 * and layouts: coef nullable, in-place allowed, nsteps >= 1) but keeps every
 * intermediate (RK stage states, accumulator, pre-projection state,
 * spectrum, twiddle and Poisson-factor tables) in one fixed device array of
 * LDSV_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends.  It makes no hipMalloc/hipFree call and calls no
 * allocating library routine; the caller passes inputs and outputs only.
 * Workspace need (each part rounded up to 256 bytes): twiddles
 * (nx + ny) * 2 * esize, and for MAC grids the FP64 Poisson factors
 * nx * ny * 8 plus the spectrum ceil(batch/2) * nx * ny * 2 * esize, then six
 * state planes of batch * nx * ny * esize (esize 4 for LDSV_F32, 8 for
 * LDSV_F64).  At 32 MiB this holds 128^2 x 64 or 256^2 x 16 FP32.  A larger
 * grid is rejected with LDSV_ESHAPE before anything is enqueued.  The array is
 * shared by every call on one device and keeps the last call's contents (the
 * tables are rewritten by each call; nothing in it needs to start at zero):
 * calls that overlap on one device, on any streams or threads, race. */
#define LDSV_NOALLOC_SCRATCH_BYTES (32u << 20)
LDSV_API int ldsv_fv_step_noalloc(const ldsv_grid* g, const ldsv_params* prm, const float* coef,
                                  const void* u_in, const void* v_in, void* u_out, void* v_out,
                                  int nsteps, void* stream);

/* ---- a9-a11: pressure projection (App. B.3-B.4; S8-S14) ----
 * u <- u - G p with D G p = D u, solved by FFT with the compact-MAC
 * eigenvalues and a zero mean mode.  p_out (nullable): the potential p,
 * [B][Ny][Nx].  MAC only.  The projection is symmetric, so it is also its
 * own adjoint (ldsv_project_bwd is the same operation). */
LDSV_API int ldsv_project(ldsv_handle* h, void* u, void* v, void* p_out, void* stream);
LDSV_API int ldsv_project_bwd(ldsv_handle* h, void* gu, void* gv, void* stream);

/* ---- a12: the coefficient network (Sec. 3.4) ----
 * out: float [B][66][Ny][Nx] (64 raw stencil values, then TC_u, TC_v).
 * A BF16 network: inputs, weights and activations are rounded to bf16
 * (round to nearest even) with FP32 accumulation, and the 64 raw stencil
 * values are returned rounded to bf16 values (their storage precision in the
 * learned step); TC_u, TC_v are FP32.  F32/MAC grids only. */
LDSV_API int ldsv_cnn_forward(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                     float* out, void* stream);

/* Copy the bf16 NHWC activation [B][Ny][Nx][64] that layer `layer` (0..4)
 * produced in the last ldsv_cnn_forward call on this handle into dst
 * (device, uint16 bit patterns).  For per-layer parity checks.  Learned
 * steps and rollouts evaluate the network too (layers 1..4 then hold their
 * activations; on grids whose sides are multiples of 16 they compute layer
 * 0 inside layer 1's tiles without storing it). */
LDSV_API int ldsv_cnn_activation(ldsv_handle* h, int layer, uint16_t* dst, void* stream);

/* ---- a12-a13: the learned step (Eq. 2) ----
 * Runs the network once on u_{k-1}, the FV module with its coefficients,
 * and, when step_index % k_c == 0, adds the temporal correction before the
 * last projection: u_k = P(FV(u_{k-1}) + TC).  step_index is k, the index
 * of the output state.  net_out (nullable): receives the network output
 * [B][66][Ny][Nx] as ldsv_cnn_forward writes it.  Without net_out the
 * stencil values stay in bf16 inside the handle (half the bytes for
 * the stage kernels); the step is the same bit for bit. */
LDSV_API int ldsv_learned_fv_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                         const float* u_in, const float* v_in, float* u_out, float* v_out,
                         int step_index, float* net_out, void* stream);

/* ---- a14: rollout (Eq. 2 recursion) ----
 * net NULL: plain FV.  Writes states u_{first+save_every-1}, ... : snapshot t
 * (t = 0 .. nsteps/save_every - 1) is the state after (t+1)*save_every steps,
 * into traj_u/traj_v [T][B][Ny][Nx].  fallback_flags (nullable, int [B]):
 * counts, per trajectory, learned steps that produced a non-finite state or
 * max(|u| + |v|) >= guard_threshold and were redone with the plain FV step
 * from the previous state (when fallback_enable), else the call returns
 * LDSV_ENONFINITE.  The guard runs on the device (a detection kernel per
 * step, the plain step launched for the flagged trajectories only): with
 * fallback_enable the call reads nothing back and can be captured in a HIP
 * graph; with the fallback disabled it synchronises once, at its end, to
 * report a trip. */
LDSV_API int ldsv_rollout(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                 const void* u0, const void* v0, int nsteps, int save_every, int first_index,
                 void* traj_u, void* traj_v, int* fallback_flags, void* stream);

/* ---- a15: adjoints ----
 * ldsv_fv_step_bwd: vector-Jacobian product of ONE fv_step at (u_in, v_in)
 * with fixed coef: given gu_out = dL/du_out, writes gu_in = dL/du_in and,
 * if gcoef != NULL and coef != NULL, ACCUMULATES dL/dr into gcoef (float
 * [B][64][Ny][Nx]).  Forward stage states are recomputed internally. */
LDSV_API int ldsv_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const float* coef,
                     const void* u_in, const void* v_in, const void* gu_out, const void* gv_out,
                     void* gu_in, void* gv_in, float* gcoef, void* stream);
/* ldsv_cnn_backward: given gout = dL/d(net output) [B][66][Ny][Nx], writes
 * gu, gv = dL/d(u, v) (nullable) and ACCUMULATES parameter gradients into
 * *dW.  Recomputes the forward activations from (u, v). */
LDSV_API int ldsv_cnn_backward(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                      const float* gout, float* gu, float* gv, const ldsv_net_grad* dW,
                      void* stream);
/* ldsv_learned_fv_step_bwd: VJP of ldsv_learned_fv_step (same arguments);
 * writes gu_in, gv_in and accumulates dW. */
LDSV_API int ldsv_learned_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                             const float* u_in, const float* v_in, int step_index,
                             const float* gu_out, const float* gv_out,
                             float* gu_in, float* gv_in, const ldsv_net_grad* dW, void* stream);

/* ldsv_rollout_bwd: unrolled backward of a learned rollout of nsteps steps
 * from (u0, v0) with activation checkpointing: the forward keeps the state
 * every checkpoint_every steps, the backward recomputes one segment at a
 * time and runs the per-step adjoint in reverse.  The cotangent of state
 * u_{first+k} (k = 0..nsteps-1, the state after k+1 steps) is
 *   loss_scale * d/du [0.5 (mean((u - lu_k)^2) + mean((v - lv_k)^2))]
 * when labels ([nsteps][B][Ny][Nx]) are given, plus g_traj_u/v[k] when
 * given.  The loss value is accumulated into *loss_dev (device double,
 * nullable).  Writes gu0, gv0 (nullable) and ACCUMULATES dW.  F32 MAC. */
LDSV_API int ldsv_rollout_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                              const float* u0, const float* v0, int nsteps, int checkpoint_every,
                              int first_index, const float* labels_u, const float* labels_v,
                              double loss_scale, const float* g_traj_u, const float* g_traj_v,
                              float* gu0, float* gv0, const ldsv_net_grad* dW, double* loss_dev,
                              void* stream);

/* ---- learned derivative stencils (Sec. 3.4: the m = d operator in per-cell
 * form; each of m = i and m = d keeps its own parameters) ----
 * dcoef: raw derivative values r, float [B][64][Ny][Nx] (channel 16K+s:
 * kind K as for coef -- K0 du/dx at the cell centre, K1 du/dy at the corner,
 * K2 dv/dx at the corner, K3 dv/dy at the cell centre -- footprint point s).
 * Per kind and cell they become the weights
 *   w = w_P + r - mean(r) - x (x . r)/16 - b (b . r)/24
 * with x_s = a_s - 1/2 and b_s the footprint point's offsets along and
 * across the face normal and w_P the fourth-order kernel [1,-27,27,-1]/24
 * (zero sum, unit normal and zero across first moment: the exact normal
 * derivative of every linear field), and the face derivative is
 * (1/h) sum_s w_s q_s in place of the fourth-order kernel.  Both coef and
 * dcoef are required (zeros give the physics stencils).  F32 MAC grids.
 *
 * ldsv_fv_step_d: the FV module with both coefficient sets (as ldsv_fv_step).
 * ldsv_fv_step_d_bwd: its VJP for one RK4 step (as ldsv_fv_step_bwd);
 *   ACCUMULATES dL/dr into gcoef and gdcoef (each nullable). */
LDSV_API int ldsv_fv_step_d(ldsv_handle* h, const ldsv_params* prm, const float* coef,
                            const float* dcoef, const void* u_in, const void* v_in, void* u_out,
                            void* v_out, int nsteps, void* stream);
LDSV_API int ldsv_fv_step_d_bwd(ldsv_handle* h, const ldsv_params* prm, const float* coef,
                                const float* dcoef, const void* u_in, const void* v_in,
                                const void* gu_out, const void* gv_out, void* gu_in, void* gv_in,
                                float* gcoef, float* gdcoef, void* stream);
/* The learned step with a second network dnet (the layer shapes of ldsv_net;
 * its 64 first outputs are the raw derivative values, its two last outputs
 * are not used) evaluated on u_{k-1} beside net: as ldsv_learned_fv_step,
 * dnet_out (nullable) receiving dnet's output [B][66][Ny][Nx].  The _bwd,
 * rollout and rollout_bwd forms are those of the coefficient network alone
 * with dnet beside net and its parameter gradients ACCUMULATED into *dWd. */
LDSV_API int ldsv_learned_d_fv_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                                    const ldsv_net* dnet, const float* u_in, const float* v_in,
                                    float* u_out, float* v_out, int step_index, float* net_out,
                                    float* dnet_out, void* stream);
LDSV_API int ldsv_learned_d_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm,
                                        const ldsv_net* net, const ldsv_net* dnet,
                                        const float* u_in, const float* v_in, int step_index,
                                        const float* gu_out, const float* gv_out, float* gu_in,
                                        float* gv_in, const ldsv_net_grad* dW,
                                        const ldsv_net_grad* dWd, void* stream);
LDSV_API int ldsv_rollout_d(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                            const ldsv_net* dnet, const void* u0, const void* v0, int nsteps,
                            int save_every, int first_index, void* traj_u, void* traj_v,
                            int* fallback_flags, void* stream);
LDSV_API int ldsv_rollout_d_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                                const ldsv_net* dnet, const float* u0, const float* v0,
                                int nsteps, int checkpoint_every, int first_index,
                                const float* labels_u, const float* labels_v, double loss_scale,
                                const float* g_traj_u, const float* g_traj_v, float* gu0,
                                float* gv0, const ldsv_net_grad* dW, const ldsv_net_grad* dWd,
                                double* loss_dev, void* stream);

/* ---- a16: loss and optimiser (Eq. 13; App. D.3) ----
 * ldsv_mse_grad: loss contribution 0.5*(mean((u-lu)^2) + mean((v-lv)^2))
 * accumulated in FP64 into *loss_dev (device double, nullable), and the
 * gradient scale*(u-lu)/n, scale*(v-lv)/n written to gu, gv. */
LDSV_API int ldsv_mse_grad(ldsv_handle* h, const float* u, const float* v, const float* lu,
                  const float* lv, double scale, float* gu, float* gv, double* loss_dev,
                  void* stream);
/* Adam with bias correction over n floats: m, v moments, step t >= 1. */
LDSV_API int ldsv_adam_step(float* w, const float* g, float* m, float* v, size_t n, int t, double lr,
                   double beta1, double beta2, double eps, void* stream);
/* Round float master weights to bfloat16 bit patterns (nearest even). */
LDSV_API int ldsv_to_bf16(const float* src, uint16_t* dst, size_t n, void* stream);

/* ---- a17: down-sampling, vorticity, correlation (Sec. 4.1; S32-S36) ----
 * MAC face averaging by integer ratio r (fine [B][r Ny][r Nx] -> coarse
 * [B][Ny][Nx] of this handle's grid). */
LDSV_API int ldsv_downsample(ldsv_handle* h, int r, const float* uf, const float* vf, float* uc,
                    float* vc, void* stream);
/* Corner vorticity w = (v - v[i-1])/dx - (u - u[j-1])/dy, [B][Ny][Nx]. */
LDSV_API int ldsv_vorticity(ldsv_handle* h, const void* u, const void* v, void* w, void* stream);
/* Pearson correlation per trajectory of two [B][Ny][Nx] fields, FP64
 * moments, written to pcc_dev (device double [B]). */
LDSV_API int ldsv_pcc(ldsv_handle* h, const void* a, const void* b, double* pcc_dev, void* stream);
/* Per-trajectory diagnostics, FP64, into diag_dev (device double [B][6]):
 * max|u|+|v|, kinetic energy 1/2<u^2+v^2>, mean u, mean v, ||D u||_2
 * (MAC only, else 0), and 1 if every value is finite else 0. */
LDSV_API int ldsv_diagnostics(ldsv_handle* h, const void* u, const void* v, double* diag_dev,
                     void* stream);
/* dt = cfl * min(dx, dy) / max over all cells and trajectories of |u|+|v|
 * (synchronises the stream; host result). */
LDSV_API int ldsv_cfl_dt(ldsv_handle* h, const void* u, const void* v, double cfl, double* dt_host,
                void* stream);

/* ---- the paper's flux block (Sec. 3.4, Eqs. 5-8) ----
 * Every interpolated face value and every face derivative of the momentum
 * residual is O_P + O_L + O_F: the physics kernel (as in ldsv_fv_step), a
 * spatially uniform learnable 5x4 kernel (O_L, Eqs. 6-7) and a per-cell
 * field from a Fourier neural operator (O_F, Eq. 8).
 *
 * Uniform kernels `stencil_w`: float [2][4][20] (device).  Index m = 0
 * interpolation, 1 derivative; kind K = 0: u along x (face at the cell
 * centre), 1: u along y (corner), 2: v along x (corner), 3: v along y (cell
 * centre), each the east or north face of the momentum volume of the cell
 * that owns it.  Point s of the 5x4 window has offset a along the face
 * normal and b across it: s = 0..11: a = s % 4 - 1, b = s / 4 - 1;
 * 12: (0,-2), 13: (1,-2), 14: (0,2), 15: (1,2), 16: (-1,-2), 17: (2,-2),
 * 18: (-1,2), 19: (2,2); along y the kernel is the transpose (q[j+a][i+b]).
 * The interpolated value adds sum_s w[0][K][s] q(a, b) and the face
 * derivative adds (1/h) sum_s w[1][K][s] q(a, b), h the spacing along the
 * normal.  `fields`: float [B][8][Ny][Nx] (device, nullable = zero):
 * channel K adds to the interpolated value of kind K, channel 4 + K to the
 * face derivative of kind K, at the face the cell owns.  The residual stays
 * conservative (every face value is single-valued).
 *
 * FNO (Li et al. 2021, the paper's frequency operator): v_0 = lift x;
 * L layers v <- GELU(K v + W v + b) with no GELU after the last; fields =
 * proj v_L.  K keeps the modes k_y in [0, M) U [Ny - M, Ny), k_x < M of the
 * real 2D transform, mixes channels per mode with complex weights and
 * applies the real inverse transform (which reads only the real part of the
 * k_x = 0 column).  Retained row r: k_y for k_y < M, k_y - Ny + 2M above.
 * F32 MAC grids with Nx * Ny <= 16384 (one LDS transform per field). */
typedef struct {
  int width;             /* C: 8 or 16 */
  int layers;            /* L >= 1 */
  int modes;             /* M: 2M <= Ny and M <= Nx/2 */
  int n_in;              /* input planes: 2 (u, v) for the flux block, 2 k_c for the
                            temporal correction */
  int n_out;             /* output channels: 4 for the flux block, 2 for the
                            temporal correction */
  const float* lift_w;   /* [C][n_in]: v_0 = lift_w x + lift_b */
  const float* lift_b;   /* [C] */
  const float* spec_w;   /* [L][C_in][C_out][2M][M] complex (re, im), 8-byte aligned */
  const float* point_w;  /* [L][C_out][C_in] */
  const float* point_b;  /* [L][C] */
  const float* proj_w;   /* [n_out][C] */
  const float* proj_b;   /* [n_out] */
} ldsv_fno;

typedef struct {
  const float* stencil_w;  /* [2][4][20] uniform kernels (device) */
  const ldsv_fno* fno[2];  /* frequency operators for m = interpolation,
                              derivative (host structs of device pointers);
                              NULL = absent (zero fields); when both are
                              given they share width, layers and modes */
} ldsv_fluxnet;

/* Gradients of the flux block's parameters (float, same layouts as
 * ldsv_fno / stencil_w), ACCUMULATED by the backward calls. */
typedef struct {
  float* lift_w;
  float* lift_b;
  float* spec_w;   /* d/dRe + i d/dIm of the loss for each complex weight */
  float* point_w;
  float* point_b;
  float* proj_w;
  float* proj_b;
} ldsv_fno_grad;

typedef struct {
  float* stencil_w;          /* [2][4][20] */
  ldsv_fno_grad* fno[2];     /* must be set where ldsv_fluxnet.fno[g] is */
} ldsv_fluxnet_grad;

/* ldsv_fno_forward: fields [B][8][Ny][Nx] = channels 0..3 from fno[0] and
 * 4..7 from fno[1] (zeros for an absent operator) on (u, v). */
LDSV_API int ldsv_fno_forward(ldsv_handle* h, const ldsv_fluxnet* net, const float* u,
                              const float* v, float* fields, void* stream);
/* ldsv_fluxblock_fv_step: nsteps RK4 steps (projection per sub-step) with
 * the flux block's uniform kernels and FIXED fields (MAC, F32 or F64; the
 * kernels and fields are FP32 in both).  In place allowed. */
LDSV_API int ldsv_fluxblock_fv_step(ldsv_handle* h, const ldsv_params* prm,
                                    const float* stencil_w, const float* fields,
                                    const void* u_in, const void* v_in, void* u_out, void* v_out,
                                    int nsteps, void* stream);
/* ldsv_fluxblock_fv_step_bwd: VJP of one ldsv_fluxblock_fv_step: writes
 * gu_in, gv_in and ACCUMULATES dL/dstencil_w into gstencil (float [160],
 * nullable) and dL/dfields into gfields ([B][8][Ny][Nx], nullable).  The
 * kernel gradient is reduced in a fixed order (deterministic). */
LDSV_API int ldsv_fluxblock_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm,
                                        const float* stencil_w, const float* fields,
                                        const void* u_in, const void* v_in, const void* gu_out,
                                        const void* gv_out, void* gu_in, void* gv_in,
                                        float* gstencil, float* gfields, void* stream);
/* ldsv_fno_backward: VJP of ldsv_fno_forward (the forward is recomputed
 * with its activations kept): given gfields = dL/dfields, ACCUMULATES the
 * FNO parameter gradients into grad->fno[g] and writes gu, gv = dL/d(u, v)
 * (nullable together).  Parameter gradients are reduced in a fixed order
 * (deterministic). */
LDSV_API int ldsv_fno_backward(ldsv_handle* h, const ldsv_fluxnet* net, const float* u,
                               const float* v, const float* gfields, float* gu, float* gv,
                               const ldsv_fluxnet_grad* grad, void* stream);
/* ldsv_fluxblock_step_bwd: VJP of ldsv_fluxblock_step: writes gu_in, gv_in
 * (through the FV step and through the FNOs) and ACCUMULATES every
 * parameter gradient into *grad. */
LDSV_API int ldsv_fluxblock_step_bwd(ldsv_handle* h, const ldsv_params* prm,
                                     const ldsv_fluxnet* net, const float* u_in,
                                     const float* v_in, const float* gu_out, const float* gv_out,
                                     float* gu_in, float* gv_in, const ldsv_fluxnet_grad* grad,
                                     void* stream);
/* ---- the paper's temporal correction block (Eq. 2; Sec. 3.5) ----
 * ldsv_fluxblock_tc_step: one step of the complete model.  u_k = FV(u_{k-1})
 * with the flux block (fields from net's FNOs on u_{k-1}); when step_index
 * (= k) is a multiple of prm->k_c and tc is given, the correction
 * TC = tc(u_{k-k_c}, v_{k-k_c}, ..., u_{k-1}, v_{k-1}) (an FNO with
 * n_in = 2 k_c planes, oldest state first, and n_out = 2) is added before
 * the last projection, u_k = P(FV(u_{k-1}) + TC).  hist_u, hist_v: HOST
 * arrays of k_c DEVICE pointers to the states u_{k-k_c} .. u_{k-1} (the last
 * one is the step's input; the others are read only when the correction is
 * applied).  Not in place. */
LDSV_API int ldsv_fluxblock_tc_step(ldsv_handle* h, const ldsv_params* prm,
                                    const ldsv_fluxnet* net, const ldsv_fno* tc,
                                    const float* const* hist_u, const float* const* hist_v,
                                    int step_index, float* u_out, float* v_out, void* stream);
/* ldsv_fluxblock_tc_step_bwd: VJP of ldsv_fluxblock_tc_step: given gu_out,
 * gv_out = dL/du_k, ACCUMULATES dL/d(history state j) into ghist_u[j],
 * ghist_v[j] (host arrays of k_c device pointers, same order as hist_u),
 * the flux-block parameter gradients into *grad and the correction's into
 * *gtc (nullable when tc is). */
LDSV_API int ldsv_fluxblock_tc_step_bwd(ldsv_handle* h, const ldsv_params* prm,
                                        const ldsv_fluxnet* net, const ldsv_fno* tc,
                                        const float* const* hist_u, const float* const* hist_v,
                                        int step_index, const float* gu_out, const float* gv_out,
                                        float* const* ghist_u, float* const* ghist_v,
                                        const ldsv_fluxnet_grad* grad, const ldsv_fno_grad* gtc,
                                        void* stream);

/* ldsv_fluxblock_step: one step of the flux-block model, u_out = FV(u_in)
 * with fields = FNO(u_in) (evaluated once, held over the four sub-steps).
 * fields_out (nullable) receives the fields.  Not in place. */
LDSV_API int ldsv_fluxblock_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_fluxnet* net,
                                 const float* u_in, const float* v_in, float* u_out, float* v_out,
                                 float* fields_out, void* stream);

/* ---- shear flow with a passive scalar (the shear-flow equations of the
 * appendix on the datasets) ----
 * s at cell centres ([B][Ny][Nx], the grid's dtype), carried by the MAC
 * velocity: ds/dt - D lap s = -u . grad s in flux form (face velocity times
 * the midpoint average of s, fourth-order face derivative for the
 * diffusion); the total of s is conserved.
 * ldsv_fv_step_scalar: nsteps RK4 steps of the plain velocity (as
 * ldsv_fv_step, projection per sub-step) and of s, whose stage residuals use
 * the velocity's stage states.  MAC, RK4.  In place allowed. */
LDSV_API int ldsv_fv_step_scalar(ldsv_handle* h, const ldsv_params* prm, double diffusivity,
                                 const void* u_in, const void* v_in, const void* s_in,
                                 void* u_out, void* v_out, void* s_out, int nsteps,
                                 void* stream);
/* ldsv_init_scalar: s = (1 + prof(y)) / 2 with prof the shear profile of
 * ldsv_init_state's SHEAR_LAYER (layers at Ly/4 and 3Ly/4, thickness
 * args->delta; NULL args: 1/30): the scalar aligned with the shear layers. */
LDSV_API int ldsv_init_scalar(ldsv_handle* h, const ldsv_ic_args* args, void* s, void* stream);

/* ---- measurement ----
 * Kernel classes timed by ldsv_timer_*: 0 RK stage (fused residual), 1 row
 * FFT + divergence, 2 column FFT + Poisson division, 3 inverse row FFT +
 * gradient correction, 4 convolution (MFMA), 5 first convolution layer,
 * 6 adjoint stage, 7 other, 8 FNO transforms, 9 FNO mode mixing.  While enabled, every launch of a class is
 * bracketed by HIP events on its stream.  ldsv_timer_read synchronises the
 * device and returns the summed duration (ms) and the launch count. */
LDSV_API int ldsv_timer_enable(ldsv_handle* h, int on);
LDSV_API int ldsv_timer_read(ldsv_handle* h, int cls, double* total_ms, int* count);

#ifdef __cplusplus
}
#endif
#endif /* LDSV_H */
