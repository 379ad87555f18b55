// Passive scalar of the shear-flow system (the shear-flow equations of the
// appendix on the datasets): ds/dt - D lap s = -u . grad s, with s at cell
// centres carried by the MAC velocity.
//
// Finite-volume residual of cell (i, j), the velocity already on its faces:
//   R_s = -[(u_e s~_e - u_w s~_w)/dx + (v_n s~_n - v_s s~_s)/dy]
//         + D [((ds/dx)_e - (ds/dx)_w)/dx + ((ds/dy)_n - (ds/dy)_s)/dy]
// with the physics kernels of the flux block (App. B.2, S6-S7): s~ the
// midpoint average across a face and ds/dn the fourth-order face
// derivative [1, -27, 27, -1]/(24 h).  Fluxes telescope, so the total of s
// is conserved to rounding.
//
// k_stage_scalar is one RK stage of the scalar, fused with its residual:
//   out = alpha s_n + beta s_s + delta acc + eps R(u_s, s_s),
//   acc' = gamma acc + wacc R
// with the velocity's stage coefficients and the velocity's stage state;
// the RK loop launches it before each velocity stage (the projection of that
// stage overwrites the velocity stage buffer).  As the velocity's stage
// kernel, one workgroup owns a TX x TY tile: the scalar with a 2-cell
// periodic halo, the u column east of the tile and the v row north of it are
// staged in LDS (all global loads of a thread in flight before the LDS
// stores), every face flux is formed once, and the residual and the RK
// combination stay in registers.  Tiles are renumbered XCD-contiguously so a
// tile's halo lines are L2 hits.
#include "internal.h"

namespace {

template <typename T>
struct ScalarStagePhys {
  T idx, idy, i24dx, i24dy, diff;
  int mask;
};

template <typename T>
struct ScalarComb {
  T alpha, beta, delta, eps, gamma, wacc;
};

constexpr int kSTX = 64, kSTY = 16, kSH = 2;

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(kBlock) k_stage_scalar(
    const T* __restrict__ us, const T* __restrict__ vs, const T* __restrict__ ss,
    const T* __restrict__ sn, const T* __restrict__ acc, T* __restrict__ out,
    T* __restrict__ oacc, ScalarStagePhys<T> ph, ScalarComb<T> cb, int nx, int ny) {
  constexpr int W = TX + 2 * kSH, H = TY + 2 * kSH;
  constexpr int kS = W * H, kU = TY * (TX + 1), kV = (TY + 1) * TX;
  constexpr int kSPer = (kS + kBlock - 1) / kBlock, kUPer = (kU + kBlock - 1) / kBlock,
                kVPer = (kV + kBlock - 1) / kBlock;
  constexpr int kCells = TX * TY, kCellPer = (kCells + kBlock - 1) / kBlock;
  __shared__ T sl[H][W];
  __shared__ T ul[TY][TX + 1];
  __shared__ T vl[TY + 1][TX];
  const int tilesx = nx / TX;
  const int tile = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int b = tile / gridDim.x;
  const int tp = tile - b * gridDim.x;
  const int i0 = (tp % tilesx) * TX, j0 = (tp / tilesx) * TY;
  const size_t boff = (size_t)b * nx * ny;
  {
    T ts[kSPer], tu[kUPer], tv[kVPer];
#pragma unroll
    for (int k = 0; k < kSPer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kS) {
        const int r = t / W, c = t - r * W;
        ts[k] = ss[boff + (size_t)((j0 - kSH + r + ny) & (ny - 1)) * nx + ((i0 - kSH + c + nx) & (nx - 1))];
      }
    }
#pragma unroll
    for (int k = 0; k < kUPer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kU) {
        const int r = t / (TX + 1), c = t - r * (TX + 1);
        tu[k] = us[boff + (size_t)(j0 + r) * nx + ((i0 + c) & (nx - 1))];
      }
    }
#pragma unroll
    for (int k = 0; k < kVPer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kV) {
        const int r = t / TX, c = t - r * TX;
        tv[k] = vs[boff + (size_t)((j0 + r) & (ny - 1)) * nx + (i0 + c)];
      }
    }
#pragma unroll
    for (int k = 0; k < kSPer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kS) sl[t / W][t % W] = ts[k];
    }
#pragma unroll
    for (int k = 0; k < kUPer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kU) ul[t / (TX + 1)][t % (TX + 1)] = tu[k];
    }
#pragma unroll
    for (int k = 0; k < kVPer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kV) vl[t / TX][t % TX] = tv[k];
    }
  }
  // operands of the RK combination, loaded before the barrier
  T pn[kCellPer], pa[kCellPer];
  const bool need_n = cb.alpha != (T)0, need_a = cb.delta != (T)0 || cb.gamma != (T)0;
#pragma unroll
  for (int k = 0; k < kCellPer; ++k) {
    const int t = k * kBlock + (int)threadIdx.x;
    pn[k] = pa[k] = (T)0;
    if (t < kCells) {
      const size_t g = boff + (size_t)(j0 + t / TX) * nx + (i0 + t % TX);
      if (need_n) pn[k] = sn[g];
      if (need_a) pa[k] = acc[g];
    }
  }
  __syncthreads();
  const bool adv = ph.mask & LDSV_ADVECTION, visc = ph.mask & LDSV_VISCOSITY;
#pragma unroll
  for (int k = 0; k < kCellPer; ++k) {
    const int t = k * kBlock + (int)threadIdx.x;
    if (t >= kCells) break;
    const int r = t / TX, c = t - r * TX;
    const int lj = r + kSH, li = c + kSH;
    const T s0 = sl[lj][li];
    T rr = 0;
    if (adv) {
      const T fe = ul[r][c + 1] * (T)0.5 * (s0 + sl[lj][li + 1]);
      const T fw = ul[r][c] * (T)0.5 * (sl[lj][li - 1] + s0);
      const T gn = vl[r + 1][c] * (T)0.5 * (s0 + sl[lj + 1][li]);
      const T gs = vl[r][c] * (T)0.5 * (sl[lj - 1][li] + s0);
      rr = -(fe - fw) * ph.idx - (gn - gs) * ph.idy;
    }
    if (visc) {
      const T de = (sl[lj][li - 1] - (T)27 * s0 + (T)27 * sl[lj][li + 1] - sl[lj][li + 2]) * ph.i24dx;
      const T dw = (sl[lj][li - 2] - (T)27 * sl[lj][li - 1] + (T)27 * s0 - sl[lj][li + 1]) * ph.i24dx;
      const T dn = (sl[lj - 1][li] - (T)27 * s0 + (T)27 * sl[lj + 1][li] - sl[lj + 2][li]) * ph.i24dy;
      const T ds = (sl[lj - 2][li] - (T)27 * sl[lj - 1][li] + (T)27 * s0 - sl[lj + 1][li]) * ph.i24dy;
      rr += ph.diff * ((de - dw) * ph.idx + (dn - ds) * ph.idy);
    }
    const size_t g = boff + (size_t)(j0 + r) * nx + (i0 + c);
    out[g] = cb.beta * s0 + cb.eps * rr + cb.alpha * pn[k] + cb.delta * pa[k];
    if (oacc) oacc[g] = cb.gamma * pa[k] + cb.wacc * rr;
  }
}

template <typename T>
int launch_scalar_t(ldsv_handle* h, const ldsv_params* prm, double diff, const void* us,
                    const void* vs, const void* ss, const void* sn, const void* acc, void* out,
                    void* oacc, double alpha, double beta, double delta, double eps, double gamma,
                    double wacc, hipStream_t st) {
  const double dx = h->g.lx / h->g.nx, dy = h->g.ly / h->g.ny;
  ScalarStagePhys<T> ph{(T)(1.0 / dx), (T)(1.0 / dy), (T)(1.0 / (24.0 * dx)),
                        (T)(1.0 / (24.0 * dy)), (T)diff, prm->physics_mask};
  ScalarComb<T> cb{(T)alpha, (T)beta, (T)delta, (T)eps, (T)gamma, (T)wacc};
  const int nx = h->g.nx, ny = h->g.ny;
#define LDSV_SCALAR_CASE(tx, ty)                                                              \
  if (nx >= tx && ny >= ty) {                                                                 \
    dim3 grid((nx / tx) * (ny / ty), h->g.batch);                                             \
    LDSV_TLAUNCH(h, 7, (k_stage_scalar<T, tx, ty>), grid, dim3(kBlock), 0, st, (const T*)us,  \
                 (const T*)vs, (const T*)ss, (const T*)sn, (const T*)acc, (T*)out, (T*)oacc,  \
                 ph, cb, nx, ny);                                                             \
  }
  LDSV_SCALAR_CASE(kSTX, kSTY)
  else LDSV_SCALAR_CASE(32, 8) else LDSV_SCALAR_CASE(8, 8)
#undef LDSV_SCALAR_CASE
  LDSV_LAUNCHED();
  return LDSV_OK;
}

// s = (1 + prof(y)) / 2 at cell centres, prof the shear profile: layers at
// L_y/4 and 3 L_y/4 of thickness delta
template <typename T>
__global__ void k_init_scalar(T* s, int nx, int ny, int batch, double ly, double delta) {
  const size_t n = (size_t)nx * ny;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n * batch;
       g += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)((g % n) / nx);
    const double y = (j + 0.5) * ly / ny;
    const double prof =
        (y <= 0.5 * ly) ? tanh((y - 0.25 * ly) / delta) : -tanh((y - 0.75 * ly) / delta);
    s[g] = (T)(0.5 * (1.0 + prof));
  }
}

}  // namespace

int ldsv_launch_scalar_stage(ldsv_handle* h, const ldsv_params* prm, double diff, const void* us,
                             const void* vs, const void* ss, const void* sn, const void* acc,
                             void* out, void* oacc, double alpha, double beta, double delta,
                             double eps, double gamma, double wacc, hipStream_t st) {
  if (h->g.dtype == LDSV_F64)
    return launch_scalar_t<double>(h, prm, diff, us, vs, ss, sn, acc, out, oacc, alpha, beta,
                                   delta, eps, gamma, wacc, st);
  return launch_scalar_t<float>(h, prm, diff, us, vs, ss, sn, acc, out, oacc, alpha, beta, delta,
                                eps, gamma, wacc, st);
}

int ldsv_internal_step_scalar(ldsv_handle* h, const ldsv_params* p, double diff, const void* su,
                              const void* sv, const void* ss, void* du, void* dv, void* ds,
                              hipStream_t st);

extern "C" {

int ldsv_init_scalar(ldsv_handle* h, const ldsv_ic_args* args, void* s, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(s, LDSV_EINVAL, "init_scalar: null output");
  const double delta = args ? args->delta : 1.0 / 30.0;
  LDSV_REQUIRE(delta > 0, LDSV_EINVAL, "init_scalar: delta=%g", delta);
  const hipStream_t st = (hipStream_t)stream;
  if (h->g.dtype == LDSV_F64)
    LDSV_TLAUNCH(h, 7, k_init_scalar<double>, grid1d(h->nstate), dim3(kBlock), 0, st, (double*)s,
                 h->g.nx, h->g.ny, h->g.batch, h->g.ly, delta);
  else
    LDSV_TLAUNCH(h, 7, k_init_scalar<float>, grid1d(h->nstate), dim3(kBlock), 0, st, (float*)s,
                 h->g.nx, h->g.ny, h->g.batch, h->g.ly, delta);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

int ldsv_fv_step_scalar(ldsv_handle* h, const ldsv_params* prm, double diffusivity,
                        const void* u_in, const void* v_in, const void* s_in, void* u_out,
                        void* v_out, void* s_out, int nsteps, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && u_in && v_in && s_in && u_out && v_out && s_out, LDSV_EINVAL,
               "fv_step_scalar: null argument");
  LDSV_REQUIRE(nsteps >= 1, LDSV_EINVAL, "fv_step_scalar: nsteps=%d", nsteps);
  LDSV_REQUIRE(diffusivity >= 0, LDSV_EINVAL, "fv_step_scalar: diffusivity=%g", diffusivity);
  LDSV_REQUIRE(h->g.layout == LDSV_MAC && prm->rk == LDSV_RK4, LDSV_EDTYPE,
               "fv_step_scalar: RK4 on the MAC layout");
  const hipStream_t st = (hipStream_t)stream;
  for (int k = 0; k < nsteps; ++k)
    LDSV_TRY(ldsv_internal_step_scalar(h, prm, diffusivity, k ? u_out : u_in, k ? v_out : v_in,
                                       k ? s_out : s_in, u_out, v_out, s_out, st));
  return LDSV_OK;
}

}  // extern "C"
