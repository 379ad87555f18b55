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
// stage overwrites the velocity stage buffer).  One thread per cell; the 9
// scalar values of the two face-derivative stencils and the four face
// velocities come through L1/L2 (a wavefront covers 64 consecutive cells of
// a row, so the x neighbours are the same lines and the y neighbours the
// rows next to it).
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

template <typename T>
__global__ void __launch_bounds__(kBlock) k_stage_scalar(
    const T* __restrict__ us, const T* __restrict__ vs, const T* __restrict__ ss,
    const T* __restrict__ sn, const T* __restrict__ acc, T* __restrict__ out,
    T* __restrict__ oacc, ScalarStagePhys<T> ph, ScalarComb<T> cb, int nx, int ny, int batch) {
  const size_t n = (size_t)nx * ny;
  const size_t total = n * batch;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (size_t)gridDim.x * blockDim.x) {
    const size_t b0 = (g / n) * n;
    const size_t c = g - b0;
    const int i = (int)(c % nx), j = (int)(c / nx);
    auto at = [&](const T* p, int ii, int jj) {
      return p[b0 + (size_t)(jj & (ny - 1)) * nx + (ii & (nx - 1))];
    };
    const T s0 = ss[g];
    T r = 0;
    if (ph.mask & LDSV_ADVECTION) {
      const T se = at(ss, i + 1, j), sw = at(ss, i - 1, j);
      const T sN = at(ss, i, j + 1), sS = at(ss, i, j - 1);
      const T fe = at(us, i + 1, j) * (T)0.5 * (s0 + se);
      const T fw = us[g] * (T)0.5 * (sw + s0);
      const T gn = at(vs, i, j + 1) * (T)0.5 * (s0 + sN);
      const T gs = vs[g] * (T)0.5 * (sS + s0);
      r = -(fe - fw) * ph.idx - (gn - gs) * ph.idy;
    }
    if (ph.mask & LDSV_VISCOSITY) {
      const T sm2 = at(ss, i - 2, j), sm1 = at(ss, i - 1, j), sp1 = at(ss, i + 1, j),
              sp2 = at(ss, i + 2, j);
      const T tm2 = at(ss, i, j - 2), tm1 = at(ss, i, j - 1), tp1 = at(ss, i, j + 1),
              tp2 = at(ss, i, j + 2);
      const T de = (sm1 - (T)27 * s0 + (T)27 * sp1 - sp2) * ph.i24dx;
      const T dw = (sm2 - (T)27 * sm1 + (T)27 * s0 - sp1) * ph.i24dx;
      const T dn = (tm1 - (T)27 * s0 + (T)27 * tp1 - tp2) * ph.i24dy;
      const T ds = (tm2 - (T)27 * tm1 + (T)27 * s0 - tp1) * ph.i24dy;
      r += ph.diff * ((de - dw) * ph.idx + (dn - ds) * ph.idy);
    }
    T o = cb.beta * s0 + cb.eps * r;
    if (cb.alpha != (T)0) o += cb.alpha * sn[g];
    T a = 0;
    if (cb.delta != (T)0 || cb.gamma != (T)0) a = acc[g];
    o += cb.delta * a;
    out[g] = o;
    if (oacc) oacc[g] = cb.gamma * a + cb.wacc * r;
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
  LDSV_TLAUNCH(h, 7, k_stage_scalar<T>, grid1d(h->nstate), dim3(kBlock), 0, st, (const T*)us,
               (const T*)vs, (const T*)ss, (const T*)sn, (const T*)acc, (T*)out, (T*)oacc, ph, cb,
               h->g.nx, h->g.ny, h->g.batch);
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
