// C-ABI entry points of libldsv: argument checking, workspace management and
// the stream-ordered orchestration of the kernels (RK stages, projections,
// rollout loop).  Every numerical step runs in the HIP kernels of the other
// translation units.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "adjoint.h"
#include "reduce.h"
#include "stage.h"

int ldsv_launch_init(ldsv_handle* h, int kind, uint64_t seed, const ldsv_ic_args* args, void* u,
                     void* v, hipStream_t st);
int ldsv_launch_diagnostics(ldsv_handle* h, const void* u, const void* v, double* out,
                            hipStream_t st);
int ldsv_launch_maxspeed(ldsv_handle* h, const void* u, const void* v, double* out,
                         hipStream_t st);
int ldsv_launch_downsample(ldsv_handle* h, int r, const float* uf, const float* vf, float* uc,
                           float* vc, hipStream_t st);
int ldsv_launch_vorticity(ldsv_handle* h, const void* u, const void* v, void* w, hipStream_t st);
int ldsv_launch_pcc(ldsv_handle* h, const void* a, const void* b, double* out, hipStream_t st);
int ldsv_launch_scalar_stage(ldsv_handle* h, const ldsv_params* prm, double diff, const void* us,
                             const void* vs, const void* ss, const void* sn, const void* acc,
                             void* out, void* oacc, double alpha, double beta, double delta,
                             double eps, double gamma, double wacc, hipStream_t st);
int ldsv_launch_mse_grad(ldsv_handle* h, const float* u, const float* v, const float* lu,
                         const float* lv, double scale, float* gu, float* gv, double* loss,
                         hipStream_t st, int accumulate);

namespace {
thread_local char g_err[512] = "";
}

void ldsv_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int ldsv_alloc(ldsv_handle* h, void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    ldsv_set_error("%s: cannot allocate %zu bytes", what, bytes);
    return LDSV_ENOMEM;
  }
  h->allocs.push_back(*p);
  h->bytes += bytes;
  return LDSV_OK;
}

int ldsv_check_handle(const ldsv_handle* h) {
  LDSV_REQUIRE(h != nullptr, LDSV_EINVAL, "null handle");
  return LDSV_OK;
}

int ldsv_check_params(const ldsv_handle* h, const ldsv_params* p) {
  LDSV_REQUIRE(p != nullptr, LDSV_EINVAL, "null params");
  LDSV_REQUIRE(std::isfinite(p->dt) && std::isfinite(p->nu) && p->nu >= 0.0, LDSV_EINVAL,
               "params: dt and nu must be finite, nu >= 0");
  LDSV_REQUIRE(p->rk == LDSV_RK4 || p->rk == LDSV_SSPRK3, LDSV_EINVAL, "params: rk must be RK4 or SSPRK3");
  LDSV_REQUIRE(p->physics_mask >= 0 && p->physics_mask <= 7, LDSV_EINVAL, "params: bad physics_mask");
  (void)h;
  return LDSV_OK;
}

namespace {

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

bool pow2_in_range(int n) { return n >= 8 && n <= 4096 && (n & (n - 1)) == 0; }


template <typename T>
std::vector<Cx<T>> twiddles(int n) {
  std::vector<Cx<T>> t(n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int m = 0; m < n; ++m) {
    const double a = two_pi * (double)m / (double)n;
    t[m] = Cx<T>{(T)std::cos(a), (T)(-std::sin(a))};
  }
  return t;
}

// a passive scalar stepped with the velocity: s_in -> s_out (in place
// allowed), diffusivity D
struct ScalarStep {
  const void* s_in;
  void* s_out;
  double diff;
};

// one time step src -> dst (dst may equal src).  keep (nullable, RK4/MAC):
// the projected stage states u1, u2, u3 are written to keep[2s], keep[2s+1]
// (state-sized planes) instead of the shared stage buffer.
int one_step(ldsv_handle* h, const ldsv_params* p, const float* coef, size_t cbs, const void* su,
             const void* sv, void* du, void* dv, const float* tcu, const float* tcv, size_t tcbs,
             hipStream_t st, void* keep = nullptr, const uint16_t* coef16 = nullptr,
             size_t cbs16 = 0, const FluxBlockArgs* fb = nullptr,
             const ScalarStep* sc = nullptr, const DerivCoef* dc = nullptr,
             const int* active = nullptr) {
  const size_t sbk = h->nstate * h->esize;
  auto ku = [&](int s) -> void* { return keep ? (char*)keep + (size_t)(2 * s) * sbk : h->ws_u; };
  auto kv = [&](int s) -> void* { return keep ? (char*)keep + (size_t)(2 * s + 1) * sbk : h->ws_v; };
  const double dt = p->dt;
  const bool mac = h->g.layout == LDSV_MAC;
  StageArgs a;
  a.active = active;
  a.coef = coef;
  a.coef_bstride = cbs;
  a.coef16 = coef16;
  a.coef16_bstride = cbs16;
  if (dc) {
    a.dcoef = coef ? dc->d : nullptr;
    a.dcoef16 = coef16 ? dc->d16 : nullptr;
  }
  if (fb) {
    a.fbw = fb->w;
    a.fbf = fb->f;
    a.fb_bstride = fb->fbs;
  }
  if (p->rk == LDSV_RK4) {
    const double eps[4] = {0.5 * dt, 0.5 * dt, dt, dt / 6.0};
    for (int s = 0; s < 4; ++s) {
      a.us = (s == 0) ? su : ku(s - 1);
      a.vs = (s == 0) ? sv : kv(s - 1);
      a.un = (s == 0) ? nullptr : su;
      a.vn = (s == 0) ? nullptr : sv;
      a.alpha = (s == 0) ? 0.0 : 1.0;
      a.beta = (s == 0) ? 1.0 : 0.0;
      a.eps = eps[s];
      a.delta = (s == 3) ? dt / 6.0 : 0.0;
      a.gamma = (s == 1 || s == 2) ? 1.0 : 0.0;
      a.wacc = (s == 0) ? 1.0 : 2.0;
      a.accu = h->acc_u;
      a.accv = h->acc_v;
      a.oaccu = (s < 3) ? h->acc_u : nullptr;
      a.oaccv = (s < 3) ? h->acc_v : nullptr;
      a.tcu = (s == 3) ? tcu : nullptr;
      a.tcv = (s == 3) ? tcv : nullptr;
      a.tc_bstride = tcbs;
      if (sc) {
        // the scalar's stage reads the velocity stage state before this
        // stage's projection overwrites it; its stage states ping-pong
        const size_t sbs = h->nstate * h->esize;
        char* sws = (char*)h->sc_ws;
        const void* sin = (s == 0) ? sc->s_in : sws + ((s + 1) & 1) * sbs;
        void* sout = (s == 3) ? sc->s_out : sws + (s & 1) * sbs;
        void* sacc = sws + 2 * sbs;
        LDSV_TRY(ldsv_launch_scalar_stage(h, p, sc->diff, a.us, a.vs, sin, sc->s_in, sacc, sout,
                                          (s < 3) ? sacc : nullptr, a.alpha, a.beta, a.delta,
                                          a.eps, a.gamma, a.wacc, st));
      }
      if (mac) {
        a.ou = h->st_u;
        a.ov = h->st_v;
        LDSV_TRY(ldsv_launch_stage(h, p, a, st));
        h->speed_now = s == 3 ? h->speed_out : nullptr;
        const int rp = ldsv_launch_project(h, h->st_u, h->st_v, s == 3 ? du : ku(s),
                                           s == 3 ? dv : kv(s), nullptr, st, active);
        h->speed_now = nullptr;
        LDSV_TRY(rp);
      } else {
        // collocated RK4 without projection: stage outputs ping-pong
        LDSV_REQUIRE(false, LDSV_EDTYPE, "RK4 on the collocated layout is not provided; use SSPRK3");
      }
    }
    return LDSV_OK;
  }
  // SSP-RK3 (Shu-Osher): u1 = u + dt R(u); u2 = 3/4 u + 1/4 (u1 + dt R(u1));
  // u_{n+1} = 1/3 u + 2/3 (u2 + dt R(u2))
  const double al[3] = {0.0, 0.75, 1.0 / 3.0};
  const double be[3] = {1.0, 0.25, 2.0 / 3.0};
  const double ep[3] = {dt, 0.25 * dt, 2.0 / 3.0 * dt};
  const void* cu = su;
  const void* cv = sv;
  for (int s = 0; s < 3; ++s) {
    a.us = cu;
    a.vs = cv;
    a.un = (s == 0) ? nullptr : su;
    a.vn = (s == 0) ? nullptr : sv;
    a.alpha = al[s];
    a.beta = be[s];
    a.eps = ep[s];
    a.delta = a.gamma = a.wacc = 0.0;
    a.oaccu = a.oaccv = nullptr;
    a.tcu = (s == 2) ? tcu : nullptr;
    a.tcv = (s == 2) ? tcv : nullptr;
    a.tc_bstride = tcbs;
    if (mac) {
      a.ou = h->st_u;
      a.ov = h->st_v;
      LDSV_TRY(ldsv_launch_stage(h, p, a, st));
      LDSV_TRY(ldsv_launch_project(h, h->st_u, h->st_v, s == 2 ? du : h->ws_u,
                                   s == 2 ? dv : h->ws_v, nullptr, st, active));
      cu = h->ws_u;
      cv = h->ws_v;
    } else {
      void* ou = (s == 2) ? du : (s == 0 ? h->ws_u : h->st_u);
      void* ov = (s == 2) ? dv : (s == 0 ? h->ws_v : h->st_v);
      a.ou = ou;
      a.ov = ov;
      LDSV_TRY(ldsv_launch_stage(h, p, a, st));
      cu = ou;
      cv = ov;
    }
  }
  return LDSV_OK;
}

}  // namespace

// internal: a step with optional coefficients (batch stride) and TC, used by
// the learned path
int ldsv_internal_step(ldsv_handle* h, const ldsv_params* p, const float* coef, size_t cbs,
                       const void* su, const void* sv, void* du, void* dv, const float* tcu,
                       const float* tcv, size_t tcbs, hipStream_t st) {
  return one_step(h, p, coef, cbs, su, sv, du, dv, tcu, tcv, tcbs, st);
}

// the plain step for the trajectories whose `active` entry is nonzero (MAC):
// the others' workgroups return at once and their outputs du, dv are left
// as they were
int ldsv_internal_step_masked(ldsv_handle* h, const ldsv_params* p, const void* su,
                              const void* sv, void* du, void* dv, const int* active,
                              hipStream_t st) {
  return one_step(h, p, nullptr, 0, su, sv, du, dv, nullptr, nullptr, 0, st, nullptr, nullptr, 0,
                  nullptr, nullptr, nullptr, active);
}

// the same with the raw coefficients stored in bf16 [B][8][Ny][Nx][8]
int ldsv_internal_step16(ldsv_handle* h, const ldsv_params* p, const uint16_t* coef16,
                         size_t cbs16, const void* su, const void* sv, void* du, void* dv,
                         const float* tcu, const float* tcv, size_t tcbs, hipStream_t st) {
  return one_step(h, p, nullptr, 0, su, sv, du, dv, tcu, tcv, tcbs, st, nullptr, coef16, cbs16);
}

// the same with per-cell learned derivative values beside the coefficients
// (float planes with coef, bf16 blocks of 8 channels with coef16; the same strides)
int ldsv_internal_step_d(ldsv_handle* h, const ldsv_params* p, const float* coef, size_t cbs,
                         const uint16_t* coef16, size_t cbs16, const DerivCoef* dc,
                         const void* su, const void* sv, void* du, void* dv, const float* tcu,
                         const float* tcv, size_t tcbs, hipStream_t st) {
  return one_step(h, p, coef16 ? nullptr : coef, coef16 ? 0 : cbs, su, sv, du, dv, tcu, tcv, tcbs,
                  st, nullptr, coef16, cbs16, nullptr, nullptr, dc);
}

// the same with the flux block's uniform kernels and fields, and an
// optional temporal correction (tcu, tcv, batch stride tcbs) added before
// the last projection
int ldsv_internal_step_fb(ldsv_handle* h, const ldsv_params* p, const FluxBlockArgs* fb,
                          const void* su, const void* sv, void* du, void* dv, hipStream_t st,
                          const float* tcu, const float* tcv, size_t tcbs) {
  return one_step(h, p, nullptr, 0, su, sv, du, dv, tcu, tcv, tcbs, st, nullptr, nullptr, 0, fb);
}

// a step of the velocity with a passive scalar
int ldsv_internal_step_scalar(ldsv_handle* h, const ldsv_params* p, double diff, const void* su,
                              const void* sv, const void* ss, void* du, void* dv, void* ds,
                              hipStream_t st) {
  if (!h->sc_ws) LDSV_TRY(ldsv_alloc(h, &h->sc_ws, 3 * h->nstate * h->esize, "scalar workspace"));
  ScalarStep sc{ss, ds, diff};
  return one_step(h, p, nullptr, 0, su, sv, du, dv, nullptr, nullptr, 0, st, nullptr, nullptr, 0,
                  nullptr, &sc);
}

// VJP of one RK4 step with a projection per sub-step (reverse sweep in
// adjoint.hip's header comment)
int ldsv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const float* coef, size_t cbs,
                  float* gcoef, size_t gcbs, const void* su, const void* sv, const void* gu_out,
                  const void* gv_out, void* gu_in, void* gv_in, hipStream_t st,
                  const FluxBlockArgs* fb, const DerivCoef* dc) {
  LDSV_REQUIRE(h->g.layout == LDSV_MAC && prm->rk == LDSV_RK4, LDSV_EDTYPE,
               "adjoint: RK4 on the MAC layout only");
  LDSV_TRY(ldsv_ensure_adjoint(h));
  const size_t sb = h->nstate * h->esize;
  char* K = (char*)h->stage_keep;
  char* A = (char*)h->adj_u;
  char* S = A + 2 * sb;
  char* W = A + 4 * sb;
  char* G = A + 6 * sb;
  const double dt = prm->dt;
  // forward recompute keeping u1, u2, u3 (the output goes to W, unused)
  LDSV_TRY(one_step(h, prm, coef, cbs, su, sv, W, W + sb, nullptr, nullptr, 0, st, K, nullptr, 0,
                    fb, nullptr, dc));
  // A = P g, S = A
  LDSV_TRY(ldsv_launch_project(h, gu_out, gv_out, A, A + sb, nullptr, st));
  LDSV_HIP(hipMemcpyAsync(S, A, 2 * sb, hipMemcpyDeviceToDevice, st));
  // stage 4 .. 2
  const double aA[3] = {dt / 6.0, dt / 3.0, dt / 3.0};
  const double aG[3] = {0.0, dt, 0.5 * dt};
  for (int k = 0; k < 3; ++k) {
    const int s = 2 - k;  // stage state u_{s+1} at keep plane s
    LDSV_TRY(ldsv_launch_adj_rhs(h, prm, coef, cbs, gcoef, gcbs, K + 2 * s * sb,
                                 K + (2 * s + 1) * sb, A, A + sb, k ? G : nullptr,
                                 k ? G + sb : nullptr, aA[k], aG[k], nullptr, nullptr, W, W + sb,
                                 st, fb, dc));
    LDSV_TRY(ldsv_launch_project(h, W, W + sb, G, G + sb, nullptr, st));
    LDSV_TRY(ldsv_launch_axpy2(h, S, S + sb, G, G + sb, 1.0, st));
  }
  // stage 1: dL/du0 = S + J(u0)^T (dt/6 A + dt/2 g1)
  return ldsv_launch_adj_rhs(h, prm, coef, cbs, gcoef, gcbs, su, sv, A, A + sb, G, G + sb,
                             dt / 6.0, 0.5 * dt, S, S + sb, gu_in, gv_in, st, fb, dc);
}

int ldsv_check_grid(const ldsv_grid* g, const char* who) {
  LDSV_REQUIRE(pow2_in_range(g->nx) && pow2_in_range(g->ny), LDSV_ESHAPE,
               "%s: nx=%d ny=%d must be powers of two in [8, 4096]", who, g->nx, g->ny);
  LDSV_REQUIRE(g->batch >= 1 && g->batch <= (1 << 20), LDSV_EINVAL, "%s: batch=%d", who,
               g->batch);
  LDSV_REQUIRE(g->dtype == LDSV_F32 || g->dtype == LDSV_F64, LDSV_EDTYPE, "%s: dtype=%d", who,
               g->dtype);
  LDSV_REQUIRE(g->layout == LDSV_COLLOCATED ||
                   (g->nx <= (g->dtype == LDSV_F64 ? 1024 : 2048) &&
                    g->ny <= (g->dtype == LDSV_F64 ? 1024 : 2048)),
               LDSV_ESHAPE, "%s: MAC grids need nx, ny <= 2048 (FP32) or 1024 (FP64)", who);
  LDSV_REQUIRE(g->layout == LDSV_MAC || g->layout == LDSV_COLLOCATED, LDSV_EINVAL,
               "%s: layout=%d", who, g->layout);
  LDSV_REQUIRE(g->lx > 0 && g->ly > 0 && std::isfinite(g->lx) && std::isfinite(g->ly), LDSV_EINVAL,
               "%s: box lengths must be positive", who);
  return LDSV_OK;
}

int ldsv_handle_shape(ldsv_handle* h, const ldsv_grid* g) {
  h->g = *g;
  LDSV_HIP(hipGetDevice(&h->device));
  h->log2nx = ilog2(g->nx);
  h->log2ny = ilog2(g->ny);
  h->ncell = (size_t)g->nx * g->ny;
  h->nstate = h->ncell * g->batch;
  h->npairs = (g->batch + 1) / 2;
  h->esize = (g->dtype == LDSV_F64) ? 8 : 4;
  return LDSV_OK;
}

int ldsv_check_fv_step(const ldsv_handle* h, const ldsv_params* prm, const float* coef,
                       const void* u_in, const void* v_in, const void* u_out,
                       const void* v_out, int nsteps, const char* who) {
  LDSV_TRY(ldsv_check_params(h, prm));
  LDSV_REQUIRE(u_in && v_in && u_out && v_out, LDSV_EINVAL, "%s: null array", who);
  LDSV_REQUIRE(nsteps >= 1, LDSV_EINVAL, "%s: nsteps=%d", who, nsteps);
  LDSV_REQUIRE(!coef || (h->g.layout == LDSV_MAC), LDSV_EDTYPE,
               "%s: learned coefficients need the MAC layout", who);
  LDSV_REQUIRE(h->g.layout == LDSV_MAC || prm->rk == LDSV_SSPRK3, LDSV_EDTYPE,
               "%s: the collocated layout integrates with SSPRK3", who);
  return LDSV_OK;
}

extern "C" {

int ldsv_version(void) { return 100; }

const char* ldsv_last_error(void) { return g_err; }

int ldsv_create(ldsv_handle** out, const ldsv_grid* g) {
  LDSV_REQUIRE(out && g, LDSV_EINVAL, "create: null argument");
  *out = nullptr;
  LDSV_TRY(ldsv_check_grid(g, "create"));
  ldsv_handle* h = new ldsv_handle();
  const int rc = ldsv_handle_shape(h, g);
  if (rc != LDSV_OK) {
    delete h;
    return rc;
  }
  const size_t sb = h->nstate * h->esize;
  char* blk = nullptr;
  hipError_t e = hipMalloc(&blk, 8 * sb);
  if (e != hipSuccess) {
    delete h;
    ldsv_set_error("create: cannot allocate %zu bytes of state workspace", 8 * sb);
    return LDSV_ENOMEM;
  }
  h->allocs.push_back(blk);
  h->ws_u = blk;
  h->ws_v = blk + sb;
  h->st_u = blk + 2 * sb;
  h->st_v = blk + 3 * sb;
  h->acc_u = blk + 4 * sb;
  h->acc_v = blk + 5 * sb;
  h->base_u = blk + 6 * sb;
  h->base_v = blk + 7 * sb;
  h->bytes = 8 * sb;
  const size_t zb = (size_t)h->npairs * h->ncell * 2 * h->esize;
  const size_t twb = ((size_t)g->nx + g->ny) * 2 * h->esize;
  h->red_len = (size_t)64 * 8 * (g->batch + 1);
  const size_t smallb = (size_t)16 * (g->batch + 1) * sizeof(double);
  char* blk2 = nullptr;
  e = hipMalloc(&blk2, zb + twb + h->red_len * sizeof(double) + smallb + 256);
  if (e != hipSuccess) {
    (void)hipFree(blk);
    delete h;
    ldsv_set_error("create: cannot allocate spectrum workspace");
    return LDSV_ENOMEM;
  }
  h->allocs.push_back(blk2);
  h->zspec = blk2;
  h->twx = blk2 + zb;
  h->twy = blk2 + zb + (size_t)g->nx * 2 * h->esize;
  h->red = (double*)(blk2 + zb + twb);
  h->small = h->red + h->red_len;
  h->flag_dev = (int*)((char*)h->small + smallb);
  h->bytes += zb + twb + h->red_len * sizeof(double) + smallb + 256;
  if (g->dtype == LDSV_F64) {
    auto tx = twiddles<double>(g->nx);
    auto ty = twiddles<double>(g->ny);
    LDSV_HIP(hipMemcpy(h->twx, tx.data(), tx.size() * sizeof(tx[0]), hipMemcpyHostToDevice));
    LDSV_HIP(hipMemcpy(h->twy, ty.data(), ty.size() * sizeof(ty[0]), hipMemcpyHostToDevice));
  } else {
    auto tx = twiddles<float>(g->nx);
    auto ty = twiddles<float>(g->ny);
    LDSV_HIP(hipMemcpy(h->twx, tx.data(), tx.size() * sizeof(tx[0]), hipMemcpyHostToDevice));
    LDSV_HIP(hipMemcpy(h->twy, ty.data(), ty.size() * sizeof(ty[0]), hipMemcpyHostToDevice));
  }
  if (g->layout == LDSV_MAC) {
    // Poisson factors: the eigenvalues of the compact D G pair,
    // lambda_h = (2/dx)^2 sin^2(pi kx/Nx) + (2/dy)^2 sin^2(pi ky/Ny), in FP64
    std::vector<double> pinv(h->ncell);
    const double dx = g->lx / g->nx, dy = g->ly / g->ny;
    const double pi = 3.14159265358979323846;
    const double nrm = 1.0 / ((double)g->nx * (double)g->ny);
    for (int ky = 0; ky < g->ny; ++ky) {
      const double sy = std::sin(pi * ky / g->ny);
      for (int kx = 0; kx < g->nx; ++kx) {
        const double sx = std::sin(pi * kx / g->nx);
        const double lam = 4.0 / (dx * dx) * sx * sx + 4.0 / (dy * dy) * sy * sy;
        pinv[(size_t)ky * g->nx + kx] = (kx == 0 && ky == 0) ? 0.0 : -nrm / lam;
      }
    }
    void* p = nullptr;
    LDSV_TRY(ldsv_alloc(h, &p, h->ncell * sizeof(double), "Poisson factors"));
    h->pinv = (double*)p;
    LDSV_HIP(hipMemcpy(h->pinv, pinv.data(), h->ncell * sizeof(double), hipMemcpyHostToDevice));
  }
  LDSV_HIP(hipHostMalloc((void**)&h->small_host, smallb, hipHostMallocDefault));
  *out = h;
  return LDSV_OK;
}

int ldsv_destroy(ldsv_handle* h) {
  if (!h) return LDSV_OK;
  (void)hipDeviceSynchronize();
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->small_host) (void)hipHostFree(h->small_host);
  for (int c = 0; c < kTimerClasses; ++c)
    for (auto e : h->timer.ev[c]) (void)hipEventDestroy(e);
  for (auto e : h->timer.pool) (void)hipEventDestroy(e);
  delete h;
  return LDSV_OK;
}

int ldsv_workspace_bytes(const ldsv_handle* h, size_t* bytes) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(bytes, LDSV_EINVAL, "workspace_bytes: null output");
  *bytes = h->bytes;
  return LDSV_OK;
}

int ldsv_init_state(ldsv_handle* h, int kind, uint64_t seed, const ldsv_ic_args* args, void* u,
                    void* v, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(u && v, LDSV_EINVAL, "init_state: null output");
  LDSV_REQUIRE(kind >= 0 && kind <= 3, LDSV_EINVAL, "init_state: kind=%d", kind);
  LDSV_REQUIRE((kind == LDSV_IC_FOURIER_MODES) == (h->g.layout == LDSV_COLLOCATED), LDSV_EDTYPE,
               "init_state: FOURIER_MODES is the collocated initial condition, the others are MAC");
  if (args) {
    LDSV_REQUIRE(args->delta > 0 && args->kpeak > 0 && args->noise_rms >= 0, LDSV_EINVAL,
                 "init_state: bad ic args");
  }
  return ldsv_launch_init(h, kind, seed, args, u, v, (hipStream_t)stream);
}

int ldsv_rhs(ldsv_handle* h, const ldsv_params* prm, const float* coef, const void* u,
             const void* v, void* ru, void* rv, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_params(h, prm));
  LDSV_REQUIRE(u && v && ru && rv, LDSV_EINVAL, "rhs: null array");
  LDSV_REQUIRE(!coef || (h->g.layout == LDSV_MAC), LDSV_EDTYPE,
               "rhs: learned coefficients need the MAC layout");
  StageArgs a;
  a.us = u;
  a.vs = v;
  a.ou = ru;
  a.ov = rv;
  a.eps = 1.0;
  a.coef = coef;
  a.coef_bstride = (size_t)LDSV_NCOEF * h->ncell;
  return ldsv_launch_stage(h, prm, a, (hipStream_t)stream);
}

int ldsv_fv_step(ldsv_handle* h, const ldsv_params* prm, const float* coef, const void* u_in,
                 const void* v_in, void* u_out, void* v_out, int nsteps, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_fv_step(h, prm, coef, u_in, v_in, u_out, v_out, nsteps, "fv_step"));
  const hipStream_t st = (hipStream_t)stream;
  const size_t cbs = (size_t)LDSV_NCOEF * h->ncell;
  for (int k = 0; k < nsteps; ++k) {
    const void* su = (k == 0) ? u_in : u_out;
    const void* sv = (k == 0) ? v_in : v_out;
    LDSV_TRY(one_step(h, prm, coef, cbs, su, sv, u_out, v_out, nullptr, nullptr, 0, st));
  }
  return LDSV_OK;
}

int ldsv_project(ldsv_handle* h, void* u, void* v, void* p_out, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(u && v, LDSV_EINVAL, "project: null array");
  LDSV_REQUIRE(h->g.layout == LDSV_MAC, LDSV_EDTYPE, "project: MAC layout only");
  return ldsv_launch_project(h, u, v, u, v, p_out, (hipStream_t)stream);
}

int ldsv_project_bwd(ldsv_handle* h, void* gu, void* gv, void* stream) {
  // the projection is an orthogonal projector (symmetric and idempotent)
  return ldsv_project(h, gu, gv, nullptr, stream);
}

int ldsv_diagnostics(ldsv_handle* h, const void* u, const void* v, double* diag, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(u && v && diag, LDSV_EINVAL, "diagnostics: null array");
  return ldsv_launch_diagnostics(h, u, v, diag, (hipStream_t)stream);
}

int ldsv_cfl_dt(ldsv_handle* h, const void* u, const void* v, double cfl, double* dt_host,
                void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(u && v && dt_host && cfl > 0, LDSV_EINVAL, "cfl_dt: bad argument");
  const hipStream_t st = (hipStream_t)stream;
  LDSV_TRY(ldsv_launch_maxspeed(h, u, v, h->small, st));
  LDSV_HIP(hipMemcpyAsync(h->small_host, h->small, h->g.batch * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  LDSV_HIP(hipStreamSynchronize(st));
  double m = 0;
  for (int b = 0; b < h->g.batch; ++b) m = std::fmax(m, h->small_host[b]);
  LDSV_REQUIRE(m > 0 && std::isfinite(m), LDSV_ENONFINITE, "cfl_dt: max speed %g", m);
  const double hmin = std::fmin(h->g.lx / h->g.nx, h->g.ly / h->g.ny);
  *dt_host = cfl * hmin / m;
  return LDSV_OK;
}

int ldsv_downsample(ldsv_handle* h, int r, const float* uf, const float* vf, float* uc,
                    float* vc, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(uf && vf && uc && vc && r >= 1, LDSV_EINVAL, "downsample: bad argument");
  LDSV_REQUIRE(h->g.dtype == LDSV_F32 && h->g.layout == LDSV_MAC, LDSV_EDTYPE,
               "downsample: F32 MAC grids");
  return ldsv_launch_downsample(h, r, uf, vf, uc, vc, (hipStream_t)stream);
}

int ldsv_vorticity(ldsv_handle* h, const void* u, const void* v, void* w, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(u && v && w, LDSV_EINVAL, "vorticity: null array");
  return ldsv_launch_vorticity(h, u, v, w, (hipStream_t)stream);
}

int ldsv_pcc(ldsv_handle* h, const void* a, const void* b, double* pcc, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(a && b && pcc, LDSV_EINVAL, "pcc: null array");
  return ldsv_launch_pcc(h, a, b, pcc, (hipStream_t)stream);
}

int ldsv_mse_grad(ldsv_handle* h, const float* u, const float* v, const float* lu,
                  const float* lv, double scale, float* gu, float* gv, double* loss,
                  void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(u && v && lu && lv, LDSV_EINVAL, "mse_grad: null array");
  LDSV_REQUIRE(h->g.dtype == LDSV_F32, LDSV_EDTYPE, "mse_grad: F32 grids");
  return ldsv_launch_mse_grad(h, u, v, lu, lv, scale, gu, gv, loss, (hipStream_t)stream, 0);
}

}  // extern "C"

// ---------------------------------------------------------------- timing
bool ldsv_timer_pair(ldsv_handle* h, int cls, hipEvent_t* e0, hipEvent_t* e1) {
  if (!h->timer.on) return false;
  hipEvent_t e[2];
  for (int k = 0; k < 2; ++k) {
    if (h->timer.pool.empty()) {
      if (hipEventCreate(&e[k]) != hipSuccess) {
        (void)hipGetLastError();
        if (k == 1) h->timer.pool.push_back(e[0]);
        return false;
      }
    } else {
      e[k] = h->timer.pool.back();
      h->timer.pool.pop_back();
    }
  }
  h->timer.ev[cls].push_back(e[0]);
  h->timer.ev[cls].push_back(e[1]);
  *e0 = e[0];
  *e1 = e[1];
  return true;
}

extern "C" int ldsv_timer_enable(ldsv_handle* h, int on) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_HIP(hipDeviceSynchronize());
  for (int c = 0; c < kTimerClasses; ++c) {
    for (auto e : h->timer.ev[c]) h->timer.pool.push_back(e);
    h->timer.ev[c].clear();
  }
  h->timer.on = on != 0;
  return LDSV_OK;
}

extern "C" int ldsv_timer_read(ldsv_handle* h, int cls, double* total_ms, int* count) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(cls >= 0 && cls < kTimerClasses && total_ms && count, LDSV_EINVAL,
               "timer_read: bad argument");
  LDSV_HIP(hipDeviceSynchronize());
  double t = 0;
  const auto& v = h->timer.ev[cls];
  for (size_t i = 0; i + 1 < v.size(); i += 2) {
    float ms = 0;
    LDSV_HIP(hipEventElapsedTime(&ms, v[i], v[i + 1]));
    t += ms;
  }
  *total_ms = t;
  *count = (int)(v.size() / 2);
  return LDSV_OK;
}
