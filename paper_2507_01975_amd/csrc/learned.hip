// The learned step and the rollout (Eq. 2):
//   u_k = FV(u_{k-1}; c(u_{k-1})) + TC(u_{k-1})   if k mod k_c == 0
//   u_k = FV(u_{k-1}; c(u_{k-1}))                  otherwise
// with the stencil coefficients c and the correction TC from one pass of the
// coefficient network on u_{k-1}.  The correction enters the last RK stage
// before its projection, u_k = P(u* + TC), which equals P(P(u*) + TC)
// because P is a linear projector.  The rollout guards every learned step:
// a trajectory whose new state is non-finite or exceeds the max-speed bound
// is recomputed from u_{k-1} with the plain FV step, all on the device.
#include "adjoint.h"
#include "cnn.h"
#include "reduce.h"
#include "stage.h"

int ldsv_launch_mse_grad(ldsv_handle* h, const float* u, const float* v, const float* lu,
                         const float* lv, double scale, float* gu, float* gv, double* loss,
                         hipStream_t st, int accumulate);
int ldsv_check_params(const ldsv_handle* h, const ldsv_params* p);
int ldsv_internal_step(ldsv_handle* h, const ldsv_params* p, const float* coef, size_t cbs,
                       const void* su, const void* sv, void* du, void* dv, const float* tcu,
                       const float* tcv, size_t tcbs, hipStream_t st);
int ldsv_internal_step16(ldsv_handle* h, const ldsv_params* p, const uint16_t* coef16,
                         size_t cbs16, const void* su, const void* sv, void* du, void* dv,
                         const float* tcu, const float* tcv, size_t tcbs, hipStream_t st);
int ldsv_internal_step_masked(ldsv_handle* h, const ldsv_params* p, const void* su,
                              const void* sv, void* du, void* dv, const int* active,
                              hipStream_t st);
int ldsv_launch_guard_redo(ldsv_handle* h, const ldsv_params* prm, const float* cu,
                           const float* cv, float* nu, float* nv, double thr, int redo,
                           int* counts, int* any, const double* smax, hipStream_t st);
int ldsv_internal_step_d(ldsv_handle* h, const ldsv_params* p, const float* coef, size_t cbs,
                         const uint16_t* coef16, size_t cbs16, const DerivCoef* dc,
                         const void* su, const void* sv, void* du, void* dv, const float* tcu,
                         const float* tcv, size_t tcbs, hipStream_t st);

namespace {

// zero fill (a kernel rather than a memset node, so that a captured graph
// of the training calls replays correctly)
__global__ void k_zero(float* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

int launch_zero(ldsv_handle* h, float* p, size_t n, hipStream_t st) {
  LDSV_TLAUNCH(h, 7, k_zero, grid1d(n), dim3(kBlock), 0, st, p, n);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

// The rollout guard of one learned step, one workgroup per trajectory: the
// largest |u| + |v| over the trajectory's cells (in FP64; a non-finite value
// counts as infinite) against the bound thr, or that maximum as the step's
// last projection reported it (smax, nullable).  Writes bad[b] (1: redo
// with the plain step), adds it to counts[b] (nullable) and raises *any.
constexpr int kGuardBlock = 256;
__global__ void __launch_bounds__(kGuardBlock) k_guard_detect(const float* __restrict__ u,
                                                              const float* __restrict__ v,
                                                              size_t n, double thr, int* bad,
                                                              int* counts, int* any,
                                                              const double* __restrict__ smax) {
  __shared__ double red[kGuardBlock / 64];
  const int b = blockIdx.x;
  const float* ub = u + (size_t)b * n;
  const float* vb = v + (size_t)b * n;
  double m = 0.0;
  if (smax) {  // written by the step's last projection
    m = smax[b];
  } else {
    for (size_t i = threadIdx.x; i < n; i += kGuardBlock) {
      const double s = (double)fabsf(ub[i]) + (double)fabsf(vb[i]);
      m = isfinite(s) ? fmax(m, s) : INFINITY;
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kGuardBlock / 64; ++w) m = fmax(m, red[w]);
    const int f = !(m < thr);
    bad[b] = f;
    if (f) {
      if (counts) counts[b] += 1;
      atomicOr(any, 1);
    }
  }
}

__global__ void k_zero_int(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// The network's 64 stencil-coefficient outputs are stored in bf16 (like its
// activations): in bf16 blocks of 8 channels when nothing asks for the float output (half
// the bytes the four stage kernels read), else as bf16-rounded values in the
// float output.  Both forms give the same step.  With a derivative-stencil
// network (dnet) its 64 raw derivative values take the same form beside them.
int ensure_deriv_buffers(ldsv_handle* h) {
  if (h->dnetout) return LDSV_OK;
  const size_t P = h->nstate;
  void* blk = nullptr;
  LDSV_TRY(ldsv_alloc(h, &blk,
                      2 * P * LDSV_NOUT * sizeof(float) + P * LDSV_NCOEF * sizeof(uint16_t) +
                          P * (LDSV_NOUT - LDSV_NCOEF) * sizeof(float),
                      "derivative-network workspace"));
  h->dnetout = (float*)blk;
  h->gdnet = h->dnetout + P * LDSV_NOUT;
  h->dcoef16 = (uint16_t*)(h->gdnet + P * LDSV_NOUT);
  h->dtcbuf = (float*)(h->dcoef16 + P * LDSV_NCOEF);
  return LDSV_OK;
}

int learned_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net, const float* u_in,
                 const float* v_in, float* u_out, float* v_out, int step_index, float* net_out,
                 hipStream_t st, const ldsv_net* dnet = nullptr, float* dnet_out = nullptr) {
  const size_t N = h->ncell;
  const bool tc = prm->k_c > 0 && (step_index % prm->k_c) == 0;
  const size_t ts = (size_t)(LDSV_NOUT - LDSV_NCOEF) * N;
  const size_t bs = (size_t)LDSV_NOUT * N;
  bool packed = false;
  if (dnet) {
    LDSV_TRY(ensure_deriv_buffers(h));
    float* dout = dnet_out ? dnet_out : h->dnetout;
    if (!net_out && !dnet_out) {
      bool dpacked = false;
      LDSV_TRY(ldsv_launch_cnn(h, dnet, u_in, v_in, dout, nullptr, st, h->dcoef16, h->dtcbuf,
                               &dpacked, true));
      LDSV_TRY(ldsv_launch_cnn(h, net, u_in, v_in, h->netout, nullptr, st, h->coef16, h->tcbuf,
                               &packed, true));
      LDSV_REQUIRE(packed == dpacked, LDSV_EINVAL, "learned step: network output forms differ");
      if (packed) {
        DerivCoef dc;
        dc.d16 = h->dcoef16;
        return ldsv_internal_step_d(h, prm, nullptr, 0, h->coef16, (size_t)LDSV_NCOEF * N, &dc,
                                    u_in, v_in, u_out, v_out, tc ? h->tcbuf : nullptr,
                                    tc ? h->tcbuf + N : nullptr, ts, st);
      }
    } else {
      LDSV_TRY(ldsv_launch_cnn(h, dnet, u_in, v_in, dout, nullptr, st, nullptr, nullptr, nullptr,
                               true));
    }
    float* out = net_out ? net_out : h->netout;
    if (net_out || dnet_out)
      LDSV_TRY(ldsv_launch_cnn(h, net, u_in, v_in, out, nullptr, st, nullptr, nullptr, nullptr, true));
    DerivCoef dc;
    dc.d = dout;
    return ldsv_internal_step_d(h, prm, out, bs, nullptr, 0, &dc, u_in, v_in, u_out, v_out,
                                tc ? out + (size_t)LDSV_NCOEF * N : nullptr,
                                tc ? out + (size_t)(LDSV_NCOEF + 1) * N : nullptr, bs, st);
  }
  if (!net_out) {
    LDSV_TRY(ldsv_launch_cnn(h, net, u_in, v_in, h->netout, nullptr, st, h->coef16, h->tcbuf,
                             &packed, true));
    if (packed)
      return ldsv_internal_step16(h, prm, h->coef16, (size_t)LDSV_NCOEF * N, u_in, v_in, u_out,
                                  v_out, tc ? h->tcbuf : nullptr, tc ? h->tcbuf + N : nullptr, ts,
                                  st);
  }
  float* out = net_out ? net_out : h->netout;
  if (net_out)
    LDSV_TRY(ldsv_launch_cnn(h, net, u_in, v_in, out, nullptr, st, nullptr, nullptr, nullptr, true));
  return ldsv_internal_step(h, prm, out, bs, u_in, v_in, u_out, v_out,
                            tc ? out + (size_t)LDSV_NCOEF * N : nullptr,
                            tc ? out + (size_t)(LDSV_NCOEF + 1) * N : nullptr, bs, st);
}

// the guarded rollout's second state buffer (the learned steps ping-pong
// between it and the handle's base state), per-trajectory flags and the
// any-flag
int ensure_rollout_buffers(ldsv_handle* h) {
  if (h->save_u) return LDSV_OK;
  const size_t sb = h->nstate * h->esize;
  // u, v of a step, the any-flag, per-trajectory flags and speeds
  return ldsv_alloc(h, &h->save_u,
                    2 * sb + 64 * sizeof(int) + (size_t)h->g.batch * (sizeof(int) + sizeof(double)) + 8,
                    "rollout guard buffers");
}

}  // namespace

namespace {

int rollout_impl(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net, const ldsv_net* dnet,
                 const void* u0, const void* v0, int nsteps, int save_every, int first_index,
                 void* traj_u, void* traj_v, int* fallback_flags, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && u0 && v0 && traj_u && traj_v, LDSV_EINVAL, "rollout: null argument");
  LDSV_REQUIRE(nsteps >= 1 && save_every >= 1 && save_every <= nsteps, LDSV_EINVAL,
               "rollout: nsteps=%d save_every=%d", nsteps, save_every);
  LDSV_REQUIRE(h->g.layout == LDSV_MAC || prm->rk == LDSV_SSPRK3, LDSV_EDTYPE,
               "rollout: the collocated layout integrates with SSPRK3");
  const hipStream_t st = (hipStream_t)stream;
  LDSV_REQUIRE(net || !dnet, LDSV_EINVAL, "rollout: a derivative network needs the coefficient network");
  if (net) {
    LDSV_TRY(ldsv_check_net(net));
    if (dnet) LDSV_TRY(ldsv_check_net(dnet));
    LDSV_TRY(ldsv_ensure_learned(h));
    LDSV_TRY(ensure_rollout_buffers(h));
  }
  const size_t sb = h->nstate * h->esize;
  void* cu = h->base_u;
  void* cv = h->base_v;
  LDSV_HIP(hipMemcpyAsync(cu, u0, sb, hipMemcpyDeviceToDevice, st));
  LDSV_HIP(hipMemcpyAsync(cv, v0, sb, hipMemcpyDeviceToDevice, st));
  // The guard stays on the device: after every learned step the
  // trajectories whose new state is non-finite or above the bound are
  // flagged and (with fallback) recomputed with the plain FV step from the
  // previous state, the others keeping their learned result.  No value is
  // read back during the loop; with fallback disabled the any-flag is read
  // once at the end of the call.
  const bool guard = net && (prm->fallback_enable || prm->guard_threshold > 0);
  void* nu = nullptr;
  void* nv = nullptr;
  int* any = nullptr;
  int* bad = nullptr;
  double* speeds = nullptr;
  if (guard) {
    nu = h->save_u;
    nv = (char*)h->save_u + sb;
    any = (int*)((char*)h->save_u + 2 * sb);
    bad = any + 64;
    const size_t so = (2 * sb + 64 * sizeof(int) + (size_t)h->g.batch * sizeof(int) + 7) & ~(size_t)7;
    speeds = (double*)((char*)h->save_u + so);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, any, 1);
    LDSV_LAUNCHED();
  }
  const double thr = prm->guard_threshold > 0 ? prm->guard_threshold : 1.0e300;
  for (int k = 0; k < nsteps; ++k) {
    const int idx = first_index + k;
    if (net) {
      if (guard) {
        // the step's last projection reports each trajectory's largest
        // |u| + |v| where it can (the one-trajectory kernels)
        h->speed_out = speeds;
        h->speed_written = false;
        const int rs = learned_step(h, prm, net, (const float*)cu, (const float*)cv, (float*)nu,
                                    (float*)nv, idx, nullptr, st, dnet);
        h->speed_out = nullptr;
        LDSV_TRY(rs);
        const double* smax = h->speed_written ? speeds : nullptr;
        h->speed_written = false;
        // small grids: detection and redo in one launch; otherwise the
        // detection kernel and the plain step masked to the flagged
        // trajectories
        const int rc = ldsv_launch_guard_redo(h, prm, (const float*)cu, (const float*)cv,
                                              (float*)nu, (float*)nv, thr, prm->fallback_enable,
                                              fallback_flags, any, smax, st);
        if (rc == LDSV_ESHAPE) {
          hipLaunchKernelGGL(k_guard_detect, dim3(h->g.batch), dim3(kGuardBlock), 0, st,
                             (const float*)nu, (const float*)nv, h->ncell, thr, bad,
                             fallback_flags, any, smax);
          LDSV_LAUNCHED();
          if (prm->fallback_enable)
            LDSV_TRY(ldsv_internal_step_masked(h, prm, cu, cv, nu, nv, bad, st));
        } else {
          LDSV_TRY(rc);
        }
        std::swap(cu, nu);
        std::swap(cv, nv);
      } else {
        LDSV_TRY(learned_step(h, prm, net, (const float*)cu, (const float*)cv, (float*)cu,
                              (float*)cv, idx, nullptr, st, dnet));
      }
    } else {
      LDSV_TRY(ldsv_internal_step(h, prm, nullptr, 0, cu, cv, cu, cv, nullptr, nullptr, 0, st));
    }
    if ((k + 1) % save_every == 0) {
      const size_t t = (size_t)((k + 1) / save_every - 1);
      LDSV_HIP(hipMemcpyAsync((char*)traj_u + t * sb, cu, sb, hipMemcpyDeviceToDevice, st));
      LDSV_HIP(hipMemcpyAsync((char*)traj_v + t * sb, cv, sb, hipMemcpyDeviceToDevice, st));
    }
  }
  if (guard && !prm->fallback_enable) {
    LDSV_HIP(hipMemcpyAsync(h->small_host, any, sizeof(int), hipMemcpyDeviceToHost, st));
    LDSV_HIP(hipStreamSynchronize(st));
    LDSV_REQUIRE(*(const int*)h->small_host == 0, LDSV_ENONFINITE,
                 "rollout: a learned step left a trajectory non-finite or above the bound "
                 "(fallback disabled)");
  }
  return LDSV_OK;
}

int learned_bwd_impl(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                     const ldsv_net* dnet, const float* u_in, const float* v_in, int step_index,
                     const float* gu_out, const float* gv_out, float* gu_in, float* gv_in,
                     const ldsv_net_grad* dW, const ldsv_net_grad* dWd, hipStream_t st) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_net(net));
  LDSV_REQUIRE(prm && u_in && v_in && gu_out && gv_out && gu_in && gv_in && dW, LDSV_EINVAL,
               "learned_fv_step_bwd: null argument");
  if (dnet) {
    LDSV_TRY(ldsv_check_net(dnet));
    LDSV_REQUIRE(dWd, LDSV_EINVAL, "learned_fv_step_bwd: the derivative network needs dWd");
  }
  LDSV_TRY(ldsv_ensure_learned(h));
  LDSV_TRY(ldsv_ensure_adjoint(h));
  if (dnet) LDSV_TRY(ensure_deriv_buffers(h));
  const size_t N = h->ncell;
  const size_t bs = (size_t)LDSV_NOUT * N;
  const size_t sb = h->nstate * h->esize;
  if (!h->gnet) {
    void* p = nullptr;
    LDSV_TRY(ldsv_alloc(h, &p, h->nstate * LDSV_NOUT * sizeof(float), "network-output gradient"));
    h->gnet = (float*)p;
  }
  // the step's coefficients (and derivative values) and correction
  DerivCoef dc;
  if (dnet) {
    LDSV_TRY(ldsv_launch_cnn(h, dnet, u_in, v_in, h->dnetout, nullptr, st, nullptr, nullptr,
                             nullptr, true));
    LDSV_TRY(launch_zero(h, h->gdnet, h->nstate * LDSV_NOUT, st));
    dc.d = h->dnetout;
    dc.gd = h->gdnet;
  }
  LDSV_TRY(ldsv_launch_cnn(h, net, u_in, v_in, h->netout, nullptr, st, nullptr, nullptr, nullptr,
                           true));
  LDSV_TRY(launch_zero(h, h->gnet, h->nstate * LDSV_NOUT, st));
  // FV path: d/du_in and d/d(raw coefficients)
  LDSV_TRY(ldsv_step_bwd(h, prm, h->netout, bs, h->gnet, bs, u_in, v_in, gu_out, gv_out, gu_in,
                         gv_in, st, nullptr, dnet ? &dc : nullptr));
  // temporal correction: u_k = P(w + TC) so dL/dTC = P g (kept by the sweep)
  const bool tc = prm->k_c > 0 && (step_index % prm->k_c) == 0;
  const char* A = (const char*)h->adj_u;
  if (tc) {
    LDSV_HIP(hipMemcpy2DAsync(h->gnet + (size_t)LDSV_NCOEF * N, bs * sizeof(float), A,
                              N * sizeof(float), N * sizeof(float), h->g.batch,
                              hipMemcpyDeviceToDevice, st));
    LDSV_HIP(hipMemcpy2DAsync(h->gnet + (size_t)(LDSV_NCOEF + 1) * N, bs * sizeof(float), A + sb,
                              N * sizeof(float), N * sizeof(float), h->g.batch,
                              hipMemcpyDeviceToDevice, st));
  }
  // network path: d/d(weights) and d/du_in through the network input
  char* W = (char*)h->adj_u + 4 * sb;
  LDSV_TRY(ldsv_launch_cnn_backward(h, net, u_in, v_in, h->gnet, (float*)W, (float*)(W + sb), dW,
                                    st));
  LDSV_TRY(ldsv_launch_axpy2(h, gu_in, gv_in, W, W + sb, 1.0, st));
  if (dnet) {
    // the derivative network (its two last outputs carry no gradient)
    LDSV_TRY(ldsv_launch_cnn_backward(h, dnet, u_in, v_in, h->gdnet, (float*)W, (float*)(W + sb),
                                      dWd, st));
    LDSV_TRY(ldsv_launch_axpy2(h, gu_in, gv_in, W, W + sb, 1.0, st));
  }
  return LDSV_OK;
}

int rollout_bwd_impl(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                     const ldsv_net* dnet, const float* u0, const float* v0, int nsteps,
                     int checkpoint_every, int first_index, const float* labels_u,
                     const float* labels_v, double loss_scale, const float* g_traj_u,
                     const float* g_traj_v, float* gu0, float* gv0, const ldsv_net_grad* dW,
                     const ldsv_net_grad* dWd, double* loss_dev, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_net(net));
  LDSV_REQUIRE(prm && u0 && v0 && dW && nsteps >= 1 && checkpoint_every >= 1, LDSV_EINVAL,
               "rollout_bwd: bad argument");
  LDSV_REQUIRE((labels_u != nullptr) == (labels_v != nullptr) &&
                   (g_traj_u != nullptr) == (g_traj_v != nullptr) && (labels_u || g_traj_u),
               LDSV_EINVAL, "rollout_bwd: give labels and/or trajectory cotangents, u and v together");
  LDSV_TRY(ldsv_ensure_learned(h));
  LDSV_TRY(ldsv_ensure_adjoint(h));
  const hipStream_t st = (hipStream_t)stream;
  const int ce = checkpoint_every < nsteps ? checkpoint_every : nsteps;
  const int nseg = (nsteps + ce - 1) / ce;
  const size_t sb = h->nstate * h->esize;
  const size_t need = (size_t)(nseg + 1 + ce + 2) * 2 * sb;
  if (h->roll_bytes < need) {
    void* p = nullptr;
    LDSV_TRY(ldsv_alloc(h, &p, need, "rollout backward checkpoints"));
    h->roll_blk = p;
    h->roll_bytes = need;
  }
  char* ck = (char*)h->roll_blk;                        // nseg + 1 checkpoints
  char* seg = ck + (size_t)(nseg + 1) * 2 * sb;         // ce segment states
  char* ga = seg + (size_t)ce * 2 * sb;                 // two cotangent buffers
  char* gb = ga + 2 * sb;
  auto U = [&](char* base, int i) { return base + (size_t)i * 2 * sb; };
  // forward, keeping the state at the start of every segment and the end
  LDSV_HIP(hipMemcpyAsync(U(seg, 0), u0, sb, hipMemcpyDeviceToDevice, st));
  LDSV_HIP(hipMemcpyAsync(U(seg, 0) + sb, v0, sb, hipMemcpyDeviceToDevice, st));
  for (int k = 0; k < nsteps; ++k) {
    if (k % ce == 0) LDSV_HIP(hipMemcpyAsync(U(ck, k / ce), U(seg, 0), 2 * sb, hipMemcpyDeviceToDevice, st));
    LDSV_TRY(learned_step(h, prm, net, (const float*)U(seg, 0), (const float*)(U(seg, 0) + sb),
                          (float*)U(seg, 0), (float*)(U(seg, 0) + sb), first_index + k, nullptr, st, dnet));
  }
  LDSV_HIP(hipMemcpyAsync(U(ck, nseg), U(seg, 0), 2 * sb, hipMemcpyDeviceToDevice, st));
  LDSV_TRY(launch_zero(h, (float*)ga, 2 * h->nstate, st));
  char* g = ga;
  char* gn = gb;
  for (int s = nseg - 1; s >= 0; --s) {
    const int k0 = s * ce, k1 = (k0 + ce < nsteps) ? k0 + ce : nsteps;
    LDSV_HIP(hipMemcpyAsync(U(seg, 0), U(ck, s), 2 * sb, hipMemcpyDeviceToDevice, st));
    for (int k = k0; k < k1 - 1; ++k)
      LDSV_TRY(learned_step(h, prm, net, (const float*)U(seg, k - k0), (const float*)(U(seg, k - k0) + sb),
                            (float*)U(seg, k - k0 + 1), (float*)(U(seg, k - k0 + 1) + sb),
                            first_index + k, nullptr, st, dnet));
    for (int k = k1 - 1; k >= k0; --k) {
      // cotangent of u_{k+1}: loss term and caller-supplied cotangent
      char* nxt = (k + 1 < k1) ? U(seg, k + 1 - k0) : U(ck, s + 1);
      if (labels_u)
        LDSV_TRY(ldsv_launch_mse_grad(h, (const float*)nxt, (const float*)(nxt + sb),
                                      labels_u + (size_t)k * h->nstate, labels_v + (size_t)k * h->nstate,
                                      loss_scale, (float*)g, (float*)(g + sb), loss_dev, st, 1));
      if (g_traj_u) {
        LDSV_TRY(ldsv_launch_axpy2(h, g, g + sb, g_traj_u + (size_t)k * h->nstate,
                                   g_traj_v + (size_t)k * h->nstate, 1.0, st));
      }
      LDSV_TRY(learned_bwd_impl(h, prm, net, dnet, (const float*)U(seg, k - k0),
                                (const float*)(U(seg, k - k0) + sb), first_index + k,
                                (const float*)g, (const float*)(g + sb), (float*)gn,
                                (float*)(gn + sb), dW, dWd, st));
      char* t = g;
      g = gn;
      gn = t;
    }
  }
  if (gu0) LDSV_HIP(hipMemcpyAsync(gu0, g, sb, hipMemcpyDeviceToDevice, st));
  if (gv0) LDSV_HIP(hipMemcpyAsync(gv0, g + sb, sb, hipMemcpyDeviceToDevice, st));
  return LDSV_OK;
}

}  // namespace

extern "C" {

int ldsv_cnn_forward(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                     float* out, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_net(net));
  LDSV_REQUIRE(u && v && out, LDSV_EINVAL, "cnn_forward: null array");
  LDSV_TRY(ldsv_ensure_learned(h));
  return ldsv_launch_cnn(h, net, u, v, out, nullptr, (hipStream_t)stream);
}

int ldsv_cnn_activation(ldsv_handle* h, int layer, uint16_t* dst, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(dst && layer >= 0 && layer < 5, LDSV_EINVAL, "cnn_activation: bad argument");
  LDSV_REQUIRE(h->netout, LDSV_EINVAL, "cnn_activation: no network evaluation yet");
  LDSV_HIP(hipMemcpyAsync(dst, h->act[layer], h->nstate * 64 * sizeof(uint16_t),
                          hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return LDSV_OK;
}

int ldsv_learned_fv_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                         const float* u_in, const float* v_in, float* u_out, float* v_out,
                         int step_index, float* net_out, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_net(net));
  LDSV_REQUIRE(prm && u_in && v_in && u_out && v_out, LDSV_EINVAL, "learned_fv_step: null argument");
  LDSV_REQUIRE(prm->rk == LDSV_RK4 || prm->rk == LDSV_SSPRK3, LDSV_EINVAL, "learned_fv_step: bad rk");
  LDSV_TRY(ldsv_ensure_learned(h));
  return learned_step(h, prm, net, u_in, v_in, u_out, v_out, step_index, net_out,
                      (hipStream_t)stream);
}

int ldsv_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const float* coef, const void* u_in,
                     const void* v_in, const void* gu_out, const void* gv_out, void* gu_in,
                     void* gv_in, float* gcoef, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && u_in && v_in && gu_out && gv_out && gu_in && gv_in, LDSV_EINVAL,
               "fv_step_bwd: null argument");
  const size_t cbs = (size_t)LDSV_NCOEF * h->ncell;
  return ldsv_step_bwd(h, prm, coef, cbs, coef ? gcoef : nullptr, cbs, u_in, v_in, gu_out, gv_out,
                       gu_in, gv_in, (hipStream_t)stream);
}
int ldsv_cnn_backward(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                      const float* gout, float* gu, float* gv, const ldsv_net_grad* dW,
                      void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_net(net));
  LDSV_REQUIRE(u && v && gout && dW, LDSV_EINVAL, "cnn_backward: null argument");
  for (int l = 0; l < LDSV_NLAYERS; ++l)
    LDSV_REQUIRE(dW->w[l] && dW->b[l], LDSV_EINVAL, "cnn_backward: null gradient of layer %d", l);
  LDSV_REQUIRE((gu == nullptr) == (gv == nullptr), LDSV_EINVAL, "cnn_backward: gu and gv together");
  LDSV_TRY(ldsv_ensure_learned(h));
  return ldsv_launch_cnn_backward(h, net, u, v, gout, gu, gv, dW, (hipStream_t)stream);
}

int ldsv_rollout(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net, const void* u0,
                 const void* v0, int nsteps, int save_every, int first_index, void* traj_u,
                 void* traj_v, int* fallback_flags, void* stream) {
  return rollout_impl(h, prm, net, nullptr, u0, v0, nsteps, save_every, first_index, traj_u,
                      traj_v, fallback_flags, stream);
}

int ldsv_learned_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                             const float* u_in, const float* v_in, int step_index,
                             const float* gu_out, const float* gv_out, float* gu_in, float* gv_in,
                             const ldsv_net_grad* dW, void* stream) {
  return learned_bwd_impl(h, prm, net, nullptr, u_in, v_in, step_index, gu_out, gv_out, gu_in,
                          gv_in, dW, nullptr, (hipStream_t)stream);
}

int ldsv_rollout_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net, const float* u0,
                     const float* v0, int nsteps, int checkpoint_every, int first_index,
                     const float* labels_u, const float* labels_v, double loss_scale,
                     const float* g_traj_u, const float* g_traj_v, float* gu0, float* gv0,
                     const ldsv_net_grad* dW, double* loss_dev, void* stream) {
  return rollout_bwd_impl(h, prm, net, nullptr, u0, v0, nsteps, checkpoint_every, first_index,
                          labels_u, labels_v, loss_scale, g_traj_u, g_traj_v, gu0, gv0, dW,
                          nullptr, loss_dev, stream);
}

/* ---- learned derivative stencils (per cell) ---- */

int ldsv_fv_step_d(ldsv_handle* h, const ldsv_params* prm, const float* coef, const float* dcoef,
                   const void* u_in, const void* v_in, void* u_out, void* v_out, int nsteps,
                   void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && coef && dcoef && u_in && v_in && u_out && v_out, LDSV_EINVAL,
               "fv_step_d: null argument");
  LDSV_TRY(ldsv_check_params(h, prm));
  LDSV_REQUIRE(nsteps >= 1, LDSV_EINVAL, "fv_step_d: nsteps=%d", nsteps);
  LDSV_REQUIRE(h->g.layout == LDSV_MAC && h->g.dtype == LDSV_F32, LDSV_EDTYPE,
               "fv_step_d: learned derivative stencils need an F32 MAC grid");
  const hipStream_t st = (hipStream_t)stream;
  const size_t cbs = (size_t)LDSV_NCOEF * h->ncell;
  DerivCoef dc;
  dc.d = dcoef;
  for (int k = 0; k < nsteps; ++k)
    LDSV_TRY(ldsv_internal_step_d(h, prm, coef, cbs, nullptr, 0, &dc, k ? u_out : u_in,
                                  k ? v_out : v_in, u_out, v_out, nullptr, nullptr, 0, st));
  return LDSV_OK;
}

int ldsv_fv_step_d_bwd(ldsv_handle* h, const ldsv_params* prm, const float* coef,
                       const float* dcoef, const void* u_in, const void* v_in, const void* gu_out,
                       const void* gv_out, void* gu_in, void* gv_in, float* gcoef, float* gdcoef,
                       void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && coef && dcoef && u_in && v_in && gu_out && gv_out && gu_in && gv_in,
               LDSV_EINVAL, "fv_step_d_bwd: null argument");
  LDSV_TRY(ldsv_check_params(h, prm));
  LDSV_REQUIRE(h->g.dtype == LDSV_F32, LDSV_EDTYPE, "fv_step_d_bwd: F32 grids only");
  const size_t cbs = (size_t)LDSV_NCOEF * h->ncell;
  DerivCoef dc;
  dc.d = dcoef;
  dc.gd = gdcoef;
  return ldsv_step_bwd(h, prm, coef, cbs, gcoef, cbs, u_in, v_in, gu_out, gv_out, gu_in, gv_in,
                       (hipStream_t)stream, nullptr, &dc);
}

int ldsv_learned_d_fv_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                           const ldsv_net* dnet, const float* u_in, const float* v_in,
                           float* u_out, float* v_out, int step_index, float* net_out,
                           float* dnet_out, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_TRY(ldsv_check_net(net));
  LDSV_TRY(ldsv_check_net(dnet));
  LDSV_REQUIRE(prm && u_in && v_in && u_out && v_out, LDSV_EINVAL,
               "learned_d_fv_step: null argument");
  LDSV_TRY(ldsv_check_params(h, prm));
  LDSV_TRY(ldsv_ensure_learned(h));
  return learned_step(h, prm, net, u_in, v_in, u_out, v_out, step_index, net_out,
                      (hipStream_t)stream, dnet, dnet_out);
}

int ldsv_learned_d_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                               const ldsv_net* dnet, const float* u_in, const float* v_in,
                               int step_index, const float* gu_out, const float* gv_out,
                               float* gu_in, float* gv_in, const ldsv_net_grad* dW,
                               const ldsv_net_grad* dWd, void* stream) {
  LDSV_REQUIRE(dnet, LDSV_EINVAL, "learned_d_fv_step_bwd: null derivative network");
  return learned_bwd_impl(h, prm, net, dnet, u_in, v_in, step_index, gu_out, gv_out, gu_in,
                          gv_in, dW, dWd, (hipStream_t)stream);
}

int ldsv_rollout_d(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                   const ldsv_net* dnet, const void* u0, const void* v0, int nsteps,
                   int save_every, int first_index, void* traj_u, void* traj_v,
                   int* fallback_flags, void* stream) {
  LDSV_REQUIRE(net && dnet, LDSV_EINVAL, "rollout_d: null network");
  return rollout_impl(h, prm, net, dnet, u0, v0, nsteps, save_every, first_index, traj_u, traj_v,
                      fallback_flags, stream);
}

int ldsv_rollout_d_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_net* net,
                       const ldsv_net* dnet, const float* u0, const float* v0, int nsteps,
                       int checkpoint_every, int first_index, const float* labels_u,
                       const float* labels_v, double loss_scale, const float* g_traj_u,
                       const float* g_traj_v, float* gu0, float* gv0, const ldsv_net_grad* dW,
                       const ldsv_net_grad* dWd, double* loss_dev, void* stream) {
  LDSV_REQUIRE(dnet && dWd, LDSV_EINVAL, "rollout_d_bwd: null derivative network or gradient");
  LDSV_TRY(ldsv_check_net(dnet));
  return rollout_bwd_impl(h, prm, net, dnet, u0, v0, nsteps, checkpoint_every, first_index,
                          labels_u, labels_v, loss_scale, g_traj_u, g_traj_v, gu0, gv0, dW, dWd,
                          loss_dev, stream);
}

}  // extern "C"
