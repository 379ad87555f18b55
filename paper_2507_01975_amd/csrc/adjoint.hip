// Adjoint (vector-Jacobian product) of the MAC finite-volume residual and of
// the RK4 step with a projection after every sub-step (the differentiable
// solver backbone of the method; Sec. 3.2 RK4 + projection, Sec. 3.3-3.4
// flux stencils).
//
// Residual adjoint.  With cotangents (lu, lv) of R = (R_u, R_v), the face
// cotangents are differences of the cotangents of the two control volumes
// the face separates, e.g. for the east face of the u volume owned by cell o
// Fb = (lu[o + x] - lu[o]) / dx.  Each face flux F = abar * atil - nu * D
// then sends
//   Fb * atil / 2   to the two velocities averaged into the advecting abar,
//   Fb * abar * c_s to every point s of the interpolation stencil atil,
//   -nu * Fb * w_m / (24 h) to the four points of the derivative D,
// and the coefficient gradient dc_s = Fb * abar * q_s, projected through the
// sum-to-one constraint (dr_t = dc_t - mean(dc)).  Drag adds -d * l
// pointwise.  Two kernels, both gather-only (no atomics, deterministic):
//   k_adj_faces   one thread per owner cell: the 12 face scalars (P: abar
//                 part, Q: stencil multiplier, V: viscous multiplier for the
//                 4 faces) and the per-kind coefficient means; accumulates the
//                 coefficient gradient of its own cell;
//   k_adj_gather  one thread per output cell: sums what every face whose
//                 stencil touches the cell sends to it.
//
// Flux block (Sec. 3.4): the interpolation stencil is c_P + w_K over the
// 5x4 window plus a field fi_K, the face derivative adds (1/h) sum w^d_K q
// plus a field fd_K.  The faces then also send Fb * abar * w_K,s to the
// points of the uniform kernel and -nu * Fb * w^d_K,s / h to the points of
// the derivative kernel; the field gradients are dfi_K = Fb * abar and
// dfd_K = -nu * Fb at the owner, and the uniform-kernel gradients are sums
// over all faces, dw_K,s = sum Fb * abar * q_s and dw^d_K,s =
// sum -nu * Fb * q_s / h, reduced per tile (k_adj_fb_wgrad) and then in a
// fixed order over the tiles (k_fb_wreduce): deterministic.
//
// Learned derivative stencils (per cell): the face derivative is
// (1/h) sum_s w_s q_s with w = w_P + r - mean(r) - x (x.r)/16 - b (b.r)/24.
// The face then sends -nu * Fb * w_s / h to every point s, and the raw
// gradient is the same projection of g_s = -nu * Fb * q_s / h:
// dr = g - mean(g) - x (x.g)/16 - b (b.g)/24.  The three moments of r per
// kind and owner go through the scratch planes to the gather.
//
// RK4 reverse sweep, with P the (symmetric) projection and u1..u3 the
// recomputed projected stage states:
//   A = P g;  S = A
//   l4 = dt/6 A           -> w3 = J(u3)^T l4, g3 = P w3, S += g3
//   l3 = dt/3 A + dt g3   -> w2 = J(u2)^T l3, g2 = P w2, S += g2
//   l2 = dt/3 A + dt/2 g2 -> w1 = J(u1)^T l2, g1 = P w1, S += g1
//   l1 = dt/6 A + dt/2 g1 -> dL/du0 = S + J(u0)^T l1
#include "adjoint.h"
#include "stage.h"

namespace {

__constant__ int kAOffA[16] = {-1, 0, 1, 2, -1, 0, 1, 2, -1, 0, 1, 2, 0, 1, 0, 1};
__constant__ int kBOffA[16] = {-1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -2, -2, 2, 2};

struct AdjPhys {
  double nu, drag, dx, dy;
  int mask;
};

template <typename T>
struct Field {
  const T* p;
  int nx, ny;
  __device__ __forceinline__ T operator()(int i, int j) const {
    return p[(size_t)(j & (ny - 1)) * nx + (i & (nx - 1))];
  }
};

// scratch layout (per trajectory plane, 28 planes): P0..P3, Q0..Q3, V0..V3,
// M0..M3, and for learned derivatives the moments mean(r), (x.r)/16 and
// (b.r)/24 of each kind (planes 16..19, 20..23, 24..27)
constexpr int kAdjPlanes = 28;

// fourth-order derivative weight of footprint point s (units of 1/h)
__device__ __forceinline__ constexpr double deriv4_w(int s) {
  return s == 4 ? 1.0 / 24.0 : s == 5 ? -27.0 / 24.0 : s == 6 ? 27.0 / 24.0 : s == 7 ? -1.0 / 24.0 : 0.0;
}

// the 5x4 window of the uniform kernels (points 0..15 as in kAOffA/kBOffA,
// then the four corners)
__device__ __forceinline__ constexpr int a_off20(int s) {
  return s < 12 ? s % 4 - 1 : (s < 16 ? (s & 1) : (s & 1 ? 2 : -1));
}
__device__ __forceinline__ constexpr int b_off20(int s) {
  return s < 12 ? s / 4 - 1 : (s < 14 ? -2 : (s < 16 ? 2 : (s < 18 ? -2 : 2)));
}

struct AdjFB {
  const float* w;   // [2][4][20]
  const float* f;   // [B][8][Ny][Nx], nullable
  size_t fbs;
  float* gf;        // nullable
  size_t gfbs;
};

// MODE: 0 physics stencil, 1 per-cell coefficients, 2 flux block, 3 per-cell
// coefficients and per-cell derivative values

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_adj_faces(const T* __restrict__ us, const T* __restrict__ vs,
                                                      const T* __restrict__ Au, const T* __restrict__ Av,
                                                      const T* __restrict__ Gu, const T* __restrict__ Gv,
                                                      double aA, double aG, const float* __restrict__ coef,
                                                      size_t cbs, float* __restrict__ gcoef, size_t gcbs,
                                                      const float* __restrict__ dcoef,
                                                      float* __restrict__ gdcoef, AdjFB fb,
                                                      T* __restrict__ scr, AdjPhys ph, int nx, int ny) {
  constexpr bool LEARNED = MODE == 1 || MODE == 3;
  const size_t n = (size_t)nx * ny;
  const int b = blockIdx.y;
  const size_t off = (size_t)b * n;
  const Field<T> U{us + off, nx, ny}, V{vs + off, nx, ny};
  const Field<T> LA_u{Au + off, nx, ny}, LA_v{Av + off, nx, ny};
  const T* gu = Gu ? Gu + off : nullptr;
  const T* gv = Gv ? Gv + off : nullptr;
  T* S = scr + (size_t)b * kAdjPlanes * n;
  const T cA = (T)aA, cG = (T)aG;
  const T idx = (T)(1.0 / ph.dx), idy = (T)(1.0 / ph.dy);
  const T nu = (T)ph.nu;
  const bool adv = ph.mask & LDSV_ADVECTION, visc = ph.mask & LDSV_VISCOSITY;
  const int lnx = __builtin_ctz(nx);  // nx is a power of two
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)c & (nx - 1), j = (int)c >> lnx;
    auto lam_u = [&](int a, int bb) {
      const size_t q = (size_t)((j + bb) & (ny - 1)) * nx + ((i + a) & (nx - 1));
      T l = cA * LA_u.p[q];
      if (gu) l += cG * gu[q];
      return l;
    };
    auto lam_v = [&](int a, int bb) {
      const size_t q = (size_t)((j + bb) & (ny - 1)) * nx + ((i + a) & (nx - 1));
      T l = cA * LA_v.p[q];
      if (gv) l += cG * gv[q];
      return l;
    };
    const T l0u = lam_u(0, 0), l0v = lam_v(0, 0);
    const T fxb = (lam_u(1, 0) - l0u) * idx;
    const T fyb = (lam_u(0, 1) - l0u) * idy;
    const T exb = (lam_v(1, 0) - l0v) * idx;
    const T eyb = (lam_v(0, 1) - l0v) * idy;
    T P[4] = {0, 0, 0, 0}, Q[4] = {0, 0, 0, 0}, Vm[4] = {0, 0, 0, 0}, M[4] = {0, 0, 0, 0};
    if (adv) {
      const T ubar_c = (T)0.5 * (U(i, j) + U(i + 1, j));
      const T vbar_n = (T)0.5 * (V(i - 1, j + 1) + V(i, j + 1));
      const T ubar_e = (T)0.5 * (U(i + 1, j - 1) + U(i + 1, j));
      const T vbar_c = (T)0.5 * (V(i, j) + V(i, j + 1));
      T face[4];
      if (LEARNED) {
        const float* cb = coef + (size_t)b * cbs;
        float* gc = gcoef ? gcoef + (size_t)b * gcbs : nullptr;
        const T qmul[4] = {fxb * ubar_c, fyb * vbar_n, exb * ubar_e, eyb * vbar_c};
#pragma unroll
        for (int K = 0; K < 4; ++K) {
          const Field<T>& F = (K < 2) ? U : V;
          const bool along_x = (K == 0 || K == 2);
          T r[16], q[16];
          T mr = 0, mq = 0;
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            r[s] = (T)cb[(size_t)(16 * K + s) * n + c];
            q[s] = along_x ? F(i + kAOffA[s], j + kBOffA[s]) : F(i + kBOffA[s], j + kAOffA[s]);
            mr += r[s];
            mq += q[s];
          }
          mr *= (T)(1.0 / 16.0);
          mq *= (T)(1.0 / 16.0);
          T val = 0;
#pragma unroll
          for (int s = 0; s < 16; ++s) val += (r[s] - mr) * q[s];
          val += (T)0.5 * (q[5] + q[6]);
          face[K] = val;
          M[K] = mr;
          if (gc) {
#pragma unroll
            for (int s = 0; s < 16; ++s)
              gc[(size_t)(16 * K + s) * n + c] += (float)(qmul[K] * (q[s] - mq));
          }
        }
      } else {
        face[0] = (T)0.5 * (U(i, j) + U(i + 1, j));
        face[1] = (T)0.5 * (U(i, j) + U(i, j + 1));
        face[2] = (T)0.5 * (V(i, j) + V(i + 1, j));
        face[3] = (T)0.5 * (V(i, j) + V(i, j + 1));
        if constexpr (MODE == 2) {
          const float* fo = fb.f ? fb.f + (size_t)b * fb.fbs : nullptr;
#pragma unroll
          for (int K = 0; K < 4; ++K) {
            const Field<T>& F = (K < 2) ? U : V;
            const bool along_x = (K == 0 || K == 2);
            T acc = 0;
#pragma unroll
            for (int s = 0; s < 20; ++s) {
              const T q = along_x ? F(i + a_off20(s), j + b_off20(s)) : F(i + b_off20(s), j + a_off20(s));
              acc += (T)fb.w[20 * K + s] * q;
            }
            face[K] += acc;
            if (fo) face[K] += (T)fo[(size_t)K * n + c];
          }
        }
      }
      P[0] = (T)0.5 * fxb * face[0];
      P[1] = (T)0.5 * fyb * face[1];
      P[2] = (T)0.5 * exb * face[2];
      P[3] = (T)0.5 * eyb * face[3];
      Q[0] = fxb * ubar_c;
      Q[1] = fyb * vbar_n;
      Q[2] = exb * ubar_e;
      Q[3] = eyb * vbar_c;
    }
    if (visc) {
      Vm[0] = -nu * fxb * (T)(1.0 / 24.0) * idx;
      Vm[1] = -nu * fyb * (T)(1.0 / 24.0) * idy;
      Vm[2] = -nu * exb * (T)(1.0 / 24.0) * idx;
      Vm[3] = -nu * eyb * (T)(1.0 / 24.0) * idy;
    }
    if constexpr (MODE == 3) {
      const float* db = dcoef + (size_t)b * cbs;
      float* gd = gdcoef ? gdcoef + (size_t)b * gcbs : nullptr;
#pragma unroll
      for (int K = 0; K < 4; ++K) {
        const Field<T>& F = (K < 2) ? U : V;
        const bool along_x = (K == 0 || K == 2);
        T r[16], q[16];
        T sr = 0, sxr = 0, sbr = 0, sq = 0, sxq = 0, sbq = 0;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const int a = a_off20(s), bb = b_off20(s);
          const T x = (T)a - (T)0.5;
          r[s] = (T)db[(size_t)(16 * K + s) * n + c];
          q[s] = along_x ? F(i + a, j + bb) : F(i + bb, j + a);
          sr += r[s];
          sxr += x * r[s];
          sbr += (T)bb * r[s];
          sq += q[s];
          sxq += x * q[s];
          sbq += (T)bb * q[s];
        }
        S[(size_t)(16 + K) * n + c] = sr * (T)(1.0 / 16.0);
        S[(size_t)(20 + K) * n + c] = sxr * (T)(1.0 / 16.0);
        S[(size_t)(24 + K) * n + c] = sbr * (T)(1.0 / 24.0);
        if (gd && visc) {
          const T g24 = (T)24 * Vm[K];  // -nu Fb / h
          sq *= (T)(1.0 / 16.0);
          sxq *= (T)(1.0 / 16.0);
          sbq *= (T)(1.0 / 24.0);
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            const T x = (T)a_off20(s) - (T)0.5;
            gd[(size_t)(16 * K + s) * n + c] += (float)(g24 * (q[s] - sq - x * sxq - (T)b_off20(s) * sbq));
          }
        }
      }
    }
    if constexpr (MODE == 2) {
      if (fb.gf) {
        float* g = fb.gf + (size_t)b * fb.gfbs;
        const T fbk[4] = {fxb, fyb, exb, eyb};
#pragma unroll
        for (int K = 0; K < 4; ++K) {
          if (adv) g[(size_t)K * n + c] += (float)Q[K];
          if (visc) g[(size_t)(4 + K) * n + c] += (float)(-nu * fbk[K]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      S[(size_t)k * n + c] = P[k];
      S[(size_t)(4 + k) * n + c] = Q[k];
      S[(size_t)(8 + k) * n + c] = Vm[k];
      S[(size_t)(12 + k) * n + c] = M[k];
    }
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_adj_gather(const T* __restrict__ scr,
                                                       const float* __restrict__ coef, size_t cbs,
                                                       const float* __restrict__ dcoef,
                                                       const float* __restrict__ fbw,
                                                       const T* __restrict__ Au, const T* __restrict__ Av,
                                                       const T* __restrict__ Gu, const T* __restrict__ Gv,
                                                       double aA, double aG,
                                                       const T* __restrict__ addu, const T* __restrict__ addv,
                                                       T* __restrict__ ou, T* __restrict__ ov, AdjPhys ph,
                                                       int nx, int ny) {
  const size_t n = (size_t)nx * ny;
  const int b = blockIdx.y;
  const size_t off = (size_t)b * n;
  constexpr bool LEARNED = MODE == 1 || MODE == 3;
  const T* S = scr + (size_t)b * kAdjPlanes * n;
  const float* cb = LEARNED ? coef + (size_t)b * cbs : nullptr;
  const float* db = MODE == 3 ? dcoef + (size_t)b * cbs : nullptr;
  const T wv[4] = {(T)1, (T)-27, (T)27, (T)-1};  // derivative weights for offsets -1..2
  const int lnx = __builtin_ctz(nx);  // nx is a power of two
  // learned modes: QS adjacent lanes per cell, lane q gathering footprint
  // points 4q..4q+3 of every kind (4x the wavefronts in flight for the
  // scattered coefficient loads); the partial sums are combined by two
  // fixed xor-shuffle steps, so every lane of the cell holds the same total
  constexpr int QS = LEARNED ? 4 : 1;
  const int q = (int)threadIdx.x & (QS - 1);
  for (size_t c = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / QS; c < n;
       c += (size_t)gridDim.x * blockDim.x / QS) {
    const int i = (int)c & (nx - 1), j = (int)c >> lnx;
    auto at = [&](int plane, int ii, int jj) {
      return S[(size_t)plane * n + (size_t)(jj & (ny - 1)) * nx + (ii & (nx - 1))];
    };
    auto cidx = [&](int ii, int jj) { return (size_t)(jj & (ny - 1)) * nx + (ii & (nx - 1)); };
    // stencil multiplier sent by owner o for point s of kind K
    auto coefv = [&](int K, int s, int ii, int jj) -> T {
      if (LEARNED) {
        const size_t o = cidx(ii, jj);
        return (T)cb[(size_t)(16 * K + s) * n + o] - S[(size_t)(12 + K) * n + o] +
               ((s == 5 || s == 6) ? (T)0.5 : (T)0);
      }
      return (s == 5 || s == 6) ? (T)0.5 : (T)0;
    };
    T gu = 0, gv = 0;
    if (q == 0) {
      // advecting-velocity parts
      gu += at(0, i, j) + at(0, i - 1, j);          // P0: u(o), u(o+x)
      gu += at(2, i - 1, j + 1) + at(2, i - 1, j);  // P2: u(o+x, o-y), u(o+x)
      gv += at(1, i + 1, j - 1) + at(1, i, j - 1);  // P1: v(o-x+y), v(o+y)
      gv += at(3, i, j) + at(3, i, j - 1);          // P3: v(o), v(o+y)
    }
    // footprint point 4q + k: a 4 x 3 block for q < 3 (offsets (k-1, q-1)),
    // the points (0|1, -2) and (0|1, 2) for q = 3
    const bool blk = q < 3;
    auto pa = [&](int k) { return blk ? k - 1 : (k & 1); };
    auto pb = [&](int k) { return blk ? q - 1 : (k < 2 ? -2 : 2); };
    // interpolation stencils
    if (LEARNED) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int s = 4 * q + k;
        const int a = pa(k), bb = pb(k);
        gu += coefv(0, s, i - a, j - bb) * at(4, i - a, j - bb);
        gu += coefv(1, s, i - bb, j - a) * at(5, i - bb, j - a);
        gv += coefv(2, s, i - a, j - bb) * at(6, i - a, j - bb);
        gv += coefv(3, s, i - bb, j - a) * at(7, i - bb, j - a);
      }
    } else {
      gu += (T)0.5 * (at(4, i, j) + at(4, i - 1, j));
      gu += (T)0.5 * (at(5, i, j) + at(5, i, j - 1));
      gv += (T)0.5 * (at(6, i, j) + at(6, i - 1, j));
      gv += (T)0.5 * (at(7, i, j) + at(7, i, j - 1));
    }
    if constexpr (MODE == 2) {
      // uniform kernels: owner o = p - offset sends w * Q (interpolation) and
      // 24 w^d * V (derivative: V holds -nu Fb / (24 h))
#pragma unroll
      for (int s = 0; s < 20; ++s) {
        const int a = a_off20(s), bb = b_off20(s);
        gu += (T)fbw[s] * at(4, i - a, j - bb) + (T)fbw[20 + s] * at(5, i - bb, j - a);
        gv += (T)fbw[40 + s] * at(6, i - a, j - bb) + (T)fbw[60 + s] * at(7, i - bb, j - a);
        gu += (T)24 * ((T)fbw[80 + s] * at(8, i - a, j - bb) + (T)fbw[100 + s] * at(9, i - bb, j - a));
        gv += (T)24 * ((T)fbw[120 + s] * at(10, i - a, j - bb) + (T)fbw[140 + s] * at(11, i - bb, j - a));
      }
    }
    if constexpr (MODE == 3) {
      // learned face derivatives: owner o sends 24 V w_s (V = -nu Fb / (24 h))
      // to its footprint point s, w rebuilt from o's raw values and moments
      auto dw = [&](int K, int s, int a, int bb, int ii, int jj) -> T {
        const size_t o = cidx(ii, jj);
        return (T)db[(size_t)(16 * K + s) * n + o] - S[(size_t)(16 + K) * n + o] -
               ((T)a - (T)0.5) * S[(size_t)(20 + K) * n + o] -
               (T)bb * S[(size_t)(24 + K) * n + o] + (T)deriv4_w(s);
      };
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int s = 4 * q + k;
        const int a = pa(k), bb = pb(k);
        gu += (T)24 * (dw(0, s, a, bb, i - a, j - bb) * at(8, i - a, j - bb) +
                       dw(1, s, a, bb, i - bb, j - a) * at(9, i - bb, j - a));
        gv += (T)24 * (dw(2, s, a, bb, i - a, j - bb) * at(10, i - a, j - bb) +
                       dw(3, s, a, bb, i - bb, j - a) * at(11, i - bb, j - a));
      }
    } else if (q == 0) {
      // viscous face derivatives: owner o = p - m sends V * w_m to p
#pragma unroll
      for (int m = -1; m <= 2; ++m) {
        const T w = wv[m + 1];
        gu += w * (at(8, i - m, j) + at(9, i, j - m));
        gv += w * (at(10, i - m, j) + at(11, i, j - m));
      }
    }
    if constexpr (QS > 1) {
      gu += __shfl_xor(gu, 1);
      gv += __shfl_xor(gv, 1);
      gu += __shfl_xor(gu, 2);
      gv += __shfl_xor(gv, 2);
      if (q != 0) continue;
    }
    if (ph.mask & LDSV_FORCING) {
      T lu = (T)aA * Au[off + c], lv = (T)aA * Av[off + c];
      if (Gu) {
        lu += (T)aG * Gu[off + c];
        lv += (T)aG * Gv[off + c];
      }
      gu -= (T)ph.drag * lu;
      gv -= (T)ph.drag * lv;
    }
    if (addu) {
      gu += addu[off + c];
      gv += addv[off + c];
    }
    ou[off + c] = gu;
    ov[off + c] = gv;
  }
}

// Per-tile partial sums of the uniform-kernel gradients.  A tile is TX x TY
// cells of one trajectory (TX * TY <= 256); thread w < 160 owns weight w =
// (m, K, s) and sums M_K * q_s over the tile's cells, with M the
// interpolation multiplier Q (m = 0) or the derivative multiplier 24 V
// (m = 1).  part[tile][w] is written, never accumulated.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_fb_wgrad(const T* __restrict__ us,
                                                         const T* __restrict__ vs,
                                                         const T* __restrict__ scr,
                                                         T* __restrict__ part, int nx, int ny, int TX,
                                                         int TY) {
  // (TY + 4) x (TX + 4) <= 544 for every TX in [4, 64] with TX * TY <= 256
  constexpr int kHalo = 544;
  __shared__ T su[kHalo];
  __shared__ T sv[kHalo];
  __shared__ T sm[8][256];
  const size_t n = (size_t)nx * ny;
  const int tilesx = nx / TX;
  const int b = blockIdx.y;
  const int i0 = (blockIdx.x % tilesx) * TX, j0 = (blockIdx.x / tilesx) * TY;
  const T* u = us + (size_t)b * n;
  const T* v = vs + (size_t)b * n;
  const T* S = scr + (size_t)b * kAdjPlanes * n;
  const int W = TX + 4, H = TY + 4;
  for (int t = threadIdx.x; t < W * H; t += blockDim.x) {
    const int r = t / W, c = t - r * W;
    const size_t g = (size_t)((j0 - 2 + r + ny) & (ny - 1)) * nx + ((i0 - 2 + c + nx) & (nx - 1));
    su[t] = u[g];
    sv[t] = v[g];
  }
  for (int t = threadIdx.x; t < TX * TY; t += blockDim.x) {
    const int r = t / TX, c = t - r * TX;
    const size_t g = (size_t)(j0 + r) * nx + (i0 + c);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sm[k][t] = S[(size_t)(4 + k) * n + g];
      sm[4 + k][t] = (T)24 * S[(size_t)(8 + k) * n + g];
    }
  }
  __syncthreads();
  const int w = threadIdx.x;
  if (w < 160) {
    const int m = w / 80, K = (w / 20) & 3, s = w % 20;
    const int a = a_off20(s), bb = b_off20(s);
    const bool along_x = (K == 0 || K == 2);
    const int dr = along_x ? bb : a, dc = along_x ? a : bb;
    const T* F = (K < 2 ? su : sv) + (2 + dr) * W + 2 + dc;
    const T* M = sm[4 * m + K];
    T acc = 0;
    for (int r = 0; r < TY; ++r)
      for (int c = 0; c < TX; ++c) acc += M[r * TX + c] * F[r * W + c];
    part[((size_t)b * gridDim.x + blockIdx.x) * 160 + w] = acc;
  }
}

// gw[w] += sum over the tiles of part[tile][w], in a fixed order
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fb_wreduce(const T* __restrict__ part, int ntiles,
                                                       float* __restrict__ gw) {
  __shared__ T red[kBlock];
  const int w = blockIdx.x;
  T acc = 0;
  for (int t = threadIdx.x; t < ntiles; t += kBlock) acc += part[(size_t)t * 160 + w];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) gw[w] += (float)red[0];
}

template <typename T>
__global__ void k_axpy2(T* yu, T* yv, const T* xu, const T* xv, T a, size_t n) {
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x) {
    yu[g] += a * xu[g];
    yv[g] += a * xv[g];
  }
}

// tile of the uniform-kernel gradient reduction: TX = min(nx, 64) columns,
// TY = min(ny, 256 / TX) rows
inline void fb_wgrad_tile(int nx, int ny, int* tx, int* ty) {
  *tx = nx < 64 ? nx : 64;
  *ty = ny < 256 / *tx ? ny : 256 / *tx;
}

template <typename T>
int adj_rhs_t(ldsv_handle* h, const ldsv_params* prm, const float* coef, size_t cbs,
              float* gcoef, size_t gcbs, const void* us, const void* vs, const void* Au,
              const void* Av, const void* Gu, const void* Gv, double aA, double aG,
              const void* addu, const void* addv, void* ou, void* ov, hipStream_t st,
              const FluxBlockArgs* fbp, const DerivCoef* dc) {
  AdjPhys ph{prm->nu, prm->drag, h->g.lx / h->g.nx, h->g.ly / h->g.ny, prm->physics_mask};
  const int nx = h->g.nx, ny = h->g.ny;
  dim3 grid((unsigned)std::min<size_t>((h->ncell + kBlock - 1) / kBlock, 4096), h->g.batch);
  // the learned-mode gathers run 4 lanes per cell
  dim3 grid4((unsigned)std::min<size_t>(4 * ((h->ncell + kBlock - 1) / kBlock), 4096), h->g.batch);
  T* scr = (T*)h->adj_g;
  AdjFB fb{nullptr, nullptr, 0, nullptr, 0};
  if (fbp) fb = AdjFB{fbp->w, fbp->f, fbp->fbs, fbp->gf, fbp->gfbs};
  if (fbp && fbp->w) {
    LDSV_TLAUNCH(h, 6, (k_adj_faces<T, 2>), grid, dim3(kBlock), 0, st, (const T*)us,
                       (const T*)vs, (const T*)Au, (const T*)Av, (const T*)Gu, (const T*)Gv, aA,
                       aG, (const float*)nullptr, (size_t)0, (float*)nullptr, (size_t)0,
                       (const float*)nullptr, (float*)nullptr, fb, scr, ph, nx, ny);
    if (fbp->gw) {
      int tx, ty;
      fb_wgrad_tile(nx, ny, &tx, &ty);
      const int tiles = (nx / tx) * (ny / ty);
      LDSV_TLAUNCH(h, 6, k_adj_fb_wgrad<T>, dim3(tiles, h->g.batch), dim3(kBlock), 0, st,
                         (const T*)us, (const T*)vs, (const T*)scr, (T*)h->fb_part, nx, ny, tx, ty);
      LDSV_TLAUNCH(h, 6, k_fb_wreduce<T>, dim3(160), dim3(kBlock), 0, st, (const T*)h->fb_part,
                         tiles * h->g.batch, fbp->gw);
    }
    LDSV_TLAUNCH(h, 6, (k_adj_gather<T, 2>), grid, dim3(kBlock), 0, st, (const T*)scr,
                       (const float*)nullptr, (size_t)0, (const float*)nullptr, fbp->w, (const T*)Au, (const T*)Av,
                       (const T*)Gu, (const T*)Gv, aA, aG, (const T*)addu, (const T*)addv,
                       (T*)ou, (T*)ov, ph, nx, ny);
  } else if (coef && dc && dc->d) {
    LDSV_TLAUNCH(h, 6, (k_adj_faces<T, 3>), grid, dim3(kBlock), 0, st, (const T*)us,
                       (const T*)vs, (const T*)Au, (const T*)Av, (const T*)Gu, (const T*)Gv, aA,
                       aG, coef, cbs, gcoef, gcbs, dc->d, dc->gd, fb, scr, ph, nx, ny);
    LDSV_TLAUNCH(h, 6, (k_adj_gather<T, 3>), grid4, dim3(kBlock), 0, st, (const T*)scr, coef,
                       cbs, dc->d, (const float*)nullptr, (const T*)Au, (const T*)Av,
                       (const T*)Gu, (const T*)Gv, aA, aG, (const T*)addu, (const T*)addv,
                       (T*)ou, (T*)ov, ph, nx, ny);
  } else if (coef) {
    LDSV_TLAUNCH(h, 6, (k_adj_faces<T, 1>), grid, dim3(kBlock), 0, st, (const T*)us,
                       (const T*)vs, (const T*)Au, (const T*)Av, (const T*)Gu, (const T*)Gv, aA,
                       aG, coef, cbs, gcoef, gcbs, (const float*)nullptr, (float*)nullptr, fb,
                       scr, ph, nx, ny);
    LDSV_TLAUNCH(h, 6, (k_adj_gather<T, 1>), grid4, dim3(kBlock), 0, st, (const T*)scr, coef,
                       cbs, (const float*)nullptr, (const float*)nullptr, (const T*)Au, (const T*)Av, (const T*)Gu,
                       (const T*)Gv, aA, aG, (const T*)addu, (const T*)addv, (T*)ou, (T*)ov, ph,
                       nx, ny);
  } else {
    LDSV_TLAUNCH(h, 6, (k_adj_faces<T, 0>), grid, dim3(kBlock), 0, st, (const T*)us,
                       (const T*)vs, (const T*)Au, (const T*)Av, (const T*)Gu, (const T*)Gv, aA,
                       aG, (const float*)nullptr, (size_t)0, (float*)nullptr, (size_t)0,
                       (const float*)nullptr, (float*)nullptr, fb, scr, ph, nx, ny);
    LDSV_TLAUNCH(h, 6, (k_adj_gather<T, 0>), grid, dim3(kBlock), 0, st, (const T*)scr,
                       (const float*)nullptr, (size_t)0, (const float*)nullptr,
                       (const float*)nullptr, (const T*)Au,
                       (const T*)Av, (const T*)Gu, (const T*)Gv, aA, aG, (const T*)addu,
                       (const T*)addv, (T*)ou, (T*)ov, ph, nx, ny);
  }
  LDSV_LAUNCHED();
  return LDSV_OK;
}

}  // namespace

int ldsv_ensure_adjoint(ldsv_handle* h) {
  if (!h->fb_part) {
    int tx, ty;
    fb_wgrad_tile(h->g.nx, h->g.ny, &tx, &ty);
    const size_t tiles = (size_t)(h->g.nx / tx) * (h->g.ny / ty) * h->g.batch;
    LDSV_TRY(ldsv_alloc(h, &h->fb_part, tiles * 160 * h->esize, "flux-block gradient partials"));
  }
  if (h->adj_g) return LDSV_OK;
  const size_t sb = h->nstate * h->esize;
  // 6 stage planes (u1..u3), A, S, W, G (2 planes each) and the scratch planes
  void* blk = nullptr;
  LDSV_TRY(ldsv_alloc(h, &blk, (6 + 8 + kAdjPlanes) * sb, "adjoint workspace"));
  h->stage_keep = blk;
  h->adj_u = (char*)blk + 6 * sb;  // A (2), S (2), W (2), G (2)
  h->adj_g = (char*)blk + 14 * sb;
  return LDSV_OK;
}

// w = J_R(u)^T (aA A + aG G) [+ add]; optional coefficient gradient
int ldsv_launch_adj_rhs(ldsv_handle* h, const ldsv_params* prm, const float* coef, size_t cbs,
                        float* gcoef, size_t gcbs, const void* us, const void* vs, const void* Au,
                        const void* Av, const void* Gu, const void* Gv, double aA, double aG,
                        const void* addu, const void* addv, void* ou, void* ov, hipStream_t st,
                        const FluxBlockArgs* fb, const DerivCoef* dc) {
  if (h->g.dtype == LDSV_F64)
    return adj_rhs_t<double>(h, prm, coef, cbs, gcoef, gcbs, us, vs, Au, Av, Gu, Gv, aA, aG, addu,
                             addv, ou, ov, st, fb, dc);
  return adj_rhs_t<float>(h, prm, coef, cbs, gcoef, gcbs, us, vs, Au, Av, Gu, Gv, aA, aG, addu,
                          addv, ou, ov, st, fb, dc);
}

int ldsv_launch_axpy2(ldsv_handle* h, void* yu, void* yv, const void* xu, const void* xv, double a,
                      hipStream_t st) {
  if (h->g.dtype == LDSV_F64)
    LDSV_TLAUNCH(h, 7, k_axpy2<double>, grid1d(h->nstate), dim3(kBlock), 0, st, (double*)yu,
                       (double*)yv, (const double*)xu, (const double*)xv, a, h->nstate);
  else
    LDSV_TLAUNCH(h, 7, k_axpy2<float>, grid1d(h->nstate), dim3(kBlock), 0, st, (float*)yu,
                       (float*)yv, (const float*)xu, (const float*)xv, (float)a, h->nstate);
  LDSV_LAUNCHED();
  return LDSV_OK;
}
