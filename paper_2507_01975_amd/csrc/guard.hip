// The rollout guard of a learned step on small grids, in one launch (Eq. 2
// recursion with the plain-FV fallback): one workgroup per trajectory pair
//   1. flags each trajectory of the pair whose learned state u_k is
//      non-finite or has max(|u| + |v|) >= the bound (FP64 comparison);
//   2. if one is flagged (and the redo is enabled), runs the whole plain FV
//      step from u_{k-1} for the pair in LDS: four RK4 stages, each the
//      finite-volume residual (App. B.2, S1-S7: linear face interpolation,
//      advective fluxes, fourth-order viscous fluxes, forcing and drag), the
//      stage combination (App. B.5, S15-S20) and the spectral projection
//      (App. B.3-B.4, S8-S14) of the pair packed as one complex field;
//   3. writes the redone state over u_k for the flagged trajectories only.
// The arithmetic is that of the stage and projection kernels (the same
// expressions, face by face and element by element), with the state of the
// pair resident in LDS between the stages instead of in HBM, so a guarded
// step costs one launch more than a bare learned step instead of the nine
// of a separately launched detection and plain step.
#include "fft_lds.h"

int ldsv_launch_guard_redo(ldsv_handle* h, const ldsv_params* prm, const float* cu,
                           const float* cv, float* nu, float* nv, double thr, int redo,
                           int* counts, int* any, const double* smax, hipStream_t st);

namespace {

constexpr int kRedoBlock = 1024;
constexpr int kRedoE = 4;  // cells per thread: grids of at most 64 x 64

struct RedoArgs {
  const float* cu;
  const float* cv;
  float* nu;
  float* nv;
  const Cx<float>* twx;
  const Cx<float>* twy;
  const double* pinv;
  int nx, ny, log2nx, log2ny, batch, ra;
  float visc_nu, drag, idx, idy, i24dx, i24dy;
  double amp, kf, dy;
  int mask;
  float comb[4][6];  // per RK4 stage: alpha, beta, delta, eps, gamma, wacc
  double thr;
  int redo;
  int* counts;
  int* any;
  const double* smax;  // nullable: max(|u| + |v|) per trajectory of the learned state
};

__global__ void __launch_bounds__(kRedoBlock) k_guard_redo_pair(RedoArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  constexpr int E = kRedoE;
  const int nx = a.nx, ny = a.ny, n = nx * ny;
  const int pair = blockIdx.x, b0 = 2 * pair;
  const bool has1 = b0 + 1 < a.batch;
  const size_t plane = (size_t)n;
  Cx<float>* Z = reinterpret_cast<Cx<float>*>(smem_raw);  // pair spectrum, rows padded to ra
  Cx<float>* Wx = Z + ny * a.ra;
  Cx<float>* Wy = Wx + nx;
  float* S = reinterpret_cast<float*>(Wy + ny);  // stage state: planes u0, v0, u1, v1
  float* frow = S + 4 * n;
  double* red = reinterpret_cast<double*>(frow + ny + (ny & 1));
  int* flag = reinterpret_cast<int*>(red + 2 * (kRedoBlock / 64));

  // 1. the guard: largest |u| + |v| per trajectory of the learned state
  // (written by the step's last projection when smax is set)
  double m0 = 0.0, m1 = 0.0;
  if (a.smax) {
    m0 = a.smax[b0];
    m1 = has1 ? a.smax[b0 + 1] : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kRedoBlock + (int)threadIdx.x;
      if (t < n) {
        const size_t g0 = (size_t)b0 * plane + t;
        const double s0 = (double)fabsf(a.nu[g0]) + (double)fabsf(a.nv[g0]);
        m0 = isfinite(s0) ? fmax(m0, s0) : INFINITY;
        if (has1) {
          const double s1 = (double)fabsf(a.nu[g0 + plane]) + (double)fabsf(a.nv[g0 + plane]);
          m1 = isfinite(s1) ? fmax(m1, s1) : INFINITY;
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    m0 = fmax(m0, __shfl_xor(m0, o));
    m1 = fmax(m1, __shfl_xor(m1, o));
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = m0;
    red[kRedoBlock / 64 + (threadIdx.x >> 6)] = m1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRedoBlock / 64; ++w) {
      m0 = fmax(m0, red[w]);
      m1 = fmax(m1, red[kRedoBlock / 64 + w]);
    }
    const int f0 = !(m0 < a.thr);
    const int f1 = has1 && !(m1 < a.thr);
    flag[0] = f0;
    flag[1] = f1;
    if (f0 || f1) {
      if (a.counts) {
        if (f0) a.counts[b0] += 1;
        if (f1) a.counts[b0 + 1] += 1;
      }
      atomicOr(a.any, 1);
    }
  }
  __syncthreads();
  const bool bad0 = flag[0] != 0, bad1 = flag[1] != 0;
  if (!a.redo || !(bad0 || bad1)) return;  // uniform over the workgroup

  // 2. the plain step of the pair from u_{k-1}
  for (int e = threadIdx.x; e < nx; e += kRedoBlock) Wx[e] = a.twx[e];
  for (int e = threadIdx.x; e < ny; e += kRedoBlock) Wy[e] = a.twy[e];
  const bool force = a.mask & LDSV_FORCING;
  if (force)
    for (int j = threadIdx.x; j < ny; j += kRedoBlock)
      frow[j] = a.amp != 0.0 ? (float)(a.amp * sin(a.kf * (j + 0.5) * a.dy)) : 0.f;
  float un[E][4], acc[E][4], ust[E][4];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int t = k * kRedoBlock + (int)threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      un[k][q] = 0.f;
      acc[k][q] = 0.f;
      ust[k][q] = 0.f;
    }
    if (t < n) {
      const size_t g0 = (size_t)b0 * plane + t;
      un[k][0] = a.cu[g0];
      un[k][1] = a.cv[g0];
      if (has1) {
        un[k][2] = a.cu[g0 + plane];
        un[k][3] = a.cv[g0 + plane];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) S[q * n + t] = un[k][q];
    }
  }
  __syncthreads();
  const bool adv = a.mask & LDSV_ADVECTION;
  const bool visc = a.mask & LDSV_VISCOSITY;
  const float vnu = a.visc_nu, i24dx = a.i24dx, i24dy = a.i24dy, idx = a.idx, idy = a.idy;
  for (int s = 0; s < 4; ++s) {
    const float al = a.comb[s][0], be = a.comb[s][1], de = a.comb[s][2], ep = a.comb[s][3],
                ga = a.comb[s][4], wa = a.comb[s][5];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kRedoBlock + (int)threadIdx.x;
      if (t >= n) break;
      const int j = t >> a.log2nx;
      const int i = t & (nx - 1);
#pragma unroll
      for (int tr = 0; tr < 2; ++tr) {
        if (tr == 1 && !has1) break;
        const float* U = S + (2 * tr) * n;
        const float* V = U + n;
        auto q = [&](const float* A, int di, int dj) {
          return A[((j + dj) & (ny - 1)) * nx + ((i + di) & (nx - 1))];
        };
        // face fluxes owned by the cell at offset (di, dj): x-faces of u and
        // v, y-faces of u and v
        auto fxu = [&](int di) {
          float f = 0.f;
          if (adv) {
            const float ubar = 0.5f * (q(U, di, 0) + q(U, di + 1, 0));
            const float uf = 0.5f * (q(U, di, 0) + q(U, di + 1, 0));
            f = ubar * uf;
          }
          if (visc)
            f -= vnu * (q(U, di - 1, 0) - 27.f * q(U, di, 0) + 27.f * q(U, di + 1, 0) -
                        q(U, di + 2, 0)) * i24dx;
          return f;
        };
        auto fxv = [&](int di) {
          float f = 0.f;
          if (adv) {
            const float ubar_e = 0.5f * (q(U, di + 1, -1) + q(U, di + 1, 0));
            const float vf = 0.5f * (q(V, di, 0) + q(V, di + 1, 0));
            f = ubar_e * vf;
          }
          if (visc)
            f -= vnu * (q(V, di - 1, 0) - 27.f * q(V, di, 0) + 27.f * q(V, di + 1, 0) -
                        q(V, di + 2, 0)) * i24dx;
          return f;
        };
        auto fyu = [&](int dj) {
          float f = 0.f;
          if (adv) {
            const float vbar_n = 0.5f * (q(V, -1, dj + 1) + q(V, 0, dj + 1));
            const float uf = 0.5f * (q(U, 0, dj) + q(U, 0, dj + 1));
            f = vbar_n * uf;
          }
          if (visc)
            f -= vnu * (q(U, 0, dj - 1) - 27.f * q(U, 0, dj) + 27.f * q(U, 0, dj + 1) -
                        q(U, 0, dj + 2)) * i24dy;
          return f;
        };
        auto fyv = [&](int dj) {
          float f = 0.f;
          if (adv) {
            const float vbar_c = 0.5f * (q(V, 0, dj) + q(V, 0, dj + 1));
            const float vf = 0.5f * (q(V, 0, dj) + q(V, 0, dj + 1));
            f = vbar_c * vf;
          }
          if (visc)
            f -= vnu * (q(V, 0, dj - 1) - 27.f * q(V, 0, dj) + 27.f * q(V, 0, dj + 1) -
                        q(V, 0, dj + 2)) * i24dy;
          return f;
        };
        const float uc = q(U, 0, 0), vc = q(V, 0, 0);
        float ru = -(fxu(0) - fxu(-1)) * idx - (fyu(0) - fyu(-1)) * idy;
        float rv = -(fxv(0) - fxv(-1)) * idx - (fyv(0) - fyv(-1)) * idy;
        if (force) {
          ru += frow[j] - a.drag * uc;
          rv -= a.drag * vc;
        }
        // u_n enters from the second stage on (as in the stage kernels,
        // which do not read it in the first)
        const float pun = s ? un[k][2 * tr] : 0.f, pvn = s ? un[k][2 * tr + 1] : 0.f;
        ust[k][2 * tr] = be * uc + ep * ru + al * pun + de * acc[k][2 * tr];
        ust[k][2 * tr + 1] = be * vc + ep * rv + al * pvn + de * acc[k][2 * tr + 1];
        if (s < 3) {
          acc[k][2 * tr] = ga * acc[k][2 * tr] + wa * ru;
          acc[k][2 * tr + 1] = ga * acc[k][2 * tr + 1] + wa * rv;
        }
      }
    }
    __syncthreads();  // every read of the stage state is done
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kRedoBlock + (int)threadIdx.x;
      if (t < n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) S[q * n + t] = ust[k][q];
      }
    }
    __syncthreads();
    // projection of u*: divergence of the pair packed as d0 + i d1
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kRedoBlock + (int)threadIdx.x;
      if (t < n) {
        const int j = t >> a.log2nx;
        const int i = t & (nx - 1);
        const int ip = (i + 1) & (nx - 1);
        const int jp = (j + 1) & (ny - 1);
        const float d0 = (S[j * nx + ip] - ust[k][0]) * idx + (S[n + jp * nx + i] - ust[k][1]) * idy;
        float d1 = 0.f;
        if (has1)
          d1 = (S[2 * n + j * nx + ip] - ust[k][2]) * idx +
               (S[3 * n + jp * nx + i] - ust[k][3]) * idy;
        Z[j * a.ra + i] = Cx<float>{d0, d1};
      }
    }
    __syncthreads();
    lds_fft<float, E, true>(Z, nx, a.log2nx, ny, a.ra, 1, -1, Wx);
    lds_fft<float, E, true>(Z, ny, a.log2ny, nx, 1, a.ra, -1, Wy);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kRedoBlock + (int)threadIdx.x;
      if (t < n) {
        const double f = a.pinv[t];
        const int e = (t >> a.log2nx) * a.ra + (t & (nx - 1));
        const Cx<float> v = Z[e];
        Z[e] = Cx<float>{(float)((double)v.x * f), (float)((double)v.y * f)};
      }
    }
    __syncthreads();
    lds_fft<float, E, true>(Z, ny, a.log2ny, nx, 1, a.ra, +1, Wy);
    lds_fft<float, E, true>(Z, nx, a.log2nx, ny, a.ra, 1, +1, Wx);
    // gradient correction: the next stage state, or the redone u_k
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kRedoBlock + (int)threadIdx.x;
      if (t >= n) break;
      const int j = t >> a.log2nx;
      const int i = t & (nx - 1);
      const Cx<float> pc = Z[j * a.ra + i];
      const Cx<float> pw = Z[j * a.ra + ((i - 1) & (nx - 1))];
      const Cx<float> ps = Z[((j - 1) & (ny - 1)) * a.ra + i];
      const float u0 = ust[k][0] - (pc.x - pw.x) * idx;
      const float v0 = ust[k][1] - (pc.x - ps.x) * idy;
      const float u1 = ust[k][2] - (pc.y - pw.y) * idx;
      const float v1 = ust[k][3] - (pc.y - ps.y) * idy;
      if (s < 3) {
        S[t] = u0;
        S[n + t] = v0;
        S[2 * n + t] = u1;
        S[3 * n + t] = v1;
      } else {
        const size_t g0 = (size_t)b0 * plane + t;
        if (bad0) {
          a.nu[g0] = u0;
          a.nv[g0] = v0;
        }
        if (bad1) {
          a.nu[g0 + plane] = u1;
          a.nv[g0 + plane] = v1;
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace

// One launch: the guard of the learned state (nu, nv) and, with redo, the
// plain step from (cu, cv) written over the flagged trajectories.  Returns
// LDSV_ESHAPE (and enqueues nothing) when the grid is not one this kernel
// takes: FP32 MAC RK4 grids of at most 64 x 64 cells.
int ldsv_launch_guard_redo(ldsv_handle* h, const ldsv_params* prm, const float* cu,
                           const float* cv, float* nu, float* nv, double thr, int redo,
                           int* counts, int* any, const double* smax, hipStream_t st) {
  const int nx = h->g.nx, ny = h->g.ny;
  if (h->g.dtype != LDSV_F32 || h->g.layout != LDSV_MAC || prm->rk != LDSV_RK4 ||
      (size_t)nx * ny > (size_t)kRedoE * kRedoBlock)
    return LDSV_ESHAPE;
  int ra = nx + lds_row_pad(nx);
  auto lds_bytes = [&](int r) {
    return (size_t)ny * r * sizeof(Cx<float>) + (size_t)(nx + ny) * sizeof(Cx<float>) +
           (size_t)4 * nx * ny * sizeof(float) + (size_t)(ny + 1) * sizeof(float) +
           2 * (kRedoBlock / 64) * sizeof(double) + 4 * sizeof(int);
  };
  if (lds_bytes(ra) > 163840) ra = nx;
  const size_t lds = lds_bytes(ra);
  if (lds > 163840) return LDSV_ESHAPE;
  RedoArgs a;
  a.cu = cu;
  a.cv = cv;
  a.nu = nu;
  a.nv = nv;
  a.twx = (const Cx<float>*)h->twx;
  a.twy = (const Cx<float>*)h->twy;
  a.pinv = h->pinv;
  a.nx = nx;
  a.ny = ny;
  a.log2nx = h->log2nx;
  a.log2ny = h->log2ny;
  a.batch = h->g.batch;
  a.ra = ra;
  const double dx = h->g.lx / nx, dy = h->g.ly / ny;
  // the physical constants and stage coefficients rounded as the stage
  // kernels round them
  a.visc_nu = (float)prm->nu;
  a.drag = (float)prm->drag;
  a.idx = (float)(1.0 / dx);
  a.idy = (float)(1.0 / dy);
  a.i24dx = (float)(1.0 / (24.0 * dx));
  a.i24dy = (float)(1.0 / (24.0 * dy));
  a.amp = prm->forcing_amp;
  a.kf = prm->forcing_k;
  a.dy = dy;
  a.mask = prm->physics_mask;
  const double dt = prm->dt;
  const double eps[4] = {0.5 * dt, 0.5 * dt, dt, dt / 6.0};
  for (int s = 0; s < 4; ++s) {
    a.comb[s][0] = (float)(s == 0 ? 0.0 : 1.0);                 // alpha
    a.comb[s][1] = (float)(s == 0 ? 1.0 : 0.0);                 // beta
    a.comb[s][2] = (float)(s == 3 ? dt / 6.0 : 0.0);            // delta
    a.comb[s][3] = (float)eps[s];                               // eps
    a.comb[s][4] = (float)((s == 1 || s == 2) ? 1.0 : 0.0);     // gamma
    a.comb[s][5] = (float)(s == 0 ? 1.0 : 2.0);                 // wacc
  }
  a.thr = thr;
  a.redo = redo;
  a.counts = counts;
  a.any = any;
  a.smax = smax;
  LDSV_HIP(hipFuncSetAttribute((const void*)k_guard_redo_pair,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  LDSV_TLAUNCH(h, 7, k_guard_redo_pair, dim3(h->npairs), dim3(kRedoBlock), lds, st, a);
  LDSV_LAUNCHED();
  return LDSV_OK;
}
