// The paper's flux block (Sec. 3.4, Eqs. 5-8): the Fourier neural operator
// O_F (Eq. 8; the FNO of the appendix on baseline models, after Li et al.,
// ICLR 2021) and the entry points of the flux-block step.
//
//   v_0     = P x + b_P                        pointwise lift, 2 -> C
//   v_{l+1} = GELU(K_l v_l + W_l v_l + b_l)    (no GELU after the last layer)
//   F       = Q v_L + b_Q                      pointwise projection, C -> 4
//   K v     = the real inverse transform of R . (retained modes of the real
//             2D transform of v): rows k_y in [0, M) U [Ny - M, Ny), columns
//             k_x < M, complex channel mixing per mode.
//
// The two FNOs (interpolation and derivative) run side by side: grid.z picks
// the network.  Per layer three kernels:
//   k_fno_spec  one workgroup per (channel pair, trajectory, network): the
//               pair packed as one complex field, 2D FFT in LDS (the
//               Stockham transform of the projection), the two real
//               spectra separated by Hermitian symmetry and only the
//               retained modes written out ([net][B][C][2M][M] complex);
//               the first layer computes v_0 from (u, v) on the fly;
//   k_fno_mix   per mode, Y_o = sum_i R_io X_i: a thread owns (mode, output
//               channel) and keeps its C complex weights in registers while
//               the trajectories stream through LDS (one C x 64-mode tile of
//               X per trajectory);
//   k_fno_inv   one workgroup per (output pair, trajectory, network): the
//               Hermitian extension of the two half spectra packed into one
//               complex field (the k_x = 0 column symmetrised, which is the
//               real part a real inverse transform takes), inverse 2D FFT
//               in LDS, then the pointwise term W v + b and GELU fused in
//               the epilogue.  The first layer's pointwise term recomputes
//               v_0 from (u, v).
// and after the last layer k_fno_proj writes the 4 fields of each network
// into the [B][8][Ny][Nx] field array (channels 4 g .. 4 g + 3; zeros for an
// absent network).  Everything is FP32; the FFT is O(N log N) on the vector
// ALU and the mixing is a few complex FMAs per mode, so these kernels are
// bound by their HBM traffic and LDS round trips, not by arithmetic.
#include <utility>

#include "adjoint.h"
#include "cnn_common.h"
#include "fft_lds.h"
#include "fno.h"
#include "stage.h"

namespace {

constexpr int kFnoBlock = 1024;
using c32 = Cx<float>;

struct FnoArgs {
  const float* lift_w[2];
  const float* lift_b[2];
  const c32* spec_w[2];   // this layer's [C][C][nm] complex
  const float* point_w[2];   // this layer's [C][C]
  const float* point_b[2];   // this layer's [C]
  const float* proj_w[2];
  const float* proj_b[2];
  int net[2];                // network run by grid.z slice z
  int slot[2];               // grid.z slice of network g, -1 if absent
};

__device__ __forceinline__ int retained_row(int ky, int ny, int M) {
  if (ky < M) return ky;
  if (ky >= ny - M) return ky - ny + 2 * M;
  return -1;
}

template <int E>
__device__ __forceinline__ void load_twiddles(Cx<float>* Wx, Cx<float>* Wy, const Cx<float>* twx,
                                              const Cx<float>* twy, int nx, int ny) {
  for (int e = threadIdx.x; e < nx; e += blockDim.x) Wx[e] = twx[e];
  for (int e = threadIdx.x; e < ny; e += blockDim.x) Wy[e] = twy[e];
}

// forward transform of channels (2p, 2p+1) of trajectory b, network slice z
template <int E, bool LIFT>
__global__ void __launch_bounds__(kFnoBlock) k_fno_spec(const float* __restrict__ vin,
                                                        const float* __restrict__ vin2, FnoArgs a,
                                                        c32* __restrict__ X,
                                                        const Cx<float>* __restrict__ twx,
                                                        const Cx<float>* __restrict__ twy, int nx,
                                                        int ny, int log2nx, int log2ny, int C, int M,
                                                        int B) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  Cx<float>* A = reinterpret_cast<Cx<float>*>(smem_raw);
  Cx<float>* Wx = A + nx * ny;
  Cx<float>* Wy = Wx + nx;
  load_twiddles<E>(Wx, Wy, twx, twy, nx, ny);
  const int p = blockIdx.x, b = blockIdx.y, z = blockIdx.z;
  const int g = a.net[z];
  const int c0 = 2 * p, c1 = 2 * p + 1;
  const int n = nx * ny;
  if constexpr (LIFT) {
    const float* u = vin + (size_t)b * n;
    const float* v = vin2 + (size_t)b * n;
    const float* lw = a.lift_w[g];
    const float* lb = a.lift_b[g];
    const float w00 = lw[2 * c0], w01 = lw[2 * c0 + 1], w10 = lw[2 * c1], w11 = lw[2 * c1 + 1];
    const float b0 = lb[c0], b1 = lb[c1];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kFnoBlock + (int)threadIdx.x;
      if (t < n) {
        const float x0 = u[t], x1 = v[t];
        A[t] = Cx<float>{w00 * x0 + w01 * x1 + b0, w10 * x0 + w11 * x1 + b1};
      }
    }
  } else {
    const float* s0 = vin + ((size_t)(z * B + b) * C + c0) * n;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * kFnoBlock + (int)threadIdx.x;
      if (t < n) A[t] = Cx<float>{s0[t], s0[n + t]};
    }
  }
  __syncthreads();
  lds_fft<float, E>(A, nx, log2nx, ny, nx, 1, -1, Wx);
  lds_fft<float, E>(A, ny, log2ny, nx, 1, nx, -1, Wy);
  // Z = V0 + i V1 with V0, V1 the transforms of the two real channels:
  // V0(k) = (Z(k) + conj Z(-k)) / 2, V1(k) = (Z(k) - conj Z(-k)) / (2 i)
  const int nm = 2 * M * M;
  c32* X0 = X + ((size_t)(z * B + b) * C + c0) * nm;
  c32* X1 = X0 + nm;
  for (int e = threadIdx.x; e < nm; e += blockDim.x) {
    const int r = e / M, kx = e - r * M;
    const int ky = r < M ? r : ny - 2 * M + r;
    const Cx<float> z1 = A[ky * nx + kx];
    const Cx<float> z2 = A[((ny - ky) & (ny - 1)) * nx + ((nx - kx) & (nx - 1))];
    X0[e] = c32{0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y)};
    X1[e] = c32{0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x)};
  }
}

// Y[z][b][o][m] = sum_i w(i, o, m) X[z][b][i][m]; w = R[i][o][m], or for the
// adjoint (CONJ_T) w = conj(R[o][i][m]).  Block 64 x C: lane = mode within
// the 64-mode tile, wave = output channel; trajectories b0 .. b0 + bpg - 1.
template <int C, bool CONJ_T>
__global__ void __launch_bounds__(64 * C) k_fno_mix(const c32* __restrict__ X, FnoArgs a,
                                                    c32* __restrict__ Y, int B, int nm,
                                                    int bpg) {
  __shared__ c32 xs[2][C][64];
  const int lane = threadIdx.x & 63;
  const int o = threadIdx.x >> 6;
  const int m = blockIdx.x * 64 + lane;
  const int z = blockIdx.z;
  const c32* R = a.spec_w[a.net[z]];
  c32 w[C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    c32 r = c32{0.f, 0.f};
    if (m < nm) {
      if (CONJ_T) {
        r = R[((size_t)o * C + i) * nm + m];
        r.y = -r.y;
      } else {
        r = R[((size_t)i * C + o) * nm + m];
      }
    }
    w[i] = r;
  }
  const int b0 = blockIdx.y * bpg;
  const int b1 = min(B, b0 + bpg);
  for (int b = b0; b < b1; ++b) {
    const int buf = (b - b0) & 1;
    {
      const int i = threadIdx.x >> 6;
      xs[buf][i][lane] = m < nm ? X[((size_t)(z * B + b) * C + i) * nm + m] : c32{0.f, 0.f};
    }
    __syncthreads();
    float ax = 0.f, ay = 0.f;
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const c32 x = xs[buf][i][lane];
      ax += x.x * w[i].x - x.y * w[i].y;
      ay += x.x * w[i].y + x.y * w[i].x;
    }
    if (m < nm) Y[((size_t)(z * B + b) * C + o) * nm + m] = c32{ax, ay};
  }
}

// inverse transform of output channels (2p, 2p+1) + pointwise term + GELU
template <int E, bool LIFT, bool LAST>
__global__ void __launch_bounds__(kFnoBlock) k_fno_inv(const c32* __restrict__ Y,
                                                       const float* __restrict__ vin,
                                                       const float* __restrict__ vin2, FnoArgs a,
                                                       float* __restrict__ vout,
                                                       float* __restrict__ zout,
                                                       const Cx<float>* __restrict__ twx,
                                                       const Cx<float>* __restrict__ twy, int nx,
                                                       int ny, int log2nx, int log2ny, int C, int M,
                                                       int B) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  Cx<float>* A = reinterpret_cast<Cx<float>*>(smem_raw);
  Cx<float>* Wx = A + nx * ny;
  Cx<float>* Wy = Wx + nx;
  load_twiddles<E>(Wx, Wy, twx, twy, nx, ny);
  const int p = blockIdx.x, b = blockIdx.y, z = blockIdx.z;
  const int g = a.net[z];
  const int o0 = 2 * p, o1 = 2 * p + 1;
  const int n = nx * ny;
  const int nm = 2 * M * M;
  const c32* Y0 = Y + ((size_t)(z * B + b) * C + o0) * nm;
  const c32* Y1 = Y0 + nm;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int t = k * kFnoBlock + (int)threadIdx.x;
    if (t < n) {
      const int ky = t >> log2nx, kx = t & (nx - 1);
      Cx<float> zv{0.f, 0.f};
      if (kx == 0) {
        // the real inverse transform reads the real part of the k_x = 0
        // column after the row-direction inverse: symmetrise it
        const int r1 = retained_row(ky, ny, M);
        const int r2 = retained_row((ny - ky) & (ny - 1), ny, M);
        c32 s0{0.f, 0.f}, s1{0.f, 0.f};
        if (r1 >= 0) {
          s0 = Y0[r1 * M];
          s1 = Y1[r1 * M];
        }
        if (r2 >= 0) {
          const c32 q0 = Y0[r2 * M], q1 = Y1[r2 * M];
          s0.x += q0.x;
          s0.y -= q0.y;
          s1.x += q1.x;
          s1.y -= q1.y;
        }
        zv = Cx<float>{0.5f * (s0.x - s1.y), 0.5f * (s0.y + s1.x)};
      } else if (kx < M) {
        const int r = retained_row(ky, ny, M);
        if (r >= 0) {
          const c32 y0 = Y0[r * M + kx], y1 = Y1[r * M + kx];
          zv = Cx<float>{y0.x - y1.y, y0.y + y1.x};
        }
      } else if (kx > nx - M) {
        const int r = retained_row((ny - ky) & (ny - 1), ny, M);
        if (r >= 0) {
          const c32 y0 = Y0[r * M + (nx - kx)], y1 = Y1[r * M + (nx - kx)];
          zv = Cx<float>{y0.x + y1.y, y1.x - y0.y};
        }
      }
      A[t] = zv;
    }
  }
  __syncthreads();
  lds_fft<float, E>(A, nx, log2nx, ny, nx, 1, +1, Wx);
  lds_fft<float, E>(A, ny, log2ny, nx, 1, nx, +1, Wy);
  const float sc = 1.0f / (float)n;
  const float* pw = a.point_w[g];
  const float* pb = a.point_b[g];
  const float bo0 = pb[o0], bo1 = pb[o1];
  float* d0 = vout + ((size_t)(z * B + b) * C + o0) * n;
  float* e0 = zout ? zout + ((size_t)(z * B + b) * C + o0) * n : nullptr;
#pragma unroll 2
  for (int k = 0; k < E; ++k) {
    const int t = k * kFnoBlock + (int)threadIdx.x;
    if (t >= n) break;
    float z0 = A[t].x * sc + bo0, z1 = A[t].y * sc + bo1;
    if constexpr (LIFT) {
      const float x0 = vin[(size_t)b * n + t], x1 = vin2[(size_t)b * n + t];
      const float* lw = a.lift_w[g];
      const float* lb = a.lift_b[g];
      for (int i = 0; i < C; ++i) {
        const float vi = lw[2 * i] * x0 + lw[2 * i + 1] * x1 + lb[i];
        z0 += pw[o0 * C + i] * vi;
        z1 += pw[o1 * C + i] * vi;
      }
    } else {
      const float* s = vin + (size_t)(z * B + b) * C * n + t;
      for (int i = 0; i < C; ++i) {
        const float vi = s[(size_t)i * n];
        z0 += pw[o0 * C + i] * vi;
        z1 += pw[o1 * C + i] * vi;
      }
    }
    if (e0) {
      e0[t] = z0;
      e0[n + t] = z1;
    }
    d0[t] = LAST ? z0 : cnnk::gelu_exact(z0);
    d0[n + t] = LAST ? z1 : cnnk::gelu_exact(z1);
  }
}

// fields[b][4 g + K] = Q_g v_L + b_Q (zeros for an absent network)
__global__ void __launch_bounds__(kBlock) k_fno_proj(const float* __restrict__ vL, FnoArgs a,
                                                     float* __restrict__ fields, int n, int C,
                                                     int B) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y, g = blockIdx.z;
  if (t >= n) return;
  const int z = a.slot[g];
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  if (z >= 0) {
    const float* qw = a.proj_w[g];
    const float* qb = a.proj_b[g];
    const float* s = vL + (size_t)(z * B + b) * C * n + t;
#pragma unroll
    for (int K = 0; K < 4; ++K) acc[K] = qb[K];
    for (int c = 0; c < C; ++c) {
      const float vc = s[(size_t)c * n];
#pragma unroll
      for (int K = 0; K < 4; ++K) acc[K] += qw[K * C + c] * vc;
    }
  }
#pragma unroll
  for (int K = 0; K < 4; ++K) fields[((size_t)b * 8 + 4 * g + K) * n + t] = acc[K];
}

// ---------------------------------------------------------------- host

struct FnoShape {
  int C, L, M, nnet;
};

int check_fluxnet(const ldsv_handle* h, const ldsv_fluxnet* net, FnoShape* sh) {
  LDSV_REQUIRE(net, LDSV_EINVAL, "flux block: null network");
  LDSV_REQUIRE(h->g.dtype == LDSV_F32 && h->g.layout == LDSV_MAC, LDSV_EDTYPE,
               "flux block: the FNO needs an F32 MAC grid");
  sh->nnet = 0;
  sh->C = sh->L = sh->M = 0;
  for (int g = 0; g < 2; ++g) {
    const ldsv_fno* f = net->fno[g];
    if (!f) continue;
    LDSV_REQUIRE(f->width == 8 || f->width == 16, LDSV_EINVAL, "fno[%d]: width %d (8 or 16)", g,
                 f->width);
    LDSV_REQUIRE(f->layers >= 1 && f->layers <= 64, LDSV_EINVAL, "fno[%d]: layers %d", g,
                 f->layers);
    LDSV_REQUIRE(f->modes >= 1 && 2 * f->modes <= h->g.ny && 2 * f->modes <= h->g.nx,
                 LDSV_EINVAL, "fno[%d]: modes %d needs 2 modes <= Ny and modes <= Nx/2", g,
                 f->modes);
    LDSV_REQUIRE(f->lift_w && f->lift_b && f->spec_w && f->point_w && f->point_b && f->proj_w &&
                     f->proj_b,
                 LDSV_EINVAL, "fno[%d]: null parameter", g);
    LDSV_REQUIRE(((uintptr_t)f->spec_w & 7) == 0, LDSV_EINVAL,
                 "fno[%d]: spectral weights must be 8-byte aligned", g);
    if (sh->nnet) {
      LDSV_REQUIRE(f->width == sh->C && f->layers == sh->L && f->modes == sh->M, LDSV_EINVAL,
                   "flux block: the two FNOs must have the same width, layers and modes");
    }
    sh->C = f->width;
    sh->L = f->layers;
    sh->M = f->modes;
    sh->nnet++;
  }
  LDSV_REQUIRE((size_t)h->ncell <= (size_t)16 * kFnoBlock &&
                   (size_t)h->ncell * sizeof(Cx<float>) <= 131072,
               LDSV_ESHAPE, "fno: the grid must fit one LDS transform (Nx Ny <= 16384)");
  return LDSV_OK;
}

// buffers: v ping-pong (2 x nnet B C N floats), X and Y (nnet B C nm complex)
// and, for the backward, the L pre-activations (nnet B C N floats each)
int ensure_fno(ldsv_handle* h, const FnoShape& sh, bool keep_pre, float** v0, float** v1,
               c32** X, c32** Y, float** pre) {
  const size_t act = (size_t)sh.nnet * h->g.batch * sh.C * h->ncell;
  const size_t spec = (size_t)sh.nnet * h->g.batch * sh.C * 2 * sh.M * sh.M;
  const size_t need = (2 * act) * sizeof(float) + 2 * spec * sizeof(c32) +
                      (keep_pre ? (size_t)sh.L * act * sizeof(float) : 0);
  if (need > h->fno_bytes) {
    // grown workspaces are kept (owned by the handle) until ldsv_destroy
    LDSV_TRY(ldsv_alloc(h, &h->fno_blk, need, "FNO workspace"));
    h->fno_bytes = need;
  }
  char* p = (char*)h->fno_blk;
  *X = (c32*)p;
  *Y = (c32*)(p + spec * sizeof(c32));
  *v0 = (float*)(p + 2 * spec * sizeof(c32));
  *v1 = *v0 + act;
  *pre = keep_pre ? *v1 + act : nullptr;
  return LDSV_OK;
}

FnoArgs make_args(const ldsv_fluxnet* net, const FnoShape& sh, int layer) {
  FnoArgs a{};
  int z = 0;
  for (int g = 0; g < 2; ++g) {
    a.slot[g] = -1;
    const ldsv_fno* f = net->fno[g];
    if (!f) continue;
    a.lift_w[g] = f->lift_w;
    a.lift_b[g] = f->lift_b;
    const size_t nm = (size_t)2 * sh.M * sh.M;
    a.spec_w[g] = (const c32*)f->spec_w + (size_t)layer * sh.C * sh.C * nm;
    a.point_w[g] = f->point_w + (size_t)layer * sh.C * sh.C;
    a.point_b[g] = f->point_b + (size_t)layer * sh.C;
    a.proj_w[g] = f->proj_w;
    a.proj_b[g] = f->proj_b;
    a.slot[g] = z;
    a.net[z++] = g;
  }
  return a;
}

template <int E>
int fno_forward_e(ldsv_handle* h, const ldsv_fluxnet* net, const FnoShape& sh, const float* u,
                  const float* v, float* fields, float* pre, float* va, float* vb, c32* X,
                  c32* Y, hipStream_t st) {
  const int nx = h->g.nx, ny = h->g.ny, B = h->g.batch, C = sh.C, M = sh.M;
  const size_t lds = ((size_t)nx * ny + nx + ny) * sizeof(Cx<float>);
  const dim3 gfft(C / 2, B, sh.nnet);
  const int nm = 2 * M * M;
  int bpg = B / 8;
  if (bpg < 1) bpg = 1;
  const dim3 gmix((nm + 63) / 64, (B + bpg - 1) / bpg, sh.nnet);
  const Cx<float>* twx = (const Cx<float>*)h->twx;
  const Cx<float>* twy = (const Cx<float>*)h->twy;
  const size_t act = (size_t)sh.nnet * B * C * h->ncell;
  float* cur = va;
  float* nxt = vb;
  for (int l = 0; l < sh.L; ++l) {
    const FnoArgs a = make_args(net, sh, l);
    const bool first = l == 0, last = l == sh.L - 1;
    float* zl = pre ? pre + (size_t)l * act : nullptr;
    if (first) {
      auto k = k_fno_spec<E, true>;
      LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(kFnoBlock), lds, st, u, v, a, X, twx, twy, nx, ny,
                   h->log2nx, h->log2ny, C, M, B);
    } else {
      auto k = k_fno_spec<E, false>;
      LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(kFnoBlock), lds, st, (const float*)cur,
                   (const float*)nullptr, a, X, twx, twy, nx, ny, h->log2nx, h->log2ny, C, M, B);
    }
    if (C == 16)
      LDSV_TLAUNCH(h, 9, (k_fno_mix<16, false>), gmix, dim3(64 * 16), 0, st, (const c32*)X,
                   a, Y, B, nm, bpg);
    else
      LDSV_TLAUNCH(h, 9, (k_fno_mix<8, false>), gmix, dim3(64 * 8), 0, st, (const c32*)X, a,
                   Y, B, nm, bpg);
    const float* in0 = first ? u : cur;
    const float* in1 = first ? v : nullptr;
#define LDSV_FNO_INV(LF, LS)                                                                     \
  {                                                                                              \
    auto k = k_fno_inv<E, LF, LS>;                                                               \
    LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,     \
                                 (int)lds));                                                     \
    LDSV_TLAUNCH(h, 8, k, gfft, dim3(kFnoBlock), lds, st, (const c32*)Y, in0, in1, a, nxt, zl, \
                 twx, twy, nx, ny, h->log2nx, h->log2ny, C, M, B);                               \
  }
    if (first && last) LDSV_FNO_INV(true, true)
    else if (first) LDSV_FNO_INV(true, false)
    else if (last) LDSV_FNO_INV(false, true)
    else LDSV_FNO_INV(false, false)
#undef LDSV_FNO_INV
    std::swap(cur, nxt);
  }
  const FnoArgs a = make_args(net, sh, 0);
  LDSV_TLAUNCH(h, 7, k_fno_proj, dim3((unsigned)((h->ncell + kBlock - 1) / kBlock), B, 2),
               dim3(kBlock), 0, st, (const float*)cur, a, fields, (int)h->ncell, C, B);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

}  // namespace

int ldsv_launch_fno_forward(ldsv_handle* h, const ldsv_fluxnet* net, const float* u,
                            const float* v, float* fields, bool keep_pre, hipStream_t st) {
  FnoShape sh;
  LDSV_TRY(check_fluxnet(h, net, &sh));
  if (sh.nnet == 0) {
    // no frequency operator: zero fields (a kernel, not a memset, so that
    // the call can sit in a captured graph)
    const FnoArgs a = make_args(net, sh, 0);
    LDSV_TLAUNCH(h, 7, k_fno_proj, dim3((unsigned)((h->ncell + kBlock - 1) / kBlock), h->g.batch, 2),
                 dim3(kBlock), 0, st, (const float*)nullptr, a, fields, (int)h->ncell, 0,
                 h->g.batch);
    LDSV_LAUNCHED();
    return LDSV_OK;
  }
  float *va, *vb, *pre;
  c32 *X, *Y;
  LDSV_TRY(ensure_fno(h, sh, keep_pre, &va, &vb, &X, &Y, &pre));
  if (h->ncell <= (size_t)4 * kFnoBlock)
    return fno_forward_e<4>(h, net, sh, u, v, fields, pre, va, vb, X, Y, st);
  return fno_forward_e<16>(h, net, sh, u, v, fields, pre, va, vb, X, Y, st);
}

int ldsv_ensure_fluxblock(ldsv_handle* h) {
  if (h->fb_fields) return LDSV_OK;
  void* p = nullptr;
  LDSV_TRY(ldsv_alloc(h, &p, (size_t)16 * h->nstate * sizeof(float), "flux-block fields"));
  h->fb_fields = (float*)p;
  h->fb_gfields = h->fb_fields + 8 * h->nstate;
  return LDSV_OK;
}

int ldsv_internal_step_fb(ldsv_handle* h, const ldsv_params* p, const FluxBlockArgs* fb,
                          const void* su, const void* sv, void* du, void* dv, hipStream_t st);

extern "C" {

int ldsv_fno_forward(ldsv_handle* h, const ldsv_fluxnet* net, const float* u, const float* v,
                     float* fields, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(u && v && fields, LDSV_EINVAL, "fno_forward: null array");
  return ldsv_launch_fno_forward(h, net, u, v, fields, false, (hipStream_t)stream);
}

int ldsv_fluxblock_fv_step(ldsv_handle* h, const ldsv_params* prm, const float* stencil_w,
                           const float* fields, const void* u_in, const void* v_in, void* u_out,
                           void* v_out, int nsteps, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && stencil_w && u_in && v_in && u_out && v_out, LDSV_EINVAL,
               "fluxblock_fv_step: null argument");
  LDSV_REQUIRE(nsteps >= 1, LDSV_EINVAL, "fluxblock_fv_step: nsteps=%d", nsteps);
  LDSV_REQUIRE(h->g.layout == LDSV_MAC && prm->rk == LDSV_RK4, LDSV_EDTYPE,
               "fluxblock_fv_step: RK4 on the MAC layout");
  FluxBlockArgs fb;
  fb.w = stencil_w;
  fb.f = fields;
  fb.fbs = (size_t)8 * h->ncell;
  const hipStream_t st = (hipStream_t)stream;
  for (int k = 0; k < nsteps; ++k)
    LDSV_TRY(ldsv_internal_step_fb(h, prm, &fb, k ? u_out : u_in, k ? v_out : v_in, u_out, v_out,
                                   st));
  return LDSV_OK;
}

int ldsv_fluxblock_fv_step_bwd(ldsv_handle* h, const ldsv_params* prm, const float* stencil_w,
                               const float* fields, const void* u_in, const void* v_in,
                               const void* gu_out, const void* gv_out, void* gu_in, void* gv_in,
                               float* gstencil, float* gfields, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && stencil_w && u_in && v_in && gu_out && gv_out && gu_in && gv_in, LDSV_EINVAL,
               "fluxblock_fv_step_bwd: null argument");
  FluxBlockArgs fb;
  fb.w = stencil_w;
  fb.f = fields;
  fb.fbs = (size_t)8 * h->ncell;
  fb.gw = gstencil;
  fb.gf = gfields;
  fb.gfbs = (size_t)8 * h->ncell;
  return ldsv_step_bwd(h, prm, nullptr, 0, nullptr, 0, u_in, v_in, gu_out, gv_out, gu_in, gv_in,
                       (hipStream_t)stream, &fb);
}

int ldsv_fluxblock_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_fluxnet* net,
                        const float* u_in, const float* v_in, float* u_out, float* v_out,
                        float* fields_out, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && net && net->stencil_w && u_in && v_in && u_out && v_out, LDSV_EINVAL,
               "fluxblock_step: null argument");
  LDSV_REQUIRE(prm->rk == LDSV_RK4, LDSV_EDTYPE, "fluxblock_step: RK4");
  const hipStream_t st = (hipStream_t)stream;
  float* fields = fields_out;
  if (!fields) {
    LDSV_TRY(ldsv_ensure_fluxblock(h));
    fields = h->fb_fields;
  }
  LDSV_TRY(ldsv_launch_fno_forward(h, net, u_in, v_in, fields, false, st));
  FluxBlockArgs fb;
  fb.w = net->stencil_w;
  fb.f = fields;
  fb.fbs = (size_t)8 * h->ncell;
  return ldsv_internal_step_fb(h, prm, &fb, u_in, v_in, u_out, v_out, st);
}

}  // extern "C"
