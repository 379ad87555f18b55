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
//               the epilogue (the first layer's transform kernel writes v_0
//               for it).
// and after the last layer k_fno_proj writes the 4 fields of each network
// into the [B][8][Ny][Nx] field array (channels 4 g .. 4 g + 3; zeros for an
// absent network).  Everything is FP32; the FFT is O(N log N) on the vector
// ALU and the mixing is a few complex FMAs per mode, so these kernels are
// bound by their HBM traffic and LDS round trips, not by arithmetic.
#include <utility>

#include "adjoint.h"
#include "cnn_common.h"
#include "fft_lds.h"
#include "fft_reg.h"
#include "fno.h"
#include "stage.h"

namespace {

constexpr int kFnoBlock = 1024;  // largest transform workgroup
// transform workgroup for E values per thread: 512 threads for E = 8, else
// 1024.  Grids of up to 4096 cells run the forward transform with E = 8
// (every radix-8 butterfly of a stage has its thread and four workgroups
// share a CU: 9-11 % faster than E = 4) and the inverse, whose pointwise
// term and GELU need more registers, with E = 4 (E = 8 at two workgroups
// per CU was 18 % slower); larger grids use E = 16 for both.
template <int E>
__host__ __device__ constexpr int fno_block() {
  return E == 8 ? 512 : kFnoBlock;
}
template <int E>
constexpr int spec_e() {
  return E == 4 ? 8 : E;
}
constexpr int kMaxIn = 16;  // input planes of one FNO (two per state of a history)
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
  int nin, nout;             // input planes (2 per state) and output channels
  const float* xin[kMaxIn];  // input planes, each [B][Ny][Nx]
  float* out;                // output channel c of network g, trajectory b at
  size_t out_cs, out_bs;     //   out + (out_ch[g] + c) out_cs + b out_bs
  int out_ch[2];
};

__device__ __forceinline__ int retained_row(int ky, int ny, int M) {
  if (ky < M) return ky;
  if (ky >= ny - M) return ky - ny + 2 * M;
  return -1;
}

// (channel pair, trajectory, network slice) of a transform workgroup of the
// grid (C/2, B, nets), renumbered so that the pairs of one trajectory run
// on one XCD: they all read that trajectory's input (every channel for the
// pointwise term, or u and v), which then comes from that XCD's L2 once
// instead of once per XCD
__device__ __forceinline__ void pair_of_block(int& p, int& b, int& z) {
  const int np = gridDim.x, nb = gridDim.y;
  const int lid = blockIdx.x + np * (blockIdx.y + nb * blockIdx.z);
  const int r = xcd_contiguous(lid, np * nb * gridDim.z);
  p = r % np;
  const int rest = r / np;
  b = rest % nb;
  z = rest / nb;
}

template <int E>
__device__ __forceinline__ void load_twiddles(Cx<float>* Wx, Cx<float>* Wy, const Cx<float>* twx,
                                              const Cx<float>* twy, int nx, int ny) {
  for (int e = threadIdx.x; e < nx; e += blockDim.x) Wx[e] = twx[e];
  for (int e = threadIdx.x; e < ny; e += blockDim.x) Wy[e] = twy[e];
}

// forward transform of channels (2p, 2p+1) of trajectory b, network slice z
template <int E, bool LIFT>
__global__ void __launch_bounds__(fno_block<E>()) k_fno_spec(const float* __restrict__ vin,
                                                        const float* __restrict__ vin2, FnoArgs a,
                                                        float* __restrict__ v0out,
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
  int p, b, z;
  pair_of_block(p, b, z);
  const int g = a.net[z];
  const int c0 = 2 * p, c1 = 2 * p + 1;
  const int n = nx * ny;
  if constexpr (LIFT) {
    const float* lw = a.lift_w[g];
    const float* lb = a.lift_b[g];
    const int nin = a.nin;
    const float b0 = lb[c0], b1 = lb[c1];
    float* d0 = v0out + ((size_t)(z * B + b) * C + c0) * n;
    float q0[E], q1[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      q0[k] = b0;
      q1[k] = b1;
    }
    for (int j = 0; j < nin; ++j) {
      const float* x = a.xin[j] + (size_t)b * n;
      const float w0 = lw[c0 * nin + j], w1 = lw[c1 * nin + j];
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int t = k * fno_block<E>() + (int)threadIdx.x;
        if (t < n) {
          const float xv = x[t];
          q0[k] += w0 * xv;
          q1[k] += w1 * xv;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * fno_block<E>() + (int)threadIdx.x;
      if (t < n) {
        A[t] = Cx<float>{q0[k], q1[k]};
        d0[t] = q0[k];  // v_0 kept for the pointwise term and the backward
        d0[n + t] = q1[k];
      }
    }
  } else {
    const float* s0 = vin + ((size_t)(z * B + b) * C + c0) * n;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int t = k * fno_block<E>() + (int)threadIdx.x;
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

// The same forward transform for square FP32 grids of 2^LOGN x 2^LOGN cells
// (64^2) on the compile-time transforms of fft_reg.h, one thread per radix-8
// butterfly: the columns first, so that the inputs (or the lift of the
// inputs) load straight into the first stage with each row of the field
// read across lanes; an LDS transpose into the row transform; the retained
// modes unpacked from the row transform's results through LDS.
template <int LOGN, bool LIFT>
__global__ void __launch_bounds__((1 << (2 * LOGN)) / 8) k_fno_spec_r(
    const float* __restrict__ vin, FnoArgs a, float* __restrict__ v0out, c32* __restrict__ X,
    const Cx<float>* __restrict__ tw, int C, int M, int B) {
  constexpr int N = 1 << LOGN, BLOCK = (N * N) / 8, S = fftreg::plan_stages(LOGN);
  constexpr int LR0 = fftreg::plan_lr(LOGN, 0), LRL = fftreg::plan_lr(LOGN, S - 1);
  constexpr int R0 = 1 << LR0, RL = 1 << LRL;
  constexpr int kE1 = fftreg::lds_elems<true, LOGN, LOGN>();
  constexpr int kE2 = fftreg::lds_elems<false, LOGN, LOGN>();
  __shared__ Cx<float> A[kE1 > kE2 ? kE1 : kE2];
  __shared__ Cx<float> W[N];
  for (int e = threadIdx.x; e < N; e += BLOCK) W[e] = tw[e];
  int p, b, z;
  pair_of_block(p, b, z);
  const int g = a.net[z];
  const int c0 = 2 * p, c1 = 2 * p + 1;
  constexpr int n = N * N;
  Cx<float> x[8];
  if constexpr (LIFT) {
    const float* lw = a.lift_w[g];
    const int nin = a.nin;
    float q0[8], q1[8];
    const float b0 = a.lift_b[g][c0], b1 = a.lift_b[g][c1];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      q0[e] = b0;
      q1[e] = b1;
    }
    for (int j = 0; j < nin; ++j) {
      const float* xj = a.xin[j] + (size_t)b * n;
      const float w0 = lw[c0 * nin + j], w1 = lw[c1 * nin + j];
#pragma unroll
      for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          int t, y;
          fftreg::point<false, LOGN, LOGN, BLOCK, LR0>(q, r, t, y);
          const float xv = xj[y * N + t];
          q0[q * R0 + r] += w0 * xv;
          q1[q * R0 + r] += w1 * xv;
        }
    }
    float* d0 = v0out + ((size_t)(z * B + b) * C + c0) * n;
#pragma unroll
    for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        int t, y;
        fftreg::point<false, LOGN, LOGN, BLOCK, LR0>(q, r, t, y);
        const int e = q * R0 + r;
        d0[y * N + t] = q0[e];  // v_0 kept for the pointwise term and the backward
        d0[n + y * N + t] = q1[e];
        x[e] = Cx<float>{q0[e], q1[e]};
      }
  } else {
    const float* s0 = vin + ((size_t)(z * B + b) * C + c0) * n;
#pragma unroll
    for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        int t, y;
        fftreg::point<false, LOGN, LOGN, BLOCK, LR0>(q, r, t, y);
        x[q * R0 + r] = Cx<float>{s0[y * N + t], s0[n + y * N + t]};
      }
  }
  __syncthreads();
  // along y (column t, then row ky = the last stage's point)
  fftreg::run<false, LOGN, LOGN, BLOCK, -1, false>(x, A, W);
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int t, ky;
      fftreg::point<false, LOGN, LOGN, BLOCK, LRL>(q, r, t, ky);
      A[fftreg::lds_at<true, LOGN, LOGN>(t, ky)] = x[q * RL + r];
    }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int ky, i;
      fftreg::point<true, LOGN, LOGN, BLOCK, LR0>(q, r, ky, i);
      x[q * R0 + r] = A[fftreg::lds_at<true, LOGN, LOGN>(i, ky)];
    }
  __syncthreads();
  // along x
  fftreg::run<true, LOGN, LOGN, BLOCK, -1, false>(x, A, W);
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int ky, kx;
      fftreg::point<true, LOGN, LOGN, BLOCK, LRL>(q, r, ky, kx);
      A[fftreg::lds_at<true, LOGN, LOGN>(kx, ky)] = x[q * RL + r];
    }
  __syncthreads();
  // Z = V0 + i V1 with V0, V1 the transforms of the two real channels:
  // V0(k) = (Z(k) + conj Z(-k)) / 2, V1(k) = (Z(k) - conj Z(-k)) / (2 i)
  const int nm = 2 * M * M;
  c32* X0 = X + ((size_t)(z * B + b) * C + c0) * nm;
  c32* X1 = X0 + nm;
  for (int e = threadIdx.x; e < nm; e += BLOCK) {
    const int r = e / M, kx = e - r * M;
    const int ky = r < M ? r : N - 2 * M + r;
    const Cx<float> z1 = A[fftreg::lds_at<true, LOGN, LOGN>(kx, ky)];
    const Cx<float> z2 = A[fftreg::lds_at<true, LOGN, LOGN>((N - kx) & (N - 1), (N - ky) & (N - 1))];
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

// inverse transform of output channels (2p, 2p+1) + pointwise term + GELU.
// The weights of the pair are read once into registers; every spectrum
// load of a thread is issued before the LDS stores, and the pointwise sum
// over the C input channels is unrolled so its loads are in flight together.
// MODE 0: forward layer, out = GELU(z) with z = K v + W v + b (z kept in
// zout when given); 1: last forward layer, out = z; 2: backward, the pair
// are input channels i: dv_i = (K^T dz)_i + sum_o W[o][i] dz_o, out =
// dv_i GELU'(gpre_i) (the cotangent of the previous layer's pre-activation);
// 3: backward of the first layer, out = dv_i.
template <int E, int C, int MODE>
__global__ void __launch_bounds__(fno_block<E>(), E <= 4 ? 8 : 4) k_fno_inv(const c32* __restrict__ Y,
                                                       const float* __restrict__ vin, FnoArgs a,
                                                       float* __restrict__ vout,
                                                       float* __restrict__ zout,
                                                       const float* __restrict__ gpre,
                                                       const Cx<float>* __restrict__ twx,
                                                       const Cx<float>* __restrict__ twy, int nx,
                                                       int ny, int log2nx, int log2ny, int M,
                                                       int B) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  Cx<float>* A = reinterpret_cast<Cx<float>*>(smem_raw);
  Cx<float>* Wx = A + nx * ny;
  Cx<float>* Wy = Wx + nx;
  load_twiddles<E>(Wx, Wy, twx, twy, nx, ny);
  int p, b, z;
  pair_of_block(p, b, z);
  const int g = a.net[z];
  const int o0 = 2 * p, o1 = 2 * p + 1;
  const int n = nx * ny;
  const int nm = 2 * M * M;
  const c32* Y0 = Y + ((size_t)(z * B + b) * C + o0) * nm;
  const c32* Y1 = Y0 + nm;
  // weights of the two outputs (and the lift for the first layer)
  constexpr bool BWD = MODE >= 2;
  // the pointwise weights of the pair in LDS (read back four at a time)
  __shared__ __attribute__((aligned(16))) float sw[2][C];
  if (threadIdx.x < 2 * C) {
    const float* pw = a.point_w[g];
    const int q = threadIdx.x >> (C == 16 ? 4 : 3), i = threadIdx.x & (C - 1);
    const int oq = q ? o1 : o0;
    sw[q][i] = BWD ? pw[i * C + oq] : pw[oq * C + i];
  }
  const float bo0 = BWD ? 0.f : a.point_b[g][o0], bo1 = BWD ? 0.f : a.point_b[g][o1];
  // Hermitian extension: element (ky, kx) takes Y(r, kx) directly for
  // 0 < kx < M, conj Y(r', nx - kx) at the mirrored row for kx > nx - M, and
  // the symmetrised pair (Y(r, 0) + conj Y(r', 0)) / 2 in the k_x = 0 column
  // groups of 4 elements per thread: their loads are in flight together
  // without holding all E in registers
  constexpr int kG = E < 4 ? E : 4;
#pragma unroll
  for (int g0 = 0; g0 < E; g0 += kG) {
  c32 ya0[kG], ya1[kG], yb0[kG], yb1[kG];
#pragma unroll
  for (int kk = 0; kk < kG; ++kk) {
    const int k = g0 + kk;
    const int t = k * fno_block<E>() + (int)threadIdx.x;
    ya0[kk] = ya1[kk] = yb0[kk] = yb1[kk] = c32{0.f, 0.f};
    if (t < n) {
      const int ky = t >> log2nx, kx = t & (nx - 1);
      const int r = retained_row(ky, ny, M);
      const int rm = retained_row((ny - ky) & (ny - 1), ny, M);
      int ia = -1, ib = -1;
      if (kx == 0) {
        ia = r >= 0 ? r * M : -1;
        ib = rm >= 0 ? rm * M : -1;
      } else if (kx < M) {
        ia = r >= 0 ? r * M + kx : -1;
      } else if (kx > nx - M) {
        ib = rm >= 0 ? rm * M + (nx - kx) : -1;
      }
      if (ia >= 0) {
        ya0[kk] = Y0[ia];
        ya1[kk] = Y1[ia];
      }
      if (ib >= 0) {
        yb0[kk] = Y0[ib];
        yb1[kk] = Y1[ib];
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < kG; ++kk) {
    const int t = (g0 + kk) * fno_block<E>() + (int)threadIdx.x;
    if (t < n) {
      // s = ya + conj(yb) (one of the two is zero outside the k_x = 0 column)
      const float h = (t & (nx - 1)) == 0 ? 0.5f : 1.0f;
      const float s0x = h * (ya0[kk].x + yb0[kk].x), s0y = h * (ya0[kk].y - yb0[kk].y);
      const float s1x = h * (ya1[kk].x + yb1[kk].x), s1y = h * (ya1[kk].y - yb1[kk].y);
      A[t] = Cx<float>{s0x - s1y, s0y + s1x};
    }
  }
  }
  __syncthreads();
  lds_fft<float, E>(A, nx, log2nx, ny, nx, 1, +1, Wx);
  lds_fft<float, E>(A, ny, log2ny, nx, 1, nx, +1, Wy);
  const float sc = 1.0f / (float)n;
  float* d0 = vout + ((size_t)(z * B + b) * C + o0) * n;
  float* e0 = zout ? zout + ((size_t)(z * B + b) * C + o0) * n : nullptr;
  // the pointwise term over quads of consecutive pixels: every input-channel
  // read, output store and spectrum read is 16 bytes per lane
  static_assert(E % 4 == 0, "pixel quads");
  const float* srcb = vin + (size_t)(z * B + b) * C * n;
  for (int k = 0; k < E / 4; ++k) {
    const int q = k * fno_block<E>() + (int)threadIdx.x;
    const int t = 4 * q;
    if (t >= n) break;
    float z0[4], z1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      z0[j] = A[t + j].x * sc + bo0;
      z1[j] = A[t + j].y * sc + bo1;
    }
#pragma unroll
    for (int c0 = 0; c0 < C; c0 += 4) {
      float4 vi[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) vi[i] = *reinterpret_cast<const float4*>(srcb + (size_t)(c0 + i) * n + t);
      const float4 a0 = *reinterpret_cast<const float4*>(&sw[0][c0]);
      const float4 a1 = *reinterpret_cast<const float4*>(&sw[1][c0]);
      const float w0[4] = {a0.x, a0.y, a0.z, a0.w}, w1[4] = {a1.x, a1.y, a1.z, a1.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        z0[0] += w0[i] * vi[i].x;
        z0[1] += w0[i] * vi[i].y;
        z0[2] += w0[i] * vi[i].z;
        z0[3] += w0[i] * vi[i].w;
        z1[0] += w1[i] * vi[i].x;
        z1[1] += w1[i] * vi[i].y;
        z1[2] += w1[i] * vi[i].z;
        z1[3] += w1[i] * vi[i].w;
      }
    }
    float h0[4], h1[4];
    if constexpr (MODE == 0 || MODE == 1) {
      if (e0) {
        *reinterpret_cast<float4*>(e0 + t) = float4{z0[0], z0[1], z0[2], z0[3]};
        *reinterpret_cast<float4*>(e0 + n + t) = float4{z1[0], z1[1], z1[2], z1[3]};
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        h0[j] = MODE == 1 ? z0[j] : cnnk::gelu_exact(z0[j]);
        h1[j] = MODE == 1 ? z1[j] : cnnk::gelu_exact(z1[j]);
      }
    } else if constexpr (MODE == 2) {
      const float* gp = gpre + ((size_t)(z * B + b) * C + o0) * n;
      const float4 g0 = *reinterpret_cast<const float4*>(gp + t);
      const float4 g1 = *reinterpret_cast<const float4*>(gp + n + t);
      const float gg0[4] = {g0.x, g0.y, g0.z, g0.w}, gg1[4] = {g1.x, g1.y, g1.z, g1.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        h0[j] = z0[j] * cnnk::gelu_grad(gg0[j]);
        h1[j] = z1[j] * cnnk::gelu_grad(gg1[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        h0[j] = z0[j];
        h1[j] = z1[j];
      }
    }
    *reinterpret_cast<float4*>(d0 + t) = float4{h0[0], h0[1], h0[2], h0[3]};
    *reinterpret_cast<float4*>(d0 + n + t) = float4{h1[0], h1[1], h1[2], h1[3]};
  }
}

// The forward-mode inverse (MODE 0 and 1 of k_fno_inv) for square FP32
// grids of 2^LOGN x 2^LOGN cells (64^2) on the compile-time transforms: the
// Hermitian-extended spectrum of the pair is formed straight into the first
// stage of the inverse transform along x (rows), an LDS transpose feeds the
// inverse transform along y (columns), whose last stage leaves each row of
// the field across lanes for the pointwise term, GELU and the stores.
template <int LOGN, int C, int MODE>
__global__ void __launch_bounds__((1 << (2 * LOGN)) / 8) k_fno_inv_r(
    const c32* __restrict__ Y, const float* __restrict__ vin, FnoArgs a, float* __restrict__ vout,
    float* __restrict__ zout, const Cx<float>* __restrict__ tw, int M, int B) {
  static_assert(MODE == 0 || MODE == 1, "forward modes");
  constexpr int N = 1 << LOGN, BLOCK = (N * N) / 8, S = fftreg::plan_stages(LOGN);
  constexpr int LR0 = fftreg::plan_lr(LOGN, 0), LRL = fftreg::plan_lr(LOGN, S - 1);
  constexpr int R0 = 1 << LR0, RL = 1 << LRL;
  constexpr int kE1 = fftreg::lds_elems<true, LOGN, LOGN>();
  constexpr int kE2 = fftreg::lds_elems<false, LOGN, LOGN>();
  __shared__ Cx<float> A[kE1 > kE2 ? kE1 : kE2];
  __shared__ Cx<float> W[N];
  __shared__ __attribute__((aligned(16))) float sw[2][C];
  for (int e = threadIdx.x; e < N; e += BLOCK) W[e] = tw[e];
  int p, b, z;
  pair_of_block(p, b, z);
  const int g = a.net[z];
  const int o0 = 2 * p, o1 = 2 * p + 1;
  constexpr int n = N * N;
  const int nm = 2 * M * M;
  if (threadIdx.x < 2 * C) {
    const float* pw = a.point_w[g];
    const int q = threadIdx.x / C, i = threadIdx.x % C;
    sw[q][i] = pw[(q ? o1 : o0) * C + i];
  }
  const float bo0 = a.point_b[g][o0], bo1 = a.point_b[g][o1];
  const c32* Y0 = Y + ((size_t)(z * B + b) * C + o0) * nm;
  const c32* Y1 = Y0 + nm;
  // Hermitian extension at the first inverse stage's points (row ky, column
  // kx): Y(r, kx) for 0 < kx < M, conj Y(r', N - kx) of the mirrored row for
  // kx > N - M, (Y(r, 0) + conj Y(r', 0)) / 2 at kx = 0, zero elsewhere
  Cx<float> x[8];
  {
    c32 ya0[8], ya1[8], yb0[8], yb1[8];
#pragma unroll
    for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        int ky, kx;
        fftreg::point<true, LOGN, LOGN, BLOCK, LRL>(q, r, ky, kx);
        const int e = q * RL + r;
        const int rr = retained_row(ky, N, M);
        const int rm = retained_row((N - ky) & (N - 1), N, M);
        int ia = -1, ib = -1;
        if (kx == 0) {
          ia = rr >= 0 ? rr * M : -1;
          ib = rm >= 0 ? rm * M : -1;
        } else if (kx < M) {
          ia = rr >= 0 ? rr * M + kx : -1;
        } else if (kx > N - M) {
          ib = rm >= 0 ? rm * M + (N - kx) : -1;
        }
        ya0[e] = ya1[e] = yb0[e] = yb1[e] = c32{0.f, 0.f};
        if (ia >= 0) {
          ya0[e] = Y0[ia];
          ya1[e] = Y1[ia];
        }
        if (ib >= 0) {
          yb0[e] = Y0[ib];
          yb1[e] = Y1[ib];
        }
      }
#pragma unroll
    for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        int ky, kx;
        fftreg::point<true, LOGN, LOGN, BLOCK, LRL>(q, r, ky, kx);
        const int e = q * RL + r;
        // s = ya + conj(yb) (one of the two is zero outside the kx = 0 column)
        const float h = kx == 0 ? 0.5f : 1.0f;
        const float s0x = h * (ya0[e].x + yb0[e].x), s0y = h * (ya0[e].y - yb0[e].y);
        const float s1x = h * (ya1[e].x + yb1[e].x), s1y = h * (ya1[e].y - yb1[e].y);
        x[e] = Cx<float>{s0x - s1y, s0y + s1x};
      }
  }
  __syncthreads();
  // along x (rows), the stages in reverse order
  fftreg::run<true, LOGN, LOGN, BLOCK, +1, true>(x, A, W);
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int ky, xx;
      fftreg::point<true, LOGN, LOGN, BLOCK, LR0>(q, r, ky, xx);
      A[fftreg::lds_at<false, LOGN, LOGN>(ky, xx)] = x[q * R0 + r];
    }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int xx, ky;
      fftreg::point<false, LOGN, LOGN, BLOCK, LRL>(q, r, xx, ky);
      x[q * RL + r] = A[fftreg::lds_at<false, LOGN, LOGN>(ky, xx)];
    }
  __syncthreads();
  // along y (columns): the outputs land at (column xx, row y), each row of
  // the field across consecutive lanes
  fftreg::run<false, LOGN, LOGN, BLOCK, +1, true>(x, A, W);
  const float sc = 1.0f / (float)n;
  const float* src = vin + (size_t)(z * B + b) * C * n;
  float* d0 = vout + ((size_t)(z * B + b) * C + o0) * n;
  float* e0 = zout ? zout + ((size_t)(z * B + b) * C + o0) * n : nullptr;
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int xx, y;
      fftreg::point<false, LOGN, LOGN, BLOCK, LR0>(q, r, xx, y);
      const int e = q * R0 + r;
      const int t = y * N + xx;
      float z0 = x[e].x * sc + bo0, z1 = x[e].y * sc + bo1;
#pragma unroll
      for (int c0 = 0; c0 < C; c0 += 4) {
        float vi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) vi[i] = src[(size_t)(c0 + i) * n + t];
        const float4 a0 = *reinterpret_cast<const float4*>(&sw[0][c0]);
        const float4 a1 = *reinterpret_cast<const float4*>(&sw[1][c0]);
        z0 += a0.x * vi[0] + a0.y * vi[1] + a0.z * vi[2] + a0.w * vi[3];
        z1 += a1.x * vi[0] + a1.y * vi[1] + a1.z * vi[2] + a1.w * vi[3];
      }
      if (e0) {
        e0[t] = z0;
        e0[n + t] = z1;
      }
      d0[t] = MODE == 1 ? z0 : cnnk::gelu_exact(z0);
      d0[n + t] = MODE == 1 ? z1 : cnnk::gelu_exact(z1);
    }
}

// output channel K of network g = Q_g v_L + b_Q (zeros for an absent
// network), K < nout <= 4
__global__ void __launch_bounds__(kBlock) k_fno_proj(const float* __restrict__ vL, FnoArgs a,
                                                     int n, int C, int B) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y, g = blockIdx.z;
  if (t >= n) return;
  const int z = a.slot[g];
  const int nout = a.nout;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  if (z >= 0) {
    const float* qw = a.proj_w[g];
    const float* qb = a.proj_b[g];
    const float* s = vL + (size_t)(z * B + b) * C * n + t;
#pragma unroll
    for (int K = 0; K < 4; ++K) acc[K] = K < nout ? qb[K] : 0.f;
    for (int c = 0; c < C; ++c) {
      const float vc = s[(size_t)c * n];
#pragma unroll
      for (int K = 0; K < 4; ++K)
        if (K < nout) acc[K] += qw[K * C + c] * vc;
    }
  }
#pragma unroll
  for (int K = 0; K < 4; ++K)
    if (K < nout) a.out[(size_t)(a.out_ch[g] + K) * a.out_cs + (size_t)b * a.out_bs + t] = acc[K];
}

// ---------------------------------------------------------------- backward
//
// With the saved pre-activations z_l, spectra X_l = F(v_l) and v_0:
//   dv_L = Q^T dF;  dQ = sum dF v_L^T;  db_Q = sum dF            (k_fno_proj_bwd)
//   layer l = L-1 .. 0, dz_l the cotangent of z_l:
//     dW_l = sum dz_l v_l^T, db_l = sum dz_l                     (k_fno_wgrad)
//     dR_l(k)[i][o] = (w(k_x) / N) sum_b conj(X_l,i(k)) DZ_o(k)  (k_fno_dR)
//        with DZ = F(dz_l) (k_fno_spec), w = 1 at k_x = 0 else 2:
//        d/dRe + i d/dIm of the loss, the gradient convention of a real
//        loss in a complex parameter that torch uses
//     dv_l = K_l^T dz_l + W_l^T dz_l, where K^T is the spectral
//        convolution with weights conj(R[i][o]) (k_fno_mix<CONJ_T>, then
//        k_fno_inv in backward mode); dz_{l-1} = dv_l GELU'(z_{l-1})
//   dP = sum dv_0 x^T, db_P = sum dv_0, dx = P^T dv_0 summed over the two
//   networks                                                        (k_fno_lift_bwd)
// Every parameter gradient is a sum over trajectories and pixels: each
// block writes its partial sums (wave shuffles, then the waves in a fixed
// order) and k_sum_partials adds them over the blocks in a fixed order, so
// the result is deterministic.

// sum of v over the block (blockDim == kBlock), returned to every thread of
// wave 0's lane 0... written to dst[j] by thread j for j < NV
template <int NV>
__device__ __forceinline__ void block_sums(float (&v)[NV], float* __restrict__ dst,
                                           int stride = 1) {
  __shared__ float red[kBlock / 64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // a previous call's readers are done with red
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    float x = v[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[wave][j] = x;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NV; j += blockDim.x) {
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) acc += red[q][j];
    dst[(size_t)j * stride] = acc;
  }
}

// dv_L[c] = sum_K Q[K][c] dF_K with dF the output cotangent (addressed like
// the output, base gout); partials of dQ[K][c] = dF_K v_L[c] and
// db_Q[K] = dF_K: part[z][b][blk][NOUT C + NOUT]
template <int C, int NOUT>
__global__ void __launch_bounds__(kBlock) k_fno_proj_bwd(const float* __restrict__ gout,
                                                         const float* __restrict__ vL, FnoArgs a,
                                                         float* __restrict__ dv,
                                                         float* __restrict__ part, int n, int B) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y, z = blockIdx.z, g = a.net[z];
  const bool in = t < n;
  float dF[NOUT];
#pragma unroll
  for (int K = 0; K < NOUT; ++K)
    dF[K] = in ? gout[(size_t)(a.out_ch[g] + K) * a.out_cs + (size_t)b * a.out_bs + t] : 0.f;
  const float* qw = a.proj_w[g];
  float prod[NOUT * C + NOUT];
  const size_t base = (size_t)(z * B + b) * C * n;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float x = in ? vL[base + (size_t)c * n + t] : 0.f;
    float d = 0.f;
#pragma unroll
    for (int K = 0; K < NOUT; ++K) {
      d += qw[K * C + c] * dF[K];
      prod[K * C + c] = dF[K] * x;
    }
    if (in) dv[base + (size_t)c * n + t] = d;
  }
#pragma unroll
  for (int K = 0; K < NOUT; ++K) prod[NOUT * C + K] = dF[K];
  block_sums<NOUT * C + NOUT>(
      prod, part + (((size_t)z * B + b) * gridDim.x + blockIdx.x) * (NOUT * C + NOUT));
}

// partials of dW[o][i] = sum dz_o v_i and db[o] = sum dz_o over a chunk of
// kWChunk pixels of one (network, trajectory): part[z][b][chunk][C C + C].
// v_i = GELU(vpre_i) when GELU_V (v_l for l >= 1 from the saved z_{l-1}),
// else vpre itself (v_0).  Grid (chunks, nnet B); block C*C: thread (o, i).
constexpr int kWChunk = 256;
template <int C, bool GELU_V>
__global__ void __launch_bounds__(C * C) k_fno_wgrad(const float* __restrict__ dz,
                                                     const float* __restrict__ vpre,
                                                     float* __restrict__ part, int n, int B) {
  constexpr int kT = 64;          // pixels per tile
  constexpr int kS = kT + 4;      // padded row (16-byte aligned, spreads banks)
  constexpr int kPer = kT / C;    // tile values per thread and operand
  __shared__ __attribute__((aligned(16))) float sdz[C][kS];
  __shared__ __attribute__((aligned(16))) float sv[C][kS];
  const int zb = blockIdx.y;      // z * B + b
  const int o = threadIdx.x / C, i = threadIdx.x % C;
  const float* d = dz + (size_t)zb * C * n;
  const float* vp = vpre + (size_t)zb * C * n;
  float acc = 0.f, accb = 0.f;
  const int pbeg = blockIdx.x * kWChunk;
  const int pend = min(n, (int)(blockIdx.x + 1) * kWChunk);
  // a tile's operands through registers (all loads in flight together), the
  // next tile's loads issued before the current tile's products
  float dv[kPer], xv[kPer];
  auto load = [&](int p0) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = k * C * C + (int)threadIdx.x;
      const int c = e / kT, q = e % kT;
      dv[k] = d[(size_t)c * n + p0 + q];
      xv[k] = vp[(size_t)c * n + p0 + q];
    }
  };
  if (pbeg < pend) load(pbeg);
  for (int p0 = pbeg; p0 < pend; p0 += kT) {
    __syncthreads();  // the previous tile's products are done
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = k * C * C + (int)threadIdx.x;
      const int c = e / kT, q = e % kT;
      sdz[c][q] = dv[k];
      sv[c][q] = GELU_V ? cnnk::gelu_exact(xv[k]) : xv[k];
    }
    __syncthreads();
    if (p0 + kT < pend) load(p0 + kT);
#pragma unroll 4
    for (int q = 0; q < kT; q += 4) {
      const float4 dd = *reinterpret_cast<const float4*>(&sdz[o][q]);
      const float4 vv = *reinterpret_cast<const float4*>(&sv[i][q]);
      acc += dd.x * vv.x + dd.y * vv.y + dd.z * vv.z + dd.w * vv.w;
      accb += dd.x + dd.y + dd.z + dd.w;
    }
  }
  float* dst = part + ((size_t)zb * gridDim.x + blockIdx.x) * (C * C + C);
  dst[o * C + i] = acc;
  if (i == 0) dst[C * C + o] = accb;
}

// partial spectral weight gradients over the trajectories of b-group
// blockIdx.y: part[z][group][i][o][m] (complex, scaled by w(k_x) / N).
// Block 64 x C: lane = mode, wave = output channel o; the X_l tile of each
// trajectory streams through LDS as in k_fno_mix.
template <int C>
__global__ void __launch_bounds__(64 * C) k_fno_dR(const c32* __restrict__ Xl,
                                                   const c32* __restrict__ DZ, c32* __restrict__ part,
                                                   int B, int nm, int M, int bpg, float inv_n) {
  __shared__ c32 xs[2][C][64];
  const int lane = threadIdx.x & 63;
  const int o = threadIdx.x >> 6;
  const int m = blockIdx.x * 64 + lane;
  const int z = blockIdx.z;
  c32 acc[C];
#pragma unroll
  for (int i = 0; i < C; ++i) acc[i] = c32{0.f, 0.f};
  const int b0 = blockIdx.y * bpg;
  const int b1 = min(B, b0 + bpg);
  for (int b = b0; b < b1; ++b) {
    const int buf = (b - b0) & 1;
    {
      const int i = threadIdx.x >> 6;
      xs[buf][i][lane] = m < nm ? Xl[((size_t)(z * B + b) * C + i) * nm + m] : c32{0.f, 0.f};
    }
    const c32 d = m < nm ? DZ[((size_t)(z * B + b) * C + o) * nm + m] : c32{0.f, 0.f};
    __syncthreads();
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const c32 x = xs[buf][i][lane];
      // conj(x) d
      acc[i].x += x.x * d.x + x.y * d.y;
      acc[i].y += x.x * d.y - x.y * d.x;
    }
  }
  if (m < nm) {
    const float sc = ((m % M) == 0 ? 1.f : 2.f) * inv_n;
    c32* dst = part + ((size_t)z * gridDim.y + blockIdx.y) * C * C * nm;
#pragma unroll
    for (int i = 0; i < C; ++i)
      dst[((size_t)i * C + o) * nm + m] = c32{sc * acc[i].x, sc * acc[i].y};
  }
}

struct GradIn {
  float* gx[kMaxIn];  // cotangents of the input planes (all null: not wanted)
};

// dx_j = sum over the networks of (P^T dv_0)_j (written or added to gx[j])
// and partials of dP[c][j] = dv_0,c x_j, db_P[c] = dv_0,c:
// part[z][b][blk][(nin + 1) C], dP in the [C][nin] order of the weights
template <int C>
__global__ void __launch_bounds__(kBlock) k_fno_lift_bwd(const float* __restrict__ dv0,
                                                         FnoArgs a, int nnet, GradIn gi,
                                                         int accumulate, float* __restrict__ part,
                                                         int n, int B) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y;
  const bool in = t < n;
  const int nin = a.nin;
  const size_t q = (size_t)b * n + t;
  float gx[kMaxIn];
#pragma unroll
  for (int j = 0; j < kMaxIn; ++j) gx[j] = 0.f;
  for (int z = 0; z < nnet; ++z) {
    const float* lw = a.lift_w[a.net[z]];
    const float* d = dv0 + (size_t)(z * B + b) * C * n;
    float dc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) dc[c] = in ? d[(size_t)c * n + t] : 0.f;
    float* dst = part + (((size_t)z * B + b) * gridDim.x + blockIdx.x) * ((nin + 1) * C);
#pragma unroll
    for (int j = 0; j < kMaxIn; ++j) {
      if (j >= nin) break;
      const float xj = in ? a.xin[j][q] : 0.f;
      float prod[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        gx[j] += lw[c * nin + j] * dc[c];
        prod[c] = dc[c] * xj;
      }
      block_sums<C>(prod, dst + j, nin);
    }
    block_sums<C>(dc, dst + nin * C);
  }
  if (in && gi.gx[0]) {
#pragma unroll
    for (int j = 0; j < kMaxIn; ++j) {
      if (j >= nin) break;
      float* o = gi.gx[j];
      o[q] = accumulate ? o[q] + gx[j] : gx[j];
    }
  }
}

struct PartOut {
  float* out[2];  // destination of network slice z (accumulated)
};

// out_z[j] += sum over blk of part[(z nblk + blk) stride + off + j]: eight
// interleaved running sums (blk mod 8, so eight loads are in flight) added
// in a fixed order at the end
template <int S>
__global__ void __launch_bounds__(kBlock) k_sum_partials(const float* __restrict__ part, int nblk,
                                                         size_t stride, int off, int len,
                                                         PartOut po) {
  // S threads share an output (short outputs over many partials): thread s
  // takes the partials s, s + S, ... eight at a time, the S sums are added
  // in order through LDS
  constexpr int kO = kBlock / S;
  __shared__ float red[S][kO];
  const int jo = threadIdx.x % kO, sp = threadIdx.x / kO;
  const int j = blockIdx.x * kO + jo;
  const int z = blockIdx.z;
  float t = 0.f;
  if (j < len) {
    const float* p = part + (size_t)z * nblk * stride + off + j;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int k = sp;
    for (; k + 7 * S < nblk; k += 8 * S) {
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += p[(size_t)(k + q * S) * stride];
    }
    for (int q = 0; k < nblk; k += S, ++q) acc[q & 7] += p[(size_t)k * stride];
    t = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  if constexpr (S == 1) {
    if (j < len) po.out[z][j] += t;
  } else {
    red[sp][jo] = t;
    __syncthreads();
    if (sp == 0 && j < len) {
      float r = 0.f;
#pragma unroll
      for (int q = 0; q < S; ++q) r += red[q][jo];
      po.out[z][j] += r;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_fill_zero(float* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    p[i] = 0.f;
}

// ---------------------------------------------------------------- host

struct FnoShape {
  int C, L, M, nnet;
};

// One or two FNOs run side by side (grid.z = network) on the same input
// planes, each writing nout output channels: the flux block's pair (inputs
// u, v; 4 fields each) or the temporal correction (inputs the history
// states; 2 channels).
struct FnoGroup {
  const ldsv_fno* f[2];
  int ngrid;                 // networks the output covers (absent ones write zeros)
  int nin, nout;
  const float* xin[kMaxIn];
  float* out;
  size_t out_cs, out_bs;
  int out_ch[2];
};

int check_group(const ldsv_handle* h, const FnoGroup& G, FnoShape* sh) {
  LDSV_REQUIRE(h->g.dtype == LDSV_F32 && h->g.layout == LDSV_MAC, LDSV_EDTYPE,
               "flux block: the FNO needs an F32 MAC grid");
  sh->nnet = 0;
  sh->C = sh->L = sh->M = 0;
  for (int g = 0; g < G.ngrid; ++g) {
    const ldsv_fno* f = G.f[g];
    if (!f) continue;
    LDSV_REQUIRE(f->width == 8 || f->width == 16, LDSV_EINVAL, "fno[%d]: width %d (8 or 16)", g,
                 f->width);
    LDSV_REQUIRE(f->layers >= 1 && f->layers <= 64, LDSV_EINVAL, "fno[%d]: layers %d", g,
                 f->layers);
    LDSV_REQUIRE(f->modes >= 1 && 2 * f->modes <= h->g.ny && 2 * f->modes <= h->g.nx,
                 LDSV_EINVAL, "fno[%d]: modes %d needs 2 modes <= Ny and modes <= Nx/2", g,
                 f->modes);
    LDSV_REQUIRE(f->n_in == G.nin && f->n_out == G.nout, LDSV_EINVAL,
                 "fno[%d]: %d inputs and %d outputs where this call needs %d and %d", g, f->n_in,
                 f->n_out, G.nin, G.nout);
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
  LDSV_REQUIRE(G.nin >= 1 && G.nin <= kMaxIn && G.nout >= 1 && G.nout <= 4, LDSV_EINVAL,
               "fno: %d inputs (1..%d) and %d outputs (1..4)", G.nin, kMaxIn, G.nout);
  for (int j = 0; j < G.nin; ++j) LDSV_REQUIRE(G.xin[j], LDSV_EINVAL, "fno: null input plane %d", j);
  LDSV_REQUIRE((size_t)h->ncell <= (size_t)16 * kFnoBlock &&
                   (size_t)h->ncell * sizeof(Cx<float>) <= 131072,
               LDSV_ESHAPE, "fno: the grid must fit one LDS transform (Nx Ny <= 16384)");
  return LDSV_OK;
}

// Workspace.  Inference: X, Y (nnet B C nm complex) and two activation
// buffers va, vb (nnet B C N floats).  Kept for the backward (keep): the L
// pre-activations z_l, the L forward spectra X_l and v_0.  Backward (bwd):
// two cotangent buffers, the per-b-group partial sums of the spectral
// weight gradient and the small per-block partial sums.
constexpr int kDRGroups = 8;  // b-groups of the spectral weight gradient
struct FnoWs {
  c32 *X, *Y;
  float *va, *vb;
  float* pre;   // [L][act]
  c32* xs;      // [L][spec]
  float* v0;    // [act] (va's partner in inference)
  float *da, *db;
  float* part;  // spectral gradient partials [nnet][kDRGroups][C C nm] complex
  float* small; // small partials
  size_t act, spec, small_len;
};

size_t fno_small_len(const ldsv_handle* h, const FnoShape& sh) {
  const size_t nblk = (h->ncell + kBlock - 1) / kBlock;
  const size_t a = (size_t)sh.nnet * h->g.batch * nblk * (4 * sh.C + 4);       // projection
  const size_t nch = (h->ncell + kWChunk - 1) / kWChunk;
  const size_t b = (size_t)sh.nnet * h->g.batch * nch * (sh.C * sh.C + sh.C);  // pointwise
  const size_t c = (size_t)sh.nnet * h->g.batch * nblk * (kMaxIn + 1) * sh.C;  // lift
  return std::max(a, std::max(b, c));
}

int ensure_fno(ldsv_handle* h, const FnoShape& sh, int level, FnoWs* w) {
  const size_t act = (size_t)sh.nnet * h->g.batch * sh.C * h->ncell;
  const size_t nm = (size_t)2 * sh.M * sh.M;
  const size_t spec = (size_t)sh.nnet * h->g.batch * sh.C * nm;
  const size_t part = (size_t)sh.nnet * kDRGroups * sh.C * sh.C * nm * 2;
  const size_t small = fno_small_len(h, sh);
  size_t need = 2 * spec * sizeof(c32) + 2 * act * sizeof(float);
  if (level >= 1) need += (size_t)sh.L * (act * sizeof(float) + spec * sizeof(c32)) + act * sizeof(float);
  if (level >= 2) need += 2 * act * sizeof(float) + (part + small) * sizeof(float);
  if (need > h->fno_bytes) {
    // grown workspaces are kept (owned by the handle) until ldsv_destroy
    LDSV_TRY(ldsv_alloc(h, &h->fno_blk, need, "FNO workspace"));
    h->fno_bytes = need;
  }
  char* p = (char*)h->fno_blk;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += bytes;
    return q;
  };
  *w = FnoWs{};
  w->act = act;
  w->spec = spec;
  w->small_len = small;
  w->X = (c32*)take(spec * sizeof(c32));
  w->Y = (c32*)take(spec * sizeof(c32));
  w->va = (float*)take(act * sizeof(float));
  w->vb = (float*)take(act * sizeof(float));
  w->v0 = w->vb;
  if (level >= 1) {
    w->pre = (float*)take((size_t)sh.L * act * sizeof(float));
    w->xs = (c32*)take((size_t)sh.L * spec * sizeof(c32));
    w->v0 = (float*)take(act * sizeof(float));
  }
  if (level >= 2) {
    w->da = (float*)take(act * sizeof(float));
    w->db = (float*)take(act * sizeof(float));
    w->part = (float*)take(part * sizeof(float));
    w->small = (float*)take(small * sizeof(float));
  }
  return LDSV_OK;
}

FnoArgs make_args(const FnoGroup& G, const FnoShape& sh, int layer) {
  FnoArgs a{};
  int z = 0;
  for (int g = 0; g < 2; ++g) {
    a.slot[g] = -1;
    a.out_ch[g] = G.out_ch[g];
    const ldsv_fno* f = g < G.ngrid ? G.f[g] : nullptr;
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
  a.nin = G.nin;
  a.nout = G.nout;
  for (int j = 0; j < G.nin; ++j) a.xin[j] = G.xin[j];
  a.out = G.out;
  a.out_cs = G.out_cs;
  a.out_bs = G.out_bs;
  return a;
}

// layer l reads v_l from v0 (l = 0) or the buffer layer l - 1 wrote, and
// writes v_{l+1} to va (l even) or vb (l odd)
inline float* fno_in(const FnoWs& w, int l) { return l == 0 ? w.v0 : (l % 2 ? w.va : w.vb); }
inline float* fno_out(const FnoWs& w, int l) { return l % 2 ? w.vb : w.va; }

template <int E>
int fno_forward_e(ldsv_handle* h, const FnoGroup& G, const FnoShape& sh, const FnoWs& w,
                  hipStream_t st) {
  c32* Y = w.Y;
  const int nx = h->g.nx, ny = h->g.ny, B = h->g.batch, C = sh.C, M = sh.M;
  const size_t lds = ((size_t)nx * ny + nx + ny) * sizeof(Cx<float>);
  const dim3 gfft(C / 2, B, sh.nnet);
  const int nm = 2 * M * M;
  int bpg = B / 8;
  if (bpg < 1) bpg = 1;
  const dim3 gmix((nm + 63) / 64, (B + bpg - 1) / bpg, sh.nnet);
  const Cx<float>* twx = (const Cx<float>*)h->twx;
  const Cx<float>* twy = (const Cx<float>*)h->twy;
  const bool sq64 = nx == 64 && ny == 64;
  for (int l = 0; l < sh.L; ++l) {
    const FnoArgs a = make_args(G, sh, l);
    const bool first = l == 0, last = l == sh.L - 1;
    float* zl = w.pre ? w.pre + (size_t)l * w.act : nullptr;
    c32* X = w.xs ? w.xs + (size_t)l * w.spec : w.X;
    float* cur = fno_in(w, l);
    float* nxt = fno_out(w, l);
    if (sq64) {
      // the compile-time transforms (64^2): v_0 = lift(inputs) written to
      // cur on the way in the first layer
      if (first)
        LDSV_TLAUNCH(h, 8, (k_fno_spec_r<6, true>), gfft, dim3(512), 0, st, (const float*)nullptr,
                     a, cur, X, twx, C, M, B);
      else
        LDSV_TLAUNCH(h, 8, (k_fno_spec_r<6, false>), gfft, dim3(512), 0, st, (const float*)cur,
                     a, (float*)nullptr, X, twx, C, M, B);
    } else if (first) {
      // v_0 = lift(inputs) is written to cur on the way
      auto k = k_fno_spec<spec_e<E>(), true>;
      LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(fno_block<spec_e<E>()>()), lds, st, (const float*)nullptr,
                   (const float*)nullptr, a, cur, X, twx, twy, nx, ny, h->log2nx, h->log2ny, C, M,
                   B);
    } else {
      auto k = k_fno_spec<spec_e<E>(), false>;
      LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(fno_block<spec_e<E>()>()), lds, st, (const float*)cur,
                   (const float*)nullptr, a, (float*)nullptr, X, twx, twy, nx, ny, h->log2nx,
                   h->log2ny, C, M, B);
    }
    if (C == 16)
      LDSV_TLAUNCH(h, 9, (k_fno_mix<16, false>), gmix, dim3(64 * 16), 0, st, (const c32*)X,
                   a, Y, B, nm, bpg);
    else
      LDSV_TLAUNCH(h, 9, (k_fno_mix<8, false>), gmix, dim3(64 * 8), 0, st, (const c32*)X, a,
                   Y, B, nm, bpg);
    if (sq64) {
      auto k = last ? (C == 16 ? k_fno_inv_r<6, 16, 1> : k_fno_inv_r<6, 8, 1>)
                    : (C == 16 ? k_fno_inv_r<6, 16, 0> : k_fno_inv_r<6, 8, 0>);
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(512), 0, st, (const c32*)Y, (const float*)cur, a, nxt, zl,
                   twx, M, B);
    } else {
      auto k = last ? (C == 16 ? k_fno_inv<E, 16, 1> : k_fno_inv<E, 8, 1>)
                    : (C == 16 ? k_fno_inv<E, 16, 0> : k_fno_inv<E, 8, 0>);
      LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(fno_block<E>()), lds, st, (const c32*)Y, (const float*)cur, a,
                   nxt, zl, (const float*)nullptr, twx, twy, nx, ny, h->log2nx, h->log2ny, M, B);
    }
  }
  const FnoArgs a = make_args(G, sh, 0);
  LDSV_TLAUNCH(h, 7, k_fno_proj, dim3((unsigned)((h->ncell + kBlock - 1) / kBlock), B, G.ngrid),
               dim3(kBlock), 0, st, (const float*)fno_out(w, sh.L - 1), a, (int)h->ncell, C, B);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

int sum_partials(ldsv_handle* h, const FnoShape& sh, const FnoArgs& a, const float* part,
                 int nblk, size_t stride, int off, int len, float* const outs[2],
                 hipStream_t st) {
  PartOut po{};
  for (int z = 0; z < sh.nnet; ++z) po.out[z] = outs[a.net[z]];
  if (len <= 4096 && nblk >= 64)
    LDSV_TLAUNCH(h, 7, k_sum_partials<16>, dim3((len + kBlock / 16 - 1) / (kBlock / 16), 1, sh.nnet),
                 dim3(kBlock), 0, st, part, nblk, stride, off, len, po);
  else
    LDSV_TLAUNCH(h, 7, k_sum_partials<1>, dim3((len + kBlock - 1) / kBlock, 1, sh.nnet),
                 dim3(kBlock), 0, st, part, nblk, stride, off, len, po);
  return LDSV_OK;
}

template <int E, int C>
int fno_backward_e(ldsv_handle* h, const FnoGroup& G, const ldsv_fno_grad* const gr[2],
                   const FnoShape& sh, const float* gout, const GradIn& gi, int accumulate,
                   const FnoWs& w, hipStream_t st) {
  const int nx = h->g.nx, ny = h->g.ny, B = h->g.batch, M = sh.M;
  const int n = (int)h->ncell;
  const size_t lds = ((size_t)nx * ny + nx + ny) * sizeof(Cx<float>);
  const dim3 gfft(C / 2, B, sh.nnet);
  const int nm = 2 * M * M;
  int bpg = B / 8;
  if (bpg < 1) bpg = 1;
  const dim3 gmix((nm + 63) / 64, (B + bpg - 1) / bpg, sh.nnet);
  const int bpg_r = (B + kDRGroups - 1) / kDRGroups;
  const int ngr = (B + bpg_r - 1) / bpg_r;
  const Cx<float>* twx = (const Cx<float>*)h->twx;
  const Cx<float>* twy = (const Cx<float>*)h->twy;
  const int nblk = (n + kBlock - 1) / kBlock;
  const int nin = G.nin, nout = G.nout;
  float* g_lift_w[2] = {nullptr, nullptr};
  float* g_lift_b[2] = {nullptr, nullptr};
  float* g_proj_w[2] = {nullptr, nullptr};
  float* g_proj_b[2] = {nullptr, nullptr};
  for (int g = 0; g < G.ngrid; ++g) {
    if (!G.f[g]) continue;
    g_lift_w[g] = gr[g]->lift_w;
    g_lift_b[g] = gr[g]->lift_b;
    g_proj_w[g] = gr[g]->proj_w;
    g_proj_b[g] = gr[g]->proj_b;
  }
  // projection
  const FnoArgs a0 = make_args(G, sh, 0);
  float* dcur = w.da;
  float* dnxt = w.db;
  const float* vL = w.pre + (size_t)(sh.L - 1) * w.act;
  if (nout == 4)
    LDSV_TLAUNCH(h, 7, (k_fno_proj_bwd<C, 4>), dim3(nblk, B, sh.nnet), dim3(kBlock), 0, st, gout,
                 vL, a0, dcur, w.small, n, B);
  else
    LDSV_TLAUNCH(h, 7, (k_fno_proj_bwd<C, 2>), dim3(nblk, B, sh.nnet), dim3(kBlock), 0, st, gout,
                 vL, a0, dcur, w.small, n, B);
  const int pw_len = nout * C + nout;
  LDSV_TRY(sum_partials(h, sh, a0, w.small, B * nblk, pw_len, 0, nout * C, g_proj_w, st));
  LDSV_TRY(sum_partials(h, sh, a0, w.small, B * nblk, pw_len, nout * C, nout, g_proj_b, st));
  for (int l = sh.L - 1; l >= 0; --l) {
    const FnoArgs a = make_args(G, sh, l);
    float* g_pw[2] = {nullptr, nullptr};
    float* g_pb[2] = {nullptr, nullptr};
    float* g_sw[2] = {nullptr, nullptr};
    for (int g = 0; g < G.ngrid; ++g) {
      if (!G.f[g]) continue;
      g_pw[g] = gr[g]->point_w + (size_t)l * C * C;
      g_pb[g] = gr[g]->point_b + (size_t)l * C;
      g_sw[g] = gr[g]->spec_w + (size_t)l * C * C * nm * 2;
    }
    // pointwise weight and bias gradients (v_l from v_0 or GELU(z_{l-1}))
    const int nch = (n + kWChunk - 1) / kWChunk;
    if (l == 0)
      LDSV_TLAUNCH(h, 7, (k_fno_wgrad<C, false>), dim3(nch, sh.nnet * B), dim3(C * C), 0, st,
                   (const float*)dcur, (const float*)w.v0, w.small, n, B);
    else
      LDSV_TLAUNCH(h, 7, (k_fno_wgrad<C, true>), dim3(nch, sh.nnet * B), dim3(C * C), 0, st,
                   (const float*)dcur, (const float*)(w.pre + (size_t)(l - 1) * w.act), w.small, n,
                   B);
    LDSV_TRY(sum_partials(h, sh, a, w.small, B * nch, C * C + C, 0, C * C, g_pw, st));
    LDSV_TRY(sum_partials(h, sh, a, w.small, B * nch, C * C + C, C * C, C, g_pb, st));
    // DZ = F(dz_l) into X
    {
      auto k = k_fno_spec<spec_e<E>(), false>;
      LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(fno_block<spec_e<E>()>()), lds, st, (const float*)dcur,
                   (const float*)nullptr, a, (float*)nullptr, w.X, twx, twy, nx, ny, h->log2nx,
                   h->log2ny, C, M, B);
    }
    // spectral weight gradient
    LDSV_TLAUNCH(h, 9, k_fno_dR<C>, dim3((nm + 63) / 64, ngr, sh.nnet), dim3(64 * C), 0, st,
                 (const c32*)(w.xs + (size_t)l * w.spec), (const c32*)w.X, (c32*)w.part, B, nm, M,
                 bpg_r, 1.0f / (float)n);
    LDSV_TRY(sum_partials(h, sh, a, w.part, ngr, (size_t)C * C * nm * 2, 0, C * C * nm * 2, g_sw,
                          st));
    // dv_l = K^T dz + W^T dz, then dz_{l-1} = dv_l GELU'(z_{l-1})
    LDSV_TLAUNCH(h, 9, (k_fno_mix<C, true>), gmix, dim3(64 * C), 0, st, (const c32*)w.X, a, w.Y,
                 B, nm, bpg);
    {
      auto k = l == 0 ? k_fno_inv<E, C, 3> : k_fno_inv<E, C, 2>;
      LDSV_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
      LDSV_TLAUNCH(h, 8, k, gfft, dim3(fno_block<E>()), lds, st, (const c32*)w.Y, (const float*)dcur,
                   a, dnxt, (float*)nullptr,
                   (const float*)(l > 0 ? w.pre + (size_t)(l - 1) * w.act : nullptr), twx, twy,
                   nx, ny, h->log2nx, h->log2ny, M, B);
    }
    std::swap(dcur, dnxt);
  }
  // lift: dcur holds dv_0
  LDSV_TLAUNCH(h, 7, k_fno_lift_bwd<C>, dim3(nblk, B), dim3(kBlock), 0, st, (const float*)dcur,
               a0, sh.nnet, gi, accumulate, w.small, n, B);
  const int lw_len = (nin + 1) * C;
  LDSV_TRY(sum_partials(h, sh, a0, w.small, B * nblk, lw_len, 0, nin * C, g_lift_w, st));
  LDSV_TRY(sum_partials(h, sh, a0, w.small, B * nblk, lw_len, nin * C, C, g_lift_b, st));
  LDSV_LAUNCHED();
  return LDSV_OK;
}

int check_grads(const FnoGroup& G, const ldsv_fno_grad* const gr[2]) {
  for (int g = 0; g < G.ngrid; ++g) {
    if (!G.f[g]) continue;
    const ldsv_fno_grad* q = gr[g];
    LDSV_REQUIRE(q && q->lift_w && q->lift_b && q->spec_w && q->point_w && q->point_b &&
                     q->proj_w && q->proj_b,
                 LDSV_EINVAL, "fno[%d]: null gradient buffer", g);
  }
  return LDSV_OK;
}

// the flux block's pair: inputs (u, v), fields [B][8][Ny][Nx]
FnoGroup flux_group(const ldsv_handle* h, const ldsv_fluxnet* net, const float* u, const float* v,
                    float* fields) {
  FnoGroup G{};
  G.f[0] = net->fno[0];
  G.f[1] = net->fno[1];
  G.ngrid = 2;
  G.nin = 2;
  G.nout = 4;
  G.xin[0] = u;
  G.xin[1] = v;
  G.out = fields;
  G.out_cs = h->ncell;
  G.out_bs = 8 * h->ncell;
  G.out_ch[0] = 0;
  G.out_ch[1] = 4;
  return G;
}

// the temporal correction: inputs the k_c states (u, v) oldest first,
// output (du, dv) as two [B][Ny][Nx] planes at out and out + B Ny Nx
FnoGroup tc_group(const ldsv_handle* h, const ldsv_fno* tc, const float* const* hu,
                  const float* const* hv, int kc, float* out) {
  FnoGroup G{};
  G.f[0] = tc;
  G.f[1] = nullptr;
  G.ngrid = 1;
  G.nin = 2 * kc;
  G.nout = 2;
  for (int j = 0; j < kc && 2 * j + 1 < kMaxIn; ++j) {
    G.xin[2 * j] = hu[j];
    G.xin[2 * j + 1] = hv[j];
  }
  G.out = out;
  G.out_cs = h->nstate;
  G.out_bs = h->ncell;
  return G;
}

int group_forward(ldsv_handle* h, const FnoGroup& G, bool keep_pre, hipStream_t st) {
  FnoShape sh;
  LDSV_TRY(check_group(h, G, &sh));
  if (sh.nnet == 0) {
    // no operator: zero outputs (a kernel, not a memset, so that the call
    // can sit in a captured graph)
    const FnoArgs a = make_args(G, sh, 0);
    LDSV_TLAUNCH(h, 7, k_fno_proj, dim3((unsigned)((h->ncell + kBlock - 1) / kBlock), h->g.batch,
                                        G.ngrid),
                 dim3(kBlock), 0, st, (const float*)nullptr, a, (int)h->ncell, 0, h->g.batch);
    LDSV_LAUNCHED();
    return LDSV_OK;
  }
  FnoWs w;
  // a forward that keeps its activations sizes the workspace for the
  // backward as well, so the backward that follows does not move them
  LDSV_TRY(ensure_fno(h, sh, keep_pre ? 2 : 0, &w));
  if (h->ncell <= (size_t)4 * kFnoBlock) return fno_forward_e<4>(h, G, sh, w, st);
  return fno_forward_e<16>(h, G, sh, w, st);
}

// backward of the group from gout (addressed like its output); when
// forward_kept is false the forward is run first (its output goes to G.out)
int group_backward(ldsv_handle* h, const FnoGroup& G, const ldsv_fno_grad* const gr[2],
                   const float* gout, const GradIn& gi, int accumulate, bool forward_kept,
                   hipStream_t st) {
  FnoShape sh;
  LDSV_TRY(check_group(h, G, &sh));
  if (sh.nnet == 0) {
    if (gi.gx[0] && !accumulate) {
      for (int j = 0; j < G.nin; ++j)
        LDSV_TLAUNCH(h, 7, k_fill_zero, grid1d(h->nstate), dim3(kBlock), 0, st, gi.gx[j],
                     h->nstate);
      LDSV_LAUNCHED();
    }
    return LDSV_OK;
  }
  LDSV_TRY(check_grads(G, gr));
  FnoWs w;
  LDSV_TRY(ensure_fno(h, sh, 2, &w));
  const bool small = h->ncell <= (size_t)4 * kFnoBlock;
  if (!forward_kept) {
    if (small) LDSV_TRY(fno_forward_e<4>(h, G, sh, w, st));
    else LDSV_TRY(fno_forward_e<16>(h, G, sh, w, st));
  }
  if (small && sh.C == 16) return fno_backward_e<4, 16>(h, G, gr, sh, gout, gi, accumulate, w, st);
  if (small) return fno_backward_e<4, 8>(h, G, gr, sh, gout, gi, accumulate, w, st);
  if (sh.C == 16) return fno_backward_e<16, 16>(h, G, gr, sh, gout, gi, accumulate, w, st);
  return fno_backward_e<16, 8>(h, G, gr, sh, gout, gi, accumulate, w, st);
}

}  // namespace

// forward with the saved activations, then the backward from gfields:
// accumulates the parameter gradients into gr; gu, gv (nullable) receive
// (or, with accumulate, add) the input gradient
int ldsv_launch_fno_backward(ldsv_handle* h, const ldsv_fluxnet* net, const ldsv_fluxnet_grad* gr,
                             const float* u, const float* v, const float* gfields, float* gu,
                             float* gv, int accumulate, hipStream_t st, bool forward_kept) {
  LDSV_REQUIRE(net && gr, LDSV_EINVAL, "fno backward: null network or gradient");
  LDSV_TRY(ldsv_ensure_fluxblock(h));
  // a forward run here writes its fields into the handle's scratch field buffer
  const FnoGroup G = flux_group(h, net, u, v, h->fb_fields);
  const ldsv_fno_grad* grs[2] = {gr->fno[0], gr->fno[1]};
  GradIn gi{};
  gi.gx[0] = gu;
  gi.gx[1] = gv;
  return group_backward(h, G, grs, gfields, gi, accumulate, forward_kept, st);
}

int ldsv_launch_fno_forward(ldsv_handle* h, const ldsv_fluxnet* net, const float* u,
                            const float* v, float* fields, bool keep_pre, hipStream_t st) {
  LDSV_REQUIRE(net, LDSV_EINVAL, "flux block: null network");
  return group_forward(h, flux_group(h, net, u, v, fields), keep_pre, st);
}

int ldsv_launch_tc_forward(ldsv_handle* h, const ldsv_fno* tc, const float* const* hu,
                           const float* const* hv, int kc, float* out, bool keep_pre,
                           hipStream_t st) {
  LDSV_REQUIRE(tc && hu && hv && kc >= 1 && 2 * kc <= kMaxIn, LDSV_EINVAL,
               "temporal correction: null operator or history, or k_c = %d outside 1..%d", kc,
               kMaxIn / 2);
  return group_forward(h, tc_group(h, tc, hu, hv, kc, out), keep_pre, st);
}

int ldsv_launch_tc_backward(ldsv_handle* h, const ldsv_fno* tc, const ldsv_fno_grad* gtc,
                            const float* const* hu, const float* const* hv, int kc,
                            const float* gout, float* const* ghu, float* const* ghv,
                            bool forward_kept, float* scratch_out, hipStream_t st) {
  LDSV_REQUIRE(tc && gtc && hu && hv && ghu && ghv && kc >= 1 && 2 * kc <= kMaxIn, LDSV_EINVAL,
               "temporal correction backward: null argument or k_c = %d outside 1..%d", kc,
               kMaxIn / 2);
  const FnoGroup G = tc_group(h, tc, hu, hv, kc, scratch_out);
  const ldsv_fno_grad* grs[2] = {gtc, nullptr};
  GradIn gi{};
  for (int j = 0; j < kc; ++j) {
    gi.gx[2 * j] = ghu[j];
    gi.gx[2 * j + 1] = ghv[j];
  }
  return group_backward(h, G, grs, gout, gi, 1, forward_kept, st);
}

int ldsv_ensure_fluxblock(ldsv_handle* h) {
  if (h->fb_fields) return LDSV_OK;
  void* p = nullptr;
  // fields and their gradient (8 planes each), the temporal correction and
  // its gradient (2 each), a state-sized scratch pair (2)
  LDSV_TRY(ldsv_alloc(h, &p, (size_t)22 * h->nstate * sizeof(float), "flux-block fields"));
  h->fb_fields = (float*)p;
  h->fb_gfields = h->fb_fields + 8 * h->nstate;
  h->fb_tc = h->fb_gfields + 8 * h->nstate;
  h->fb_gtc = h->fb_tc + 2 * h->nstate;
  h->fb_tmp = h->fb_gtc + 2 * h->nstate;
  return LDSV_OK;
}

int ldsv_internal_step_fb(ldsv_handle* h, const ldsv_params* p, const FluxBlockArgs* fb,
                          const void* su, const void* sv, void* du, void* dv, hipStream_t st,
                          const float* tcu = nullptr, const float* tcv = nullptr,
                          size_t tcbs = 0);

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

int ldsv_fno_backward(ldsv_handle* h, const ldsv_fluxnet* net, const float* u, const float* v,
                      const float* gfields, float* gu, float* gv, const ldsv_fluxnet_grad* grad,
                      void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(net && u && v && gfields, LDSV_EINVAL, "fno_backward: null argument");
  LDSV_REQUIRE((gu == nullptr) == (gv == nullptr), LDSV_EINVAL, "fno_backward: gu and gv together");
  return ldsv_launch_fno_backward(h, net, grad, u, v, gfields, gu, gv, 0, (hipStream_t)stream,
                                  false);
}

int ldsv_fluxblock_step_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_fluxnet* net,
                            const float* u_in, const float* v_in, const float* gu_out,
                            const float* gv_out, float* gu_in, float* gv_in,
                            const ldsv_fluxnet_grad* grad, void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && net && net->stencil_w && u_in && v_in && gu_out && gv_out && gu_in && gv_in &&
                   grad,
               LDSV_EINVAL, "fluxblock_step_bwd: null argument");
  LDSV_REQUIRE(prm->rk == LDSV_RK4, LDSV_EDTYPE, "fluxblock_step_bwd: RK4");
  const hipStream_t st = (hipStream_t)stream;
  LDSV_TRY(ldsv_ensure_fluxblock(h));
  FnoShape sh;
  {
    const FnoGroup G = flux_group(h, net, u_in, v_in, h->fb_fields);
    LDSV_TRY(check_group(h, G, &sh));
    const ldsv_fno_grad* grs[2] = {grad->fno[0], grad->fno[1]};
    LDSV_TRY(check_grads(G, grs));
  }
  // the fields of the forward step (activations kept for the FNO backward),
  // then the FV adjoint with their gradient
  LDSV_TRY(ldsv_launch_fno_forward(h, net, u_in, v_in, h->fb_fields, true, st));
  LDSV_TLAUNCH(h, 7, k_fill_zero, grid1d(8 * h->nstate), dim3(kBlock), 0, st, h->fb_gfields,
               8 * h->nstate);
  LDSV_LAUNCHED();
  FluxBlockArgs fb;
  fb.w = net->stencil_w;
  fb.f = h->fb_fields;
  fb.fbs = (size_t)8 * h->ncell;
  fb.gw = grad->stencil_w;
  fb.gf = h->fb_gfields;
  fb.gfbs = (size_t)8 * h->ncell;
  LDSV_TRY(ldsv_step_bwd(h, prm, nullptr, 0, nullptr, 0, u_in, v_in, gu_out, gv_out, gu_in, gv_in,
                         st, &fb));
  if (sh.nnet == 0) return LDSV_OK;
  // the operators' gradients, their input gradient added to the state's
  return ldsv_launch_fno_backward(h, net, grad, u_in, v_in, h->fb_gfields, gu_in, gv_in, 1, st,
                                  true);
}

int ldsv_fluxblock_tc_step(ldsv_handle* h, const ldsv_params* prm, const ldsv_fluxnet* net,
                           const ldsv_fno* tc, const float* const* hist_u,
                           const float* const* hist_v, int step_index, float* u_out, float* v_out,
                           void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && net && net->stencil_w && hist_u && hist_v && u_out && v_out, LDSV_EINVAL,
               "fluxblock_tc_step: null argument");
  LDSV_REQUIRE(prm->rk == LDSV_RK4, LDSV_EDTYPE, "fluxblock_tc_step: RK4");
  const int kc = prm->k_c;
  LDSV_REQUIRE(kc >= 1 && 2 * kc <= kMaxIn, LDSV_EINVAL,
               "fluxblock_tc_step: k_c = %d outside 1..%d", kc, kMaxIn / 2);
  const float* u_in = hist_u[kc - 1];
  const float* v_in = hist_v[kc - 1];
  LDSV_REQUIRE(u_in && v_in, LDSV_EINVAL, "fluxblock_tc_step: null input state");
  const hipStream_t st = (hipStream_t)stream;
  LDSV_TRY(ldsv_ensure_fluxblock(h));
  LDSV_TRY(ldsv_launch_fno_forward(h, net, u_in, v_in, h->fb_fields, false, st));
  const bool apply = tc && step_index % kc == 0;
  if (apply)
    LDSV_TRY(ldsv_launch_tc_forward(h, tc, hist_u, hist_v, kc, h->fb_tc, false, st));
  FluxBlockArgs fb;
  fb.w = net->stencil_w;
  fb.f = h->fb_fields;
  fb.fbs = (size_t)8 * h->ncell;
  return ldsv_internal_step_fb(h, prm, &fb, u_in, v_in, u_out, v_out, st,
                               apply ? h->fb_tc : nullptr, apply ? h->fb_tc + h->nstate : nullptr,
                               h->ncell);
}

int ldsv_fluxblock_tc_step_bwd(ldsv_handle* h, const ldsv_params* prm, const ldsv_fluxnet* net,
                               const ldsv_fno* tc, const float* const* hist_u,
                               const float* const* hist_v, int step_index, const float* gu_out,
                               const float* gv_out, float* const* ghist_u, float* const* ghist_v,
                               const ldsv_fluxnet_grad* grad, const ldsv_fno_grad* gtc,
                               void* stream) {
  LDSV_TRY(ldsv_check_handle(h));
  LDSV_REQUIRE(prm && net && hist_u && hist_v && gu_out && gv_out && ghist_u && ghist_v && grad,
               LDSV_EINVAL, "fluxblock_tc_step_bwd: null argument");
  const int kc = prm->k_c;
  LDSV_REQUIRE(kc >= 1 && 2 * kc <= kMaxIn, LDSV_EINVAL,
               "fluxblock_tc_step_bwd: k_c = %d outside 1..%d", kc, kMaxIn / 2);
  const bool apply = tc && step_index % kc == 0;
  LDSV_REQUIRE(!apply || gtc, LDSV_EINVAL, "fluxblock_tc_step_bwd: null correction gradient");
  const hipStream_t st = (hipStream_t)stream;
  LDSV_TRY(ldsv_ensure_fluxblock(h));
  float* tu = h->fb_tmp;
  float* tv = h->fb_tmp + h->nstate;
  // through the FV step and the flux block into the last state (the
  // correction does not change the step's Jacobian: it is added)
  LDSV_TRY(ldsv_fluxblock_step_bwd(h, prm, net, hist_u[kc - 1], hist_v[kc - 1], gu_out, gv_out, tu,
                                   tv, grad, stream));
  LDSV_TRY(ldsv_launch_axpy2(h, ghist_u[kc - 1], ghist_v[kc - 1], tu, tv, 1.0, st));
  if (!apply) return LDSV_OK;
  // dL/dTC = P^T g = P g (the correction enters before the last projection)
  float* gcu = h->fb_gtc;
  float* gcv = h->fb_gtc + h->nstate;
  LDSV_TRY(ldsv_launch_project(h, gu_out, gv_out, gcu, gcv, nullptr, st));
  LDSV_TRY(ldsv_launch_tc_forward(h, tc, hist_u, hist_v, kc, h->fb_tc, true, st));
  return ldsv_launch_tc_backward(h, tc, gtc, hist_u, hist_v, kc, gcu, ghist_u, ghist_v, true,
                                 h->fb_tc, st);
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
