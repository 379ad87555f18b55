// Pressure projection on the periodic MAC grid (App. B.3, S8-S10; App. B.4,
// S11-S14).
//
//   d = D u*   (compact MAC divergence, cell centres)
//   p = (D G)^+ d  by FFT: p_hat = -d_hat / lambda_h(k), p_hat(0) = 0,
//       lambda_h = (2/dx)^2 sin^2(pi kx/Nx) + (2/dy)^2 sin^2(pi ky/Ny)
//   u = u* - G p
//
// Two trajectories are packed into one complex field z = d_b + i d_{b+1}.
// The Poisson multiplier is real and even in k, so the real and imaginary
// parts stay independent through forward FFT, division and inverse FFT;
// this halves the transform work compared with one complex FFT per
// trajectory and needs no real-to-complex unpacking.
//
// Three passes, each one HBM sweep:
//   k_div_rowfft     reads u*, v*; forms d for the pair; FFT along x; writes z
//   k_col_solve      FFT along y, multiply by the FP64 factor -1/(lambda_h Nx Ny)
//                    (the division by the eigenvalue with the inverse
//                    normalisation folded in; tabulated in FP64 when the
//                    handle is created), inverse FFT along y, in place
//   k_rowifft_grad   inverse FFT along x for rows j-1..j+R-1, then
//                    u = u* - (p - p[i-1])/dx, v = v* - (p - p[j-1])/dy
#include "fft_lds.h"
#include "fft_reg.h"
#include <algorithm>

namespace {

// the pair (b0, b0 + 1) has work when either of its trajectories is active
// (no mask: every trajectory is)
__device__ __forceinline__ bool pair_active(const int* active, int b0, int batch) {
  return !active || active[b0] || (b0 + 1 < batch && active[b0 + 1]);
}

constexpr int kRowE = 4;       // elements per thread, pass 1
constexpr int kRow1MaxBlock = 512;
constexpr int kRowE3 = 8;      // pass 3, with its extra halo row
constexpr int kRow3Block = 1024;
constexpr int kColE = 16;      // column pass
constexpr int kColBlock = 512; // largest column-pass block

template <typename T>
__global__ void __launch_bounds__(kRow1MaxBlock) k_div_rowfft(const T* __restrict__ us,
                                                       const T* __restrict__ vs,
                                                       Cx<T>* __restrict__ z,
                                                       const Cx<T>* __restrict__ twx, int nx,
                                                       int ny, int log2nx, int batch, int rows,
                                                       T idx, T idy, const int* active) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  // row bands renumbered so one XCD walks consecutive bands (the halo row
  // of a band is the next band's first row)
  const int band = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int pair = band / gridDim.x;
  const int b0 = 2 * pair;
  if (!pair_active(active, b0, batch)) return;
  Cx<T>* A = reinterpret_cast<Cx<T>*>(smem_raw);
  Cx<T>* W = A + rows * nx;  // twiddles, read by every stage
  for (int e = threadIdx.x; e < nx; e += blockDim.x) W[e] = twx[e];
  // a masked-out trajectory of the pair contributes zeros, so that whatever
  // its buffers hold cannot reach its partner through the packed transform
  const bool has0 = !active || active[b0];
  const bool has1 = (b0 + 1) < batch && (!active || active[b0 + 1]);
  const int j0 = (band - pair * gridDim.x) * rows;
  const size_t plane = (size_t)nx * ny;
  const T* u0 = us + (size_t)b0 * plane;
  const T* v0 = vs + (size_t)b0 * plane;
  const T* u1 = u0 + plane;
  const T* v1 = v0 + plane;
#pragma unroll
  for (int k = 0; k < kRowE; ++k) {
    const int t = k * blockDim.x + threadIdx.x;
    if (t < rows * nx) {
      const int r = t >> log2nx;
      const int i = t & (nx - 1);
      const int j = j0 + r;
      const int ip = (i + 1) & (nx - 1);
      const int jp = (j + 1) & (ny - 1);
      const size_t c = (size_t)j * nx + i;
      T d0 = 0;
      if (has0) d0 = (u0[(size_t)j * nx + ip] - u0[c]) * idx + (v0[(size_t)jp * nx + i] - v0[c]) * idy;
      T d1 = 0;
      if (has1) d1 = (u1[(size_t)j * nx + ip] - u1[c]) * idx + (v1[(size_t)jp * nx + i] - v1[c]) * idy;
      A[t] = Cx<T>{d0, d1};
    }
  }
  __syncthreads();
  lds_fft<T, kRowE>(A, nx, log2nx, rows, nx, 1, -1, W);
  Cx<T>* zo = z + (size_t)pair * plane + (size_t)j0 * nx;
#pragma unroll
  for (int k = 0; k < kRowE; ++k) {
    const int t = k * blockDim.x + threadIdx.x;
    if (t < rows * nx) zo[t] = A[t];
  }
}

// columns x0..x0+cols-1 of one pair: forward FFT along y, multiply by the
// FP64 Poisson factor -1/(lambda_h Nx Ny) (0 for the zero mode), inverse FFT.
// Blocks of 8 columns (64-byte row segments in FP32): two or more blocks per
// CU overlap one block's memory phase with another's transform.  XCD x takes
// the column groups [x ncx/8, (x+1) ncx/8) of every pair, so the two halves
// of a 128-byte line and the matching rows of the factor table stay in its
// L2.
template <typename T>
__global__ void __launch_bounds__(kColBlock) k_col_solve(Cx<T>* __restrict__ z,
                                                      const Cx<T>* __restrict__ twy,
                                                      const double* __restrict__ pinv, int nx,
                                                      int ny, int log2ny, int log2cols, int batch,
                                                      const int* active) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int cols = 1 << log2cols;
  const int n = cols << log2ny;
  Cx<T>* A = reinterpret_cast<Cx<T>*>(smem_raw);  // element (column c, y) at y * cols + c
  Cx<T>* W = A + n;
  const int ncx = nx >> log2cols;
  int cx, pair;
  {
    const int lid = blockIdx.x;
    if ((ncx & 7) == 0) {
      const int cpx = ncx >> 3, slot = lid >> 3;
      const int q = slot / cpx;
      cx = (lid & 7) * cpx + (slot - q * cpx);
      pair = q;
    } else {
      pair = lid / ncx;
      cx = lid - pair * ncx;
    }
  }
  if (!pair_active(active, 2 * pair, batch)) return;
  for (int e = threadIdx.x; e < ny; e += blockDim.x) W[e] = twy[e];
  const int x0 = cx << log2cols;
  Cx<T>* zp = z + (size_t)pair * nx * ny;
  {
    Cx<T> tmp[kColE];
#pragma unroll
    for (int k = 0; k < kColE; ++k) {
      const int t = k * blockDim.x + threadIdx.x;
      if (t < n) tmp[k] = zp[(size_t)(t >> log2cols) * nx + x0 + (t & (cols - 1))];
    }
#pragma unroll
    for (int k = 0; k < kColE; ++k) {
      const int t = k * blockDim.x + threadIdx.x;
      if (t < n) A[t] = tmp[k];
    }
  }
  __syncthreads();
  lds_fft<T, kColE>(A, ny, log2ny, cols, 1, cols, -1, W);
#pragma unroll
  for (int k = 0; k < kColE; ++k) {
    const int t = k * blockDim.x + threadIdx.x;
    if (t < n) {
      const double s = pinv[(size_t)(t >> log2cols) * nx + x0 + (t & (cols - 1))];
      const Cx<T> v = A[t];
      A[t] = Cx<T>{(T)((double)v.x * s), (T)((double)v.y * s)};
    }
  }
  __syncthreads();
  lds_fft<T, kColE>(A, ny, log2ny, cols, 1, cols, +1, W);
#pragma unroll
  for (int k = 0; k < kColE; ++k) {
    const int t = k * blockDim.x + threadIdx.x;
    if (t < n) zp[(size_t)(t >> log2cols) * nx + x0 + (t & (cols - 1))] = A[t];
  }
}

// The row passes for FP32 with the row length N = 2^LOGN (= nx) and the
// rows per workgroup known at compile time (register-resident first and
// last transform stages, as in k_col_solve_r).
//
// Pass 1: the divergence of the pair (d_b + i d_{b+1}) is formed straight
// into the first stage's registers, the FFT along x runs, and its last
// stage stores the spectrum rows to global memory.
// FULL: every trajectory active and the batch even (both of every pair
// present), known at compile time: no per-point tests
template <int LOGN, int LOGR, bool FULL = false>
__global__ void __launch_bounds__(((1 << LOGN) << LOGR) / 8) k_div_rowfft_r(
    const float* __restrict__ us, const float* __restrict__ vs, Cx<float>* __restrict__ z,
    const Cx<float>* __restrict__ twx, int ny, int batch, float idx, float idy,
    const int* active) {
  constexpr int N = 1 << LOGN, BLOCK = (N << LOGR) / 8, S = fftreg::plan_stages(LOGN);
  constexpr int LR0 = fftreg::plan_lr(LOGN, 0), LRL = fftreg::plan_lr(LOGN, S - 1);
  constexpr int R0 = 1 << LR0, RL = 1 << LRL;
  __shared__ Cx<float> A[fftreg::lds_elems<true, LOGN, LOGR>()];
  __shared__ Cx<float> W[N];
  const int band = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int pair = band / gridDim.x;
  const int b0 = 2 * pair;
  if (!FULL && !pair_active(active, b0, batch)) return;
  const bool has0 = FULL || !active || active[b0];
  const bool has1 = FULL || ((b0 + 1) < batch && (!active || active[b0 + 1]));
  const int j0 = (band - pair * gridDim.x) << LOGR;
  for (int e = threadIdx.x; e < N; e += BLOCK) W[e] = twx[e];
  const size_t plane = (size_t)N * ny;
  const float* u0 = us + (size_t)b0 * plane;
  const float* v0 = vs + (size_t)b0 * plane;
  Cx<float> x[8];
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int t, i;
      fftreg::point<true, LOGN, LOGR, BLOCK, LR0>(q, r, t, i);
      const int j = j0 + t;
      const int ip = (i + 1) & (N - 1);
      const int jp = (j + 1) & (ny - 1);
      const size_t c = ((size_t)j << LOGN) + i;
      float d0 = 0.f, d1 = 0.f;
      if (has0)
        d0 = (u0[((size_t)j << LOGN) + ip] - u0[c]) * idx + (v0[((size_t)jp << LOGN) + i] - v0[c]) * idy;
      if (has1)
        d1 = (u0[plane + ((size_t)j << LOGN) + ip] - u0[plane + c]) * idx +
             (v0[plane + ((size_t)jp << LOGN) + i] - v0[plane + c]) * idy;
      x[q * R0 + r] = Cx<float>{d0, d1};
    }
  __syncthreads();
  fftreg::run<true, LOGN, LOGR, BLOCK, -1, false>(x, A, W);
  Cx<float>* zo = z + (size_t)pair * plane;
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int t, i;
      fftreg::point<true, LOGN, LOGR, BLOCK, LRL>(q, r, t, i);
      zo[((size_t)(j0 + t) << LOGN) + i] = x[q * RL + r];
    }
}

// Pass 3: inverse FFT along x of 2^LOGR rows, the first of them the halo row
// above the band, whose 2^LOGR - 1 rows get u = u* - G p.  Bands of
// 2^LOGR - 1 output rows (the last one clipped at ny, so that every output
// row is written by one workgroup and in-place calls stay safe).
// FULL: as in k_div_rowfft_r, and no p output
template <int LOGN, int LOGR, bool FULL = false>
__global__ void __launch_bounds__(((1 << LOGN) << LOGR) / 8) k_rowifft_grad_r(
    const Cx<float>* __restrict__ z, const Cx<float>* __restrict__ twx,
    const float* __restrict__ us, const float* __restrict__ vs, float* __restrict__ uo,
    float* __restrict__ vo, float* __restrict__ po, int ny, int batch, float idx, float idy,
    const int* active) {
  constexpr int N = 1 << LOGN, ROWS = 1 << LOGR, BLOCK = (N << LOGR) / 8;
  constexpr int S = fftreg::plan_stages(LOGN);
  constexpr int LR0 = fftreg::plan_lr(LOGN, 0), LRL = fftreg::plan_lr(LOGN, S - 1);
  constexpr int R0 = 1 << LR0, RL = 1 << LRL;
  __shared__ Cx<float> A[fftreg::lds_elems<true, LOGN, LOGR>()];
  __shared__ Cx<float> W[N];
  const int band = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int pair = band / gridDim.x;
  const int b0 = 2 * pair;
  if (!FULL && !pair_active(active, b0, batch)) return;
  const bool w0 = FULL || !active || active[b0];
  const bool w1 = FULL || ((b0 + 1) < batch && (!active || active[b0 + 1]));
  if (FULL) po = nullptr;
  const int o0 = (band - pair * gridDim.x) * (ROWS - 1);  // first output row
  for (int e = threadIdx.x; e < N; e += BLOCK) W[e] = twx[e];
  const size_t plane = (size_t)N * ny;
  const Cx<float>* zp = z + (size_t)pair * plane;
  Cx<float> x[8];
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int t, i;
      fftreg::point<true, LOGN, LOGR, BLOCK, LRL>(q, r, t, i);
      x[q * RL + r] = zp[((size_t)((o0 - 1 + t) & (ny - 1)) << LOGN) + i];
    }
  __syncthreads();
  fftreg::run<true, LOGN, LOGR, BLOCK, +1, true>(x, A, W);
  // p of the band's rows into LDS for the neighbour differences (every read
  // of A by the transform is behind its last barrier)
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int t, i;
      fftreg::point<true, LOGN, LOGR, BLOCK, LR0>(q, r, t, i);
      A[fftreg::lds_at<true, LOGN, LOGR>(i, t)] = x[q * R0 + r];
    }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < (8 * (ROWS - 1) + ROWS - 1) / ROWS; ++k) {
    const int e = k * BLOCK + (int)threadIdx.x;
    if (e >= (ROWS - 1) * N) break;
    const int t = 1 + (e >> LOGN);
    const int i = e & (N - 1);
    const int j = o0 + t - 1;
    if (j >= ny) break;
    const Cx<float> pc = A[fftreg::lds_at<true, LOGN, LOGR>(i, t)];
    const Cx<float> pw = A[fftreg::lds_at<true, LOGN, LOGR>((i - 1) & (N - 1), t)];
    const Cx<float> ps = A[fftreg::lds_at<true, LOGN, LOGR>(i, t - 1)];
    const size_t c0 = (size_t)b0 * plane + ((size_t)j << LOGN) + i;
    if (w0) {
      uo[c0] = us[c0] - (pc.x - pw.x) * idx;
      vo[c0] = vs[c0] - (pc.x - ps.x) * idy;
      if (po) po[c0] = pc.x;
    }
    if (w1) {
      const size_t c1 = c0 + plane;
      uo[c1] = us[c1] - (pc.y - pw.y) * idx;
      vo[c1] = vs[c1] - (pc.y - ps.y) * idy;
      if (po) po[c1] = pc.y;
    }
  }
}

// sin(pi k / n) for 0 <= k < n in FP64: folded onto [0, pi/2] by
// sin(pi k / n) = sin(pi (n - k) / n), then the Taylor series of sin through
// the x^21 term in Horner form on x^2 (the first omitted term is below
// 1.3e-18 at pi/2, under half an ulp of the result)
__device__ __forceinline__ double sin_pi_frac(int k, int n) {
  const int kf = 2 * k > n ? n - k : k;
  const double x = 3.14159265358979323846 * kf / n, x2 = x * x;
  double s = 1.0 / 51090942171709440000.0;                  // 1/21!
  s = fma(s, x2, -1.0 / 121645100408832000.0);              // -1/19!
  s = fma(s, x2, 1.0 / 355687428096000.0);                  // 1/17!
  s = fma(s, x2, -1.0 / 1307674368000.0);                   // -1/15!
  s = fma(s, x2, 1.0 / 6227020800.0);                       // 1/13!
  s = fma(s, x2, -1.0 / 39916800.0);                        // -1/11!
  s = fma(s, x2, 1.0 / 362880.0);                           // 1/9!
  s = fma(s, x2, -1.0 / 5040.0);                            // -1/7!
  s = fma(s, x2, 1.0 / 120.0);                              // 1/5!
  s = fma(s, x2, -1.0 / 6.0);                               // -1/3!
  s = fma(s, x2, 1.0);
  return x * s;
}

// The column pass for FP32 with the transform length N = 2^LOGN (= ny) and
// the column count 2^LOGC known at compile time: the same work as
// k_col_solve (forward FFT along y, the FP64 factor, inverse FFT), with the
// first forward stage fed straight from the global loads, the factor applied
// in registers between the last forward stage and the first inverse stage,
// and the last inverse stage stored straight to global memory (half the LDS
// traffic and a third of the barriers of the general kernel, and index
// arithmetic folded into constants).  One thread per radix-8 butterfly.
// The factor -1 / (lambda_h Nx Ny) is formed in FP64 from the two sin^2
// terms of lambda_h, computed once per workgroup for its columns and for
// every row while the spectrum loads are in flight, instead of read from
// the FP64 table (which costs as many bytes as the spectrum: 11 % faster
// at 1024^2 x 128); the sines come from sin_pi_frac, whose arguments need
// no general range reduction (half the kernel's FP64 instructions of the
// library sine: 7 % faster at 1024^2 x 128).  XCD x takes the column
// groups [x ncx/8, (x+1) ncx/8) of every pair, so the two halves of a
// 128-byte row segment shared by neighbouring groups stay in its L2.
template <int LOGN, int LOGC>
__global__ void __launch_bounds__(((1 << LOGN) << LOGC) / 8) k_col_solve_r(
    Cx<float>* __restrict__ z, const Cx<float>* __restrict__ twy, int nx, int batch,
    const int* active, double ax, double ay, double nrm) {
  constexpr int N = 1 << LOGN, BLOCK = (N << LOGC) / 8;
  constexpr int S = fftreg::plan_stages(LOGN);
  constexpr int R0 = 1 << fftreg::plan_lr(LOGN, 0), RL = 1 << fftreg::plan_lr(LOGN, S - 1);
  __shared__ Cx<float> A[fftreg::lds_elems<false, LOGN, LOGC>()];
  __shared__ Cx<float> W[N];
  __shared__ double LX[1 << LOGC], LY[N];
  const int ncx = nx >> LOGC;
  int cx, pair;
  {
    const int lid = blockIdx.x;
    if ((ncx & 7) == 0) {
      const int cpx = ncx >> 3, slot = lid >> 3;
      const int q = slot / cpx;
      cx = (lid & 7) * cpx + (slot - q * cpx);
      pair = q;
    } else {
      pair = lid / ncx;
      cx = lid - pair * ncx;
    }
  }
  if (!pair_active(active, 2 * pair, batch)) return;
  for (int e = threadIdx.x; e < N; e += BLOCK) W[e] = twy[e];
  const int x0 = cx << LOGC;
  Cx<float>* zp = z + (size_t)pair * nx * N;
  constexpr int LR0 = fftreg::plan_lr(LOGN, 0), LRL = fftreg::plan_lr(LOGN, S - 1);
  Cx<float> x[8];
  double f[8];
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int t, y;
      fftreg::point<false, LOGN, LOGC, BLOCK, LR0>(q, r, t, y);
      x[q * R0 + r] = zp[(size_t)y * nx + x0 + t];
    }
  // the eigenvalue terms (2/dx)^2 sin^2(pi kx/Nx), (2/dy)^2 sin^2(pi ky/Ny)
  // of the workgroup's columns and of every row, in FP64
  for (int e = threadIdx.x; e < N; e += BLOCK) {
    const double sy = sin_pi_frac(e, N);
    LY[e] = ay * sy * sy;
  }
  if (threadIdx.x < (1 << LOGC)) {
    const double sx = sin_pi_frac(x0 + (int)threadIdx.x, nx);
    LX[threadIdx.x] = ax * sx * sx;
  }
  __syncthreads();
  // the factors -1 / (lambda_h Nx Ny) of the points the last forward stage
  // leaves in registers (0 for the zero mode)
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int t, y;
      fftreg::point<false, LOGN, LOGC, BLOCK, LRL>(q, r, t, y);
      f[q * RL + r] = (x0 + t == 0 && y == 0) ? 0.0 : -nrm / (LX[t] + LY[y]);
    }
  fftreg::run<false, LOGN, LOGC, BLOCK, -1, false>(x, A, W);
#pragma unroll
  for (int e = 0; e < 8; ++e)
    x[e] = Cx<float>{(float)((double)x[e].x * f[e]), (float)((double)x[e].y * f[e])};
  fftreg::run<false, LOGN, LOGC, BLOCK, +1, true>(x, A, W);
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int t, y;
      fftreg::point<false, LOGN, LOGC, BLOCK, LR0>(q, r, t, y);
      zp[(size_t)y * nx + x0 + t] = x[q * R0 + r];
    }
}

template <typename T>
__global__ void __launch_bounds__(kRow3Block) k_rowifft_grad(const Cx<T>* __restrict__ z,
                                                         const Cx<T>* __restrict__ twx,
                                                         const T* __restrict__ us,
                                                         const T* __restrict__ vs,
                                                         T* __restrict__ uo, T* __restrict__ vo,
                                                         T* __restrict__ po, int nx, int ny,
                                                         int log2nx, int batch, int rows, T idx,
                                                         T idy, const int* active) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int nr = rows + 1;
  // row bands renumbered so one XCD walks consecutive bands (the halo row
  // of a band is the next band's first row)
  const int band = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int pair = band / gridDim.x;
  const int b0 = 2 * pair;
  if (!pair_active(active, b0, batch)) return;
  const bool w0 = !active || active[b0];
  const bool has1 = (b0 + 1) < batch;
  const bool w1 = has1 && (!active || active[b0 + 1]);
  Cx<T>* P = reinterpret_cast<Cx<T>*>(smem_raw);
  Cx<T>* W = P + nr * nx;
  for (int e = threadIdx.x; e < nx; e += blockDim.x) W[e] = twx[e];
  const int j0 = (band - pair * gridDim.x) * rows;
  const size_t plane = (size_t)nx * ny;
  const Cx<T>* zp = z + (size_t)pair * plane;
  {
    Cx<T> tmp[kRowE3];
#pragma unroll
    for (int k = 0; k < kRowE3; ++k) {
      const int t = k * blockDim.x + threadIdx.x;
      if (t < nr * nx) {
        const int r = t >> log2nx;
        const int i = t & (nx - 1);
        const int j = (j0 - 1 + r + ny) & (ny - 1);
        tmp[k] = zp[(size_t)j * nx + i];
      }
    }
#pragma unroll
    for (int k = 0; k < kRowE3; ++k) {
      const int t = k * blockDim.x + threadIdx.x;
      if (t < nr * nx) P[t] = tmp[k];
    }
  }
  __syncthreads();
  lds_fft<T, kRowE3>(P, nx, log2nx, nr, nx, 1, +1, W);
#pragma unroll
  for (int k = 0; k < kRowE3; ++k) {
    const int t = k * blockDim.x + threadIdx.x;
    if (t >= rows * nx) break;
    const int r = t >> log2nx;
    const int i = t & (nx - 1);
    const int j = j0 + r;
    const int im = (i - 1) & (nx - 1);
    const Cx<T> pc = P[(r + 1) * nx + i];
    const Cx<T> pw = P[(r + 1) * nx + im];
    const Cx<T> ps = P[r * nx + i];
    const size_t c0 = (size_t)b0 * plane + (size_t)j * nx + i;
    if (w0) {
      uo[c0] = us[c0] - (pc.x - pw.x) * idx;
      vo[c0] = vs[c0] - (pc.x - ps.x) * idy;
      if (po) po[c0] = pc.x;
    }
    if (w1) {
      const size_t c1 = c0 + plane;
      uo[c1] = us[c1] - (pc.y - pw.y) * idx;
      vo[c1] = vs[c1] - (pc.y - ps.y) * idy;
      if (po) po[c1] = pc.y;
    }
  }
}

// The whole projection of one pair in one workgroup, for grids whose complex
// pair field fits in LDS (FP32 up to 128 x 128): divergence, FFT along x and
// y, FP64 factor, inverse FFTs and the gradient correction with one read of
// u*, v* and one write of u, v.  Used for the coarse grids of the learned
// solver, where the three-pass version launches too few workgroups to hide
// its latencies.
constexpr int kOneBlock = 1024;

// E: elements per thread (nx * ny <= E * kOneBlock).  With E <= 4 the centre
// values of u*, v* and the Poisson factors stay in registers from the first
// global read to the last use, so the kernel has a single round of global
// loads; with larger E they are re-read at the end.
template <typename T, int E>
__global__ void __launch_bounds__(kOneBlock) k_project_lds(const T* __restrict__ us,
                                                          const T* __restrict__ vs,
                                                          T* __restrict__ uo, T* __restrict__ vo,
                                                          T* __restrict__ po,
                                                          const Cx<T>* __restrict__ twx,
                                                          const Cx<T>* __restrict__ twy,
                                                          const double* __restrict__ pinv, int nx,
                                                          int ny, int log2nx, int log2ny, int batch,
                                                          T idx, T idy, int ra, const int* active) {
  constexpr bool kKeep = E <= 4;
  constexpr int KE = kKeep ? E : 1;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  if (!pair_active(active, 2 * (int)blockIdx.x, batch)) return;
  const bool w0 = !active || active[2 * blockIdx.x];
  const bool w1 = 2 * (int)blockIdx.x + 1 < batch && (!active || active[2 * blockIdx.x + 1]);
  // element (i, j) at j * ra + i: rows padded (ra >= nx) so that the rows a
  // wavefront spans in the row transforms fall into different LDS banks
  Cx<T>* A = reinterpret_cast<Cx<T>*>(smem_raw);
  Cx<T>* Wx = A + ny * ra;
  Cx<T>* Wy = Wx + nx;
  for (int e = threadIdx.x; e < nx; e += blockDim.x) Wx[e] = twx[e];
  for (int e = threadIdx.x; e < ny; e += blockDim.x) Wy[e] = twy[e];
  const int pair = blockIdx.x;
  const int b0 = 2 * pair;
  const int n = nx * ny;
  const size_t plane = (size_t)n;
  const T* u0 = us + (size_t)b0 * plane;
  const T* v0 = vs + (size_t)b0 * plane;
  T cu0[KE], cv0[KE], cu1[KE], cv1[KE];
  double fac[KE];
  // groups of 4 elements per thread: their loads are in flight together
  // without holding all 16 in registers
#pragma unroll
  for (int g = 0; g < E; g += 4) {
    if (g * kOneBlock >= n) break;
    T d0[4], d1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = (g + k) * kOneBlock + (int)threadIdx.x;
      d0[k] = 0;
      d1[k] = 0;
      if (t < n) {
        const int j = t >> log2nx;
        const int i = t & (nx - 1);
        const int ip = (i + 1) & (nx - 1);
        const int jp = (j + 1) & (ny - 1);
        const T a0 = u0[t], c0v = v0[t];
        // a masked-out trajectory of the pair contributes zeros to the
        // packed transform (and is not written)
        if (w0) d0[k] = (u0[j * nx + ip] - a0) * idx + (v0[jp * nx + i] - c0v) * idy;
        T a1 = 0, c1v = 0;
        if (w1) {
          a1 = u0[plane + t];
          c1v = v0[plane + t];
          d1[k] = (u0[plane + j * nx + ip] - a1) * idx + (v0[plane + jp * nx + i] - c1v) * idy;
        }
        if (kKeep) {
          cu0[(g + k) % KE] = a0;
          cv0[(g + k) % KE] = c0v;
          cu1[(g + k) % KE] = a1;
          cv1[(g + k) % KE] = c1v;
          fac[(g + k) % KE] = pinv[t];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = (g + k) * kOneBlock + (int)threadIdx.x;
      if (t < n) A[(t >> log2nx) * ra + (t & (nx - 1))] = Cx<T>{d0[k], d1[k]};
    }
  }
  __syncthreads();
  lds_fft<T, E, true>(A, nx, log2nx, ny, ra, 1, -1, Wx);
  lds_fft<T, E, true>(A, ny, log2ny, nx, 1, ra, -1, Wy);
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int t = k * kOneBlock + (int)threadIdx.x;
    if (t < n) {
      const double s = kKeep ? fac[k % KE] : pinv[t];
      const int a = (t >> log2nx) * ra + (t & (nx - 1));
      const Cx<T> v = A[a];
      A[a] = Cx<T>{(T)((double)v.x * s), (T)((double)v.y * s)};
    }
  }
  __syncthreads();
  lds_fft<T, E, true>(A, ny, log2ny, nx, 1, ra, +1, Wy);
  lds_fft<T, E, true>(A, nx, log2nx, ny, ra, 1, +1, Wx);
#pragma unroll 4
  for (int k = 0; k < E; ++k) {
    const int t = k * kOneBlock + (int)threadIdx.x;
    if (t >= n) break;
    const int j = t >> log2nx;
    const int i = t & (nx - 1);
    const Cx<T> pc = A[j * ra + i];
    const Cx<T> pw = A[j * ra + ((i - 1) & (nx - 1))];
    const Cx<T> ps = A[((j - 1) & (ny - 1)) * ra + i];
    const size_t c0 = (size_t)b0 * plane + t;
    if (w0) {
      uo[c0] = (kKeep ? cu0[k % KE] : us[c0]) - (pc.x - pw.x) * idx;
      vo[c0] = (kKeep ? cv0[k % KE] : vs[c0]) - (pc.x - ps.x) * idy;
      if (po) po[c0] = pc.x;
    }
    if (w1) {
      const size_t c1 = c0 + plane;
      uo[c1] = (kKeep ? cu1[k % KE] : us[c1]) - (pc.y - pw.y) * idx;
      vo[c1] = (kKeep ? cv1[k % KE] : vs[c1]) - (pc.y - ps.y) * idy;
      if (po) po[c1] = pc.y;
    }
  }
}

// the compile-time row passes where they exist (FP32, 64 <= threads <=
// 1024); false: the caller launches the general ones
template <typename T>
bool launch_div_rowfft_r(ldsv_handle* h, const void* us, const void* vs, hipStream_t st,
                         const int* active) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    // 2048 points per workgroup (256 threads; 128 measured slower at
    // 1024^2 x 128, 512 no faster), 8 rows of 1024 (1024 threads: 7 %
    // faster than 2 rows at 1024^2 x 128); fewer rows for small batches
    // until the launch has a workgroup per CU
    int rows = std::max(1, (h->g.nx == 1024 ? 8192 : 2048) / h->g.nx);
    if (rows > h->g.ny) rows = h->g.ny;
    while (rows > 1 && (size_t)(h->g.ny / rows) * h->npairs < 256) rows >>= 1;
    const int logn = h->log2nx, logr = __builtin_ctz((unsigned)rows);
    const dim3 grid(h->g.ny / rows, h->npairs);
    const float idx = (float)(h->g.nx / h->g.lx), idy = (float)(h->g.ny / h->g.ly);
    const bool full = !active && h->g.batch % 2 == 0;
#define LDSV_ROWR(LN, LR)                                                                        \
  if (logn == LN && logr == LR) {                                                                \
    if (full)                                                                                    \
      LDSV_TLAUNCH(h, 1, (k_div_rowfft_r<LN, LR, true>), grid, dim3(((1 << LN) << LR) / 8), 0,    \
                   st, (const float*)us, (const float*)vs, (Cx<float>*)h->zspec,                 \
                   (const Cx<float>*)h->twx, h->g.ny, h->g.batch, idx, idy, active);             \
    else                                                                                         \
      LDSV_TLAUNCH(h, 1, (k_div_rowfft_r<LN, LR>), grid, dim3(((1 << LN) << LR) / 8), 0, st,      \
                   (const float*)us, (const float*)vs, (Cx<float>*)h->zspec,                     \
                   (const Cx<float>*)h->twx, h->g.ny, h->g.batch, idx, idy, active);             \
    return true;                                                                                 \
  }
    LDSV_ROWR(6, 3) LDSV_ROWR(6, 4)
    LDSV_ROWR(7, 2) LDSV_ROWR(7, 3) LDSV_ROWR(7, 4)
    LDSV_ROWR(8, 1) LDSV_ROWR(8, 2) LDSV_ROWR(8, 3) LDSV_ROWR(8, 4)
    LDSV_ROWR(9, 0) LDSV_ROWR(9, 1) LDSV_ROWR(9, 2) LDSV_ROWR(9, 3) LDSV_ROWR(9, 4)
    LDSV_ROWR(10, 0) LDSV_ROWR(10, 1) LDSV_ROWR(10, 2) LDSV_ROWR(10, 3)
    LDSV_ROWR(11, 0) LDSV_ROWR(11, 1) LDSV_ROWR(11, 2)
#undef LDSV_ROWR
    return false;
  }
}

template <typename T>
bool launch_rowifft_grad_r(ldsv_handle* h, const void* us, const void* vs, void* uo, void* vo,
                           void* po, hipStream_t st, const int* active) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    const int logn = h->log2nx;
    const float idx = (float)(h->g.nx / h->g.lx), idy = (float)(h->g.ny / h->g.ly);
    // 8 transformed rows (7 output rows and the halo row) per workgroup, 4 at
    // 2048 (16 measured 13 % slower at 512^2 x 16)
    const int logr = logn >= 11 ? 2 : 3;
    const int outr = (1 << logr) - 1;
    const dim3 grid((h->g.ny + outr - 1) / outr, h->npairs);
    const bool full = !active && h->g.batch % 2 == 0 && !po;
#define LDSV_ROW3R(LN, LR)                                                                       \
  if (logn == LN && logr == LR) {                                                                \
    if (full)                                                                                    \
      LDSV_TLAUNCH(h, 3, (k_rowifft_grad_r<LN, LR, true>), grid, dim3(((1 << LN) << LR) / 8), 0,  \
                   st, (const Cx<float>*)h->zspec, (const Cx<float>*)h->twx, (const float*)us,   \
                   (const float*)vs, (float*)uo, (float*)vo, (float*)po, h->g.ny, h->g.batch,    \
                   idx, idy, active);                                                            \
    else                                                                                         \
      LDSV_TLAUNCH(h, 3, (k_rowifft_grad_r<LN, LR>), grid, dim3(((1 << LN) << LR) / 8), 0, st,    \
                   (const Cx<float>*)h->zspec, (const Cx<float>*)h->twx, (const float*)us,       \
                   (const float*)vs, (float*)uo, (float*)vo, (float*)po, h->g.ny, h->g.batch,    \
                   idx, idy, active);                                                            \
    return true;                                                                                 \
  }
    LDSV_ROW3R(6, 3) LDSV_ROW3R(7, 3) LDSV_ROW3R(8, 3) LDSV_ROW3R(9, 3) LDSV_ROW3R(10, 3)
    LDSV_ROW3R(11, 2)
#undef LDSV_ROW3R
    return false;
  }
}

// the compile-time column pass where it exists (FP32; 512 <= cols * ny <=
// 8192 points per workgroup); false: the caller launches the general one
template <typename T>
bool launch_col_solve_r(ldsv_handle* h, hipStream_t st, const int* active) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    // 4096 points per workgroup (512 threads; 256 or 1024 measured slower at
    // 512^2 x 16 and 1024^2 x 128), narrower column groups for small batches
    // until the launch has a workgroup per CU, but not below 512 points (64
    // threads: at 128^2 x 8 this keeps the compile-time form, 4.9 us against
    // 8.2 us for the general kernel)
    int cols = std::max(1, 4096 / h->g.ny);
    if (cols > h->g.nx) cols = h->g.nx;
    while (cols > 1 && (size_t)(h->g.nx / cols) * h->npairs < 256 && cols * h->g.ny > 512)
      cols >>= 1;
    const int logn = h->log2ny, logc = __builtin_ctz((unsigned)cols);
    const dim3 grid((h->g.nx / cols) * h->npairs);
    const int B = h->g.batch;
    const double dx = h->g.lx / h->g.nx, dy = h->g.ly / h->g.ny;
    const double ax = 4.0 / (dx * dx), ay = 4.0 / (dy * dy);
    const double nrm = 1.0 / ((double)h->g.nx * (double)h->g.ny);
#define LDSV_COLR(LN, LC)                                                                        \
  if (logn == LN && logc == LC) {                                                                \
    LDSV_TLAUNCH(h, 2, (k_col_solve_r<LN, LC>), grid, dim3(((1 << LN) << LC) / 8), 0, st,         \
                 (Cx<float>*)h->zspec, (const Cx<float>*)h->twy, h->g.nx, B, active, ax, ay,     \
                 nrm);                                                                           \
    return true;                                                                                 \
  }
    LDSV_COLR(6, 3) LDSV_COLR(6, 4) LDSV_COLR(6, 5) LDSV_COLR(6, 6)
    LDSV_COLR(7, 2) LDSV_COLR(7, 3) LDSV_COLR(7, 4) LDSV_COLR(7, 5)
    LDSV_COLR(8, 1) LDSV_COLR(8, 2) LDSV_COLR(8, 3) LDSV_COLR(8, 4)
    LDSV_COLR(9, 0) LDSV_COLR(9, 1) LDSV_COLR(9, 2) LDSV_COLR(9, 3)
    LDSV_COLR(10, 0) LDSV_COLR(10, 1) LDSV_COLR(10, 2)
    LDSV_COLR(11, 0) LDSV_COLR(11, 1)
#undef LDSV_COLR
    return false;
  }
}

// The whole projection of one trajectory in one workgroup for square FP32
// grids of 2^LOGN x 2^LOGN cells (32^2, 64^2 and 128^2), with real-input
// transforms of half the length (twice the workgroups of one workgroup per
// trajectory pair for the same work per trajectory: 64 at 64^2 x 64).
//   - u*, v* are read once with 16-byte loads and staged in LDS (the
//     divergence reads its neighbours there; each thread keeps its own
//     values for the final write);
//   - rows 2t and 2t+1 of the divergence form one complex row
//     z_t = d_2t + i d_2t+1 (N/2 row transforms of length N);
//   - the transpose unpacks them, D_2t[kx] = (Z_t[kx] + conj Z_t[N-kx]) / 2,
//     D_2t+1[kx] = (Z_t[kx] - conj Z_t[N-kx]) / 2i, for kx = 1..N/2-1
//     (the other half is their conjugate), and packs the two real columns
//     kx = 0 and kx = N/2 into one complex column: N/2 column transforms;
//   - the FP64 factor multiplies every column in registers; the packed
//     column's two spectra are separated with its ky <-> -ky partner (one
//     LDS exchange) before their factors are applied;
//   - the inverse column transforms, then the packed inverse row transforms
//     W_t = P_2t + i P_2t+1 (Hermitian continuation for kx > N/2), give
//     p_2t + i p_2t+1; p goes to LDS for the differences, and u, v leave with
//     16-byte stores.
// In-place calls are safe: each thread writes only the values it read.
template <int LOGN>
__global__ void __launch_bounds__((1 << (2 * LOGN)) / 16) k_project_real_r(
    const float* __restrict__ us, const float* __restrict__ vs, float* __restrict__ uo,
    float* __restrict__ vo, float* __restrict__ po, const Cx<float>* __restrict__ tw,
    const double* __restrict__ pinv, float idx, float idy, const int* active,
    double* __restrict__ smax) {
  constexpr int N = 1 << LOGN, NH = N / 2, LOGT = LOGN - 1, BLOCK = (N * NH) / 8;
  constexpr int S = fftreg::plan_stages(LOGN);
  constexpr int LR0 = fftreg::plan_lr(LOGN, 0), LRL = fftreg::plan_lr(LOGN, S - 1);
  constexpr int R0 = 1 << LR0, RL = 1 << LRL;
  constexpr int SP = N + 4;   // row stride of the staged u*, v* and of p (floats)
  constexpr int ZS = N + 8;   // row stride of the packed row spectra
  constexpr int QS = NH + 4;  // row stride of the column results
  constexpr int C4 = N / 4;   // 16-byte chunks per row
  constexpr int KC = (N * N / 4) / BLOCK;
  constexpr int kE1 = fftreg::lds_elems<true, LOGN, LOGT>(), kE2 = fftreg::lds_elems<false, LOGN, LOGT>();
  constexpr int kE3 = NH * ZS > N * QS ? NH * ZS : N * QS;
  constexpr int kElems = (kE1 > kE2 ? kE1 : kE2) > kE3 ? (kE1 > kE2 ? kE1 : kE2) : kE3;
  static_assert(KC * BLOCK * 4 == N * N && BLOCK >= N, "thread mapping");
  // LDS: the staged u* (later p), the transform buffer, twiddles, the
  // packed column's values, the factors of the kx = N/2 column, and the
  // staged v* -- which at 128^2 (where the two staged fields and the
  // transform buffer would not fit) shares the transform buffer instead
  constexpr bool kAlias = LOGN >= 7;
  static_assert(N * SP * 4 <= kElems * 8 && (N * SP * 4) % 16 == 0, "LDS layout");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pr[];
  float* su = reinterpret_cast<float*>(smem_pr);
  Cx<float>* A = reinterpret_cast<Cx<float>*>(smem_pr + N * SP * 4);
  Cx<float>* W = A + kElems;
  Cx<float>* X0 = W + N;
  double* F1 = reinterpret_cast<double*>(X0 + N);
  float* sv = kAlias ? reinterpret_cast<float*>(A) : reinterpret_cast<float*>(F1 + N);
  const int b = (int)blockIdx.x;
  if (active && !active[b]) return;  // uniform per workgroup, before any barrier
  const int tid = (int)threadIdx.x;
  constexpr unsigned plane = (unsigned)N * N;
  const float4* u4 = reinterpret_cast<const float4*>(us + (size_t)b * plane);
  const float4* v4 = reinterpret_cast<const float4*>(vs + (size_t)b * plane);
  float4 ku[KC], kv[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    ku[k] = u4[k * BLOCK + tid];
    kv[k] = v4[k * BLOCK + tid];
  }
  // column c of the column transforms is the same for all of a thread's
  // butterflies; column 0 carries kx = 0 and kx = N/2
  const int col = tid & (NH - 1);
  double fac[8];
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int c, ky;
      fftreg::point<false, LOGN, LOGT, BLOCK, LRL>(q, r, c, ky);
      fac[q * RL + r] = pinv[((unsigned)ky << LOGN) + (unsigned)c];
    }
  if (tid < N) {
    W[tid] = tw[tid];
    F1[tid] = pinv[((unsigned)tid << LOGN) + NH];
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int id = k * BLOCK + tid;
    const int y = id / C4, x0 = (id - y * C4) * 4;
    *reinterpret_cast<float4*>(&su[y * SP + x0]) = ku[k];
    *reinterpret_cast<float4*>(&sv[y * SP + x0]) = kv[k];
  }
  __syncthreads();
  // divergence of rows 2t and 2t+1 at the row transform's first-stage points
  Cx<float> x[8];
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int t, i;
      fftreg::point<true, LOGN, LOGT, BLOCK, LR0>(q, r, t, i);
      const int ip = (i + 1) & (N - 1);
      const int y0 = 2 * t * SP, y1 = y0 + SP, y2 = ((2 * t + 2) & (N - 1)) * SP;
      const float d0 = (su[y0 + ip] - su[y0 + i]) * idx + (sv[y1 + i] - sv[y0 + i]) * idy;
      const float d1 = (su[y1 + ip] - su[y1 + i]) * idx + (sv[y2 + i] - sv[y1 + i]) * idy;
      x[q * R0 + r] = Cx<float>{d0, d1};
    }
  if constexpr (kAlias) __syncthreads();  // the staged v* shares the transform's buffer
  fftreg::run<true, LOGN, LOGT, BLOCK, -1, false>(x, A, W);
  // packed row spectra Z_t[kx] to LDS (every LDS read of the transform is
  // behind its last barrier)
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int t, kx;
      fftreg::point<true, LOGN, LOGT, BLOCK, LRL>(q, r, t, kx);
      A[t * ZS + kx] = x[q * RL + r];
    }
  __syncthreads();
  // column inputs at the column transform's first-stage points (c, y)
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int c, y;
      fftreg::point<false, LOGN, LOGT, BLOCK, LR0>(q, r, c, y);
      // operand selects rather than branches (every wavefront holds column
      // 0 and both row parities): with p = Z_t[c], m = Z_t[N - c] (Z_t[N/2]
      // for column 0), D_2t = ((p.x + m.x) / 2, (p.y - m.y) / 2),
      // D_2t+1 = ((p.y + m.y) / 2, (m.x - p.x) / 2), packed (p.x, m.x) or
      // (p.y, m.y)
      const int zt = (y >> 1) * ZS;
      const bool odd = (y & 1) != 0;
      const Cx<float> p = A[zt + c], m = A[zt + (c == 0 ? NH : N - c)];
      const float a = odd ? p.y : p.x, bb = odd ? m.y : m.x;
      const float cc = odd ? m.x : p.y, dd = odd ? p.x : m.y;
      const float ha = c == 0 ? 1.f : 0.5f;
      x[q * R0 + r] = Cx<float>{c == 0 ? a : ha * (a + bb), c == 0 ? bb : ha * (cc - dd)};
    }
  __syncthreads();
  fftreg::run<false, LOGN, LOGT, BLOCK, -1, false>(x, A, W);
  // the packed column's values to LDS for the ky <-> -ky pairing
  if (col == 0) {
#pragma unroll
    for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        int c, ky;
        fftreg::point<false, LOGN, LOGT, BLOCK, LRL>(q, r, c, ky);
        X0[ky] = x[q * RL + r];
      }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int c, ky;
      fftreg::point<false, LOGN, LOGT, BLOCK, LRL>(q, r, c, ky);
      const int e = q * RL + r;
      const Cx<float> v = x[e];
      // column 0: C = A + i B (A, B the spectra of the real columns kx = 0
      // and N/2), f0 A + i f1 B = (f0 + f1)/2 C + (f0 - f1)/2 conj C(-ky);
      // every other column: f C.  X0 and F1 are read by every thread (all of
      // X0 is written above) and the weights selected, rather than branches.
      const Cx<float> m = X0[(N - ky) & (N - 1)];
      const double f0 = fac[e], f1 = F1[ky];
      const double hp = col == 0 ? 0.5 * (f0 + f1) : f0;
      const double hm = col == 0 ? 0.5 * (f0 - f1) : 0.0;
      x[e] = Cx<float>{(float)(hp * (double)v.x + hm * (double)m.x),
                       (float)(hp * (double)v.y - hm * (double)m.y)};
    }
  fftreg::run<false, LOGN, LOGT, BLOCK, +1, true>(x, A, W);
  // column results P[y][c] to LDS by row
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int c, y;
      fftreg::point<false, LOGN, LOGT, BLOCK, LR0>(q, r, c, y);
      A[y * QS + c] = x[q * R0 + r];
    }
  __syncthreads();
  // packed inverse row inputs W_t[kx] = P[2t][kx] + i P[2t+1][kx]
#pragma unroll
  for (int q = 0; q < 8 / RL; ++q)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int t, kx;
      fftreg::point<true, LOGN, LOGT, BLOCK, LRL>(q, r, t, kx);
      const int q0 = 2 * t * QS, q1 = q0 + QS;
      const bool edge = (kx & (NH - 1)) == 0, lo = kx < NH;
      const int mc = edge ? 0 : (lo ? kx : N - kx);
      const Cx<float> a = A[q0 + mc], h = A[q1 + mc];
      const Cx<float> ve = kx == 0 ? Cx<float>{a.x, h.x} : Cx<float>{a.y, h.y};
      const Cx<float> vh = lo ? Cx<float>{a.x - h.y, a.y + h.x} : Cx<float>{a.x + h.y, h.x - a.y};
      x[q * RL + r] = edge ? ve : vh;
    }
  __syncthreads();
  fftreg::run<true, LOGN, LOGT, BLOCK, +1, true>(x, A, W);
  // p (rows 2t, 2t+1) into the staging rows of u* (last read before the
  // first transform)
#pragma unroll
  for (int q = 0; q < 8 / R0; ++q)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      int t, i;
      fftreg::point<true, LOGN, LOGT, BLOCK, LR0>(q, r, t, i);
      su[2 * t * SP + i] = x[q * R0 + r].x;
      su[(2 * t + 1) * SP + i] = x[q * R0 + r].y;
    }
  __syncthreads();
  float4* uo4 = reinterpret_cast<float4*>(uo + (size_t)b * plane);
  float4* vo4 = reinterpret_cast<float4*>(vo + (size_t)b * plane);
  float4* po4 = po ? reinterpret_cast<float4*>(po + (size_t)b * plane) : nullptr;
  double m = 0.0;  // largest |u| + |v| of the thread's cells (smax)
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int id = k * BLOCK + tid;
    const int y = id / C4, x0 = (id - y * C4) * 4;
    const float4 pc = *reinterpret_cast<const float4*>(&su[y * SP + x0]);
    const float4 ps = *reinterpret_cast<const float4*>(&su[((y - 1) & (N - 1)) * SP + x0]);
    const float pw = su[y * SP + ((x0 - 1) & (N - 1))];
    const float4 un{ku[k].x - (pc.x - pw) * idx, ku[k].y - (pc.y - pc.x) * idx,
                    ku[k].z - (pc.z - pc.y) * idx, ku[k].w - (pc.w - pc.z) * idx};
    const float4 vn{kv[k].x - (pc.x - ps.x) * idy, kv[k].y - (pc.y - ps.y) * idy,
                    kv[k].z - (pc.z - ps.z) * idy, kv[k].w - (pc.w - ps.w) * idy};
    uo4[id] = un;
    vo4[id] = vn;
    if (po4) po4[id] = pc;
    if (smax) {
      const float ua[4] = {un.x, un.y, un.z, un.w}, va[4] = {vn.x, vn.y, vn.z, vn.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double sp = (double)fabsf(ua[e]) + (double)fabsf(va[e]);
        m = isfinite(sp) ? fmax(m, sp) : INFINITY;
      }
    }
  }
  if (smax) {  // uniform: the workgroup's maximum, the wavefronts' through F1
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((tid & 63) == 0) F1[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < BLOCK / 64; ++w) m = fmax(m, F1[w]);
      smax[b] = m;
    }
  }
}

// dynamic LDS bytes of k_project_real_r<LOGN>
template <int LOGN>
constexpr size_t project_real_lds() {
  constexpr int N = 1 << LOGN, NH = N / 2, LOGT = LOGN - 1;
  constexpr int kE1 = fftreg::lds_elems<true, LOGN, LOGT>(), kE2 = fftreg::lds_elems<false, LOGN, LOGT>();
  constexpr int kE3 = NH * (N + 8) > N * (NH + 4) ? NH * (N + 8) : N * (NH + 4);
  constexpr int kElems = (kE1 > kE2 ? kE1 : kE2) > kE3 ? (kE1 > kE2 ? kE1 : kE2) : kE3;
  return (size_t)N * (N + 4) * 4 * (LOGN >= 7 ? 1 : 2) + (size_t)kElems * 8 + (size_t)N * (8 + 8 + 8);
}

template <int LOGN>
int launch_project_real(ldsv_handle* h, const void* us, const void* vs, void* uo, void* vo,
                        void* po, hipStream_t st, const int* active) {
  constexpr size_t lds = project_real_lds<LOGN>();
  constexpr int block = (1 << (2 * LOGN)) / 16;
  const float fx = (float)(h->g.nx / h->g.lx), fy = (float)(h->g.ny / h->g.ly);
  LDSV_HIP(hipFuncSetAttribute((const void*)k_project_real_r<LOGN>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  // the rollout guard's per-trajectory speed, when the step asks for it
  double* smax = active ? nullptr : h->speed_now;
  LDSV_TLAUNCH(h, 2, k_project_real_r<LOGN>, dim3(h->g.batch), dim3(block), lds, st,
               (const float*)us, (const float*)vs, (float*)uo, (float*)vo, (float*)po,
               (const Cx<float>*)h->twx, (const double*)h->pinv, fx, fy, active, smax);
  LDSV_LAUNCHED();
  if (smax) h->speed_written = true;
  return LDSV_OK;
}

template <typename T>
int project_impl(ldsv_handle* h, const void* us, const void* vs, void* uo, void* vo, void* po,
                 hipStream_t st, const int* active) {
  const int nx = h->g.nx, ny = h->g.ny, B = h->g.batch;
  const T idx = (T)(nx / h->g.lx), idy = (T)(ny / h->g.ly);
  const size_t cs = sizeof(Cx<T>);
  // one workgroup per trajectory pair holds the whole field in LDS: the
  // fastest path when the grid is small (one HBM round trip), but at 16
  // elements per thread (128^2) a workgroup takes ~50 us of transform
  // latency, so it pays only when the pairs alone fill the chip; otherwise
  // the three passes below spread the work over many more workgroups
  const bool one_block = (size_t)nx * ny <= (size_t)4 * kOneBlock ||
                         ((size_t)nx * ny <= (size_t)16 * kOneBlock && h->npairs >= 256);
  if constexpr (std::is_same<T, float>::value) {
    if (nx == ny && (nx == 32 || nx == 64) && one_block)
      return nx == 64 ? launch_project_real<6>(h, us, vs, uo, vo, po, st, active)
                      : launch_project_real<5>(h, us, vs, uo, vo, po, st, active);
    // 128^2: one 1024-thread workgroup per trajectory
    if (nx == ny && nx == 128)
      return launch_project_real<7>(h, us, vs, uo, vo, po, st, active);
  }
  if (one_block && (size_t)nx * ny * cs <= 131072) {
    // u*, v* are read only by the cells that write u, v at the same index
    // after all reads of neighbours are done (the divergence is formed
    // before the first barrier), so in-place calls are safe here as well
    int ra = nx + lds_row_pad(nx);
    if (((size_t)ny * ra + nx + ny) * cs > 163840) ra = nx;  // padding only within the LDS
    const size_t lds = ((size_t)ny * ra + nx + ny) * cs;
    auto kern = (size_t)nx * ny <= (size_t)4 * kOneBlock ? k_project_lds<T, 4> : k_project_lds<T, 16>;
    LDSV_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    LDSV_TLAUNCH(h, 2, kern, dim3(h->npairs), dim3(kOneBlock), lds, st, (const T*)us,
                 (const T*)vs, (T*)uo, (T*)vo, (T*)po, (const Cx<T>*)h->twx,
                 (const Cx<T>*)h->twy, (const double*)h->pinv, nx, ny, h->log2nx, h->log2ny, B,
                 idx, idy, ra, active);
    LDSV_LAUNCHED();
    return LDSV_OK;
  }
  // pass 1: rows per block (a power of two dividing ny) for kRowE values
  // per thread in blocks of 256 (512 for the longest rows)
  int rows = (kRowE * kBlock) / nx;
  if (rows < 1) rows = 1;
  if (rows > ny) rows = ny;
  // small batches: fewer rows per block until the launch has a workgroup per
  // CU, the block sized to the rows (whole wavefronts)
  while (rows > 1 && (size_t)(ny / rows) * h->npairs < 256) rows >>= 1;
  size_t lds = 0;
  if (!launch_div_rowfft_r<T>(h, us, vs, st, active)) {
    const int need1 = rows * nx / kRowE;
    const int block1 = need1 > kBlock ? kRow1MaxBlock : std::max(64, (need1 + 63) / 64 * 64);
    LDSV_REQUIRE((size_t)rows * nx <= (size_t)kRowE * block1, LDSV_ESHAPE,
                 "project: nx=%d too large for the LDS row transform", nx);
    lds = ((size_t)rows * nx + nx) * cs;
    LDSV_HIP(hipFuncSetAttribute((const void*)k_div_rowfft<T>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    LDSV_TLAUNCH(h, 1, k_div_rowfft<T>, dim3(ny / rows, h->npairs), dim3(block1), lds, st,
                 (const T*)us, (const T*)vs, (Cx<T>*)h->zspec, (const Cx<T>*)h->twx, nx, ny,
                 h->log2nx, B, rows, idx, idy, active);
  }
  LDSV_LAUNCHED();
  // pass 2: 8 columns (fewer for long columns) within kColE * kColBlock
  // values
  // (at most 32 KB of LDS per block, so that four blocks share a CU)
  int cols = 8;
  while (cols > 1 && ((size_t)cols * ny > (size_t)kColE * kColBlock || (size_t)cols * ny * cs > 32768))
    cols >>= 1;
  if (cols > nx) cols = nx;
  // small batches: narrower column groups until the launch has a workgroup
  // per CU (the XCD-contiguous numbering keeps neighbouring groups, which
  // share row segments, on one L2)
  while (cols > 2 && (size_t)(nx / cols) * h->npairs < 256) cols >>= 1;
  LDSV_REQUIRE((size_t)cols * ny <= (size_t)kColE * kColBlock && (size_t)cols * ny * cs <= 65536,
               LDSV_ESHAPE, "project: ny=%d too large for the LDS column transform", ny);
  // 8 values per thread where the block allows it: twice the wavefronts of
  // the minimum, to hide the latency of the transform's LDS round trips
  if (!launch_col_solve_r<T>(h, st, active)) {
    int cblock = (int)(((size_t)cols * ny / 8 + 63) / 64 * 64);
    if (cblock > kColBlock) cblock = kColBlock;
    if (cblock < 64) cblock = 64;
    lds = ((size_t)cols * ny + ny) * cs;
    LDSV_HIP(hipFuncSetAttribute((const void*)k_col_solve<T>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    LDSV_TLAUNCH(h, 2, k_col_solve<T>, dim3((nx / cols) * h->npairs), dim3(cblock), lds, st,
                 (Cx<T>*)h->zspec, (const Cx<T>*)h->twy, (const double*)h->pinv, nx, ny,
                 h->log2ny, __builtin_ctz((unsigned)cols), B, active);
  }
  LDSV_LAUNCHED();
  // pass 3: rows + 1 halo row per block of kRow3Block threads; more rows
  // than pass 1 so the halo row costs less
  if (launch_rowifft_grad_r<T>(h, us, vs, uo, vo, po, st, active)) {
    LDSV_LAUNCHED();
    return LDSV_OK;
  }
  int rows3 = 4096 / nx;
  if (rows3 < 1) rows3 = 1;
  if (rows3 > ny) rows3 = ny;
  // small batches as in pass 1, down to 4 rows per block (the halo row at
  // most a fifth of the block's transforms), the block then sized to them;
  // launches that already have a workgroup per CU keep the full block
  int block3 = kRow3Block;
  if ((size_t)(ny / rows3) * h->npairs < 256) {
    while (rows3 > 4 && (size_t)(ny / rows3) * h->npairs < 256) rows3 >>= 1;
    const int need3 = (rows3 + 1) * nx / kRowE3;
    block3 = std::min(kRow3Block, std::max(64, (need3 + 63) / 64 * 64));
  }
  LDSV_REQUIRE((size_t)(rows3 + 1) * nx <= (size_t)kRowE3 * block3, LDSV_ESHAPE,
               "project: nx=%d too large for the LDS row transform", nx);
  lds = ((size_t)(rows3 + 1) * nx + nx) * cs;
  LDSV_HIP(hipFuncSetAttribute((const void*)k_rowifft_grad<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  LDSV_TLAUNCH(h, 3, k_rowifft_grad<T>, dim3(ny / rows3, h->npairs), dim3(block3), lds, st,
               (const Cx<T>*)h->zspec, (const Cx<T>*)h->twx, (const T*)us, (const T*)vs, (T*)uo,
               (T*)vo, (T*)po, nx, ny, h->log2nx, B, rows3, idx, idy, active);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

}  // namespace

// u*, v* -> projected u, v (may alias u*, v* only if the caller accepts that
// pass 3 reads u*[c] before writing out[c] at the same index, which it does).
int ldsv_launch_project(ldsv_handle* h, const void* us, const void* vs, void* uo, void* vo,
                        void* po, hipStream_t st, const int* active) {
  if (h->g.dtype == LDSV_F64) return project_impl<double>(h, us, vs, uo, vo, po, st, active);
  return project_impl<float>(h, us, vs, uo, vo, po, st, active);
}
