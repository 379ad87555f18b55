// Deterministic per-trajectory FP64 reductions: each block reduces a slice of
// one trajectory with wavefront shuffles (64 lanes) and LDS, writes a partial,
// and a second kernel combines the partials of each trajectory in a fixed
// order.  No atomics, so results are bitwise reproducible.
#pragma once

#include "internal.h"

constexpr int kRedSum = 0;
constexpr int kRedMax = 1;

template <int OP>
__device__ __forceinline__ double red_op(double a, double b) {
  return OP == kRedSum ? a + b : fmax(a, b);
}

template <int OP>
__device__ __forceinline__ double red_init() {
  return OP == kRedSum ? 0.0 : -1.0e308;
}

template <int OP>
__device__ double block_reduce(double v) {
  __shared__ double part[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = red_op<OP>(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) part[w] = v;
  __syncthreads();
  double r = red_init<OP>();
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = red_op<OP>(r, part[i]);
  }
  __syncthreads();
  return r;  // valid in thread 0
}

// f(b, idx) -> double value for cell idx of trajectory b; NV values per cell
template <int OP, int NV, class F>
__global__ void __launch_bounds__(kBlock) k_reduce_partial(F f, size_t n, double* partial,
                                                           int nblk) {
  const int b = blockIdx.y;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = red_init<OP>();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)nblk * blockDim.x) {
    double v[NV];
    f(b, idx, v);
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = red_op<OP>(acc[k], v[k]);
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double r = block_reduce<OP>(acc[k]);
    if (threadIdx.x == 0) partial[((size_t)b * NV + k) * nblk + blockIdx.x] = r;
  }
}

template <int OP, int NV>
__global__ void k_reduce_final(const double* partial, int nblk, double* out) {
  const int b = blockIdx.x;
  for (int k = threadIdx.x; k < NV; k += blockDim.x) {
    double r = red_init<OP>();
    const double* p = partial + ((size_t)b * NV + k) * nblk;
    for (int i = 0; i < nblk; ++i) r = red_op<OP>(r, p[i]);
    out[(size_t)b * NV + k] = r;
  }
}

// Reduce NV values per cell over n cells for each of `batch` trajectories
// into out[b][NV] (device).  Uses h->red as partial storage.
template <int OP, int NV, class F>
int reduce_per_traj(ldsv_handle* h, F f, size_t n, int batch, double* out, hipStream_t st) {
  int nblk = (int)((n + kBlock - 1) / kBlock);
  if (nblk > 64) nblk = 64;
  if ((size_t)nblk * NV * batch > h->red_len) {
    nblk = (int)(h->red_len / ((size_t)NV * batch));
    if (nblk < 1) {
      ldsv_set_error("reduction scratch too small");
      return LDSV_ENOMEM;
    }
  }
  hipLaunchKernelGGL((k_reduce_partial<OP, NV, F>), dim3(nblk, batch), dim3(kBlock), 0, st, f, n,
                     h->red, nblk);
  LDSV_LAUNCHED();
  hipLaunchKernelGGL((k_reduce_final<OP, NV>), dim3(batch), dim3(64), 0, st, h->red, nblk, out);
  LDSV_LAUNCHED();
  return LDSV_OK;
}
