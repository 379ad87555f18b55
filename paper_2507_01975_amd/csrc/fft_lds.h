// In-LDS batched complex FFT used by the spectral Poisson solve (App. B.4,
// S11-S14).
//
// Stockham autosort formulation (natural-order output, no bit reversal)
// with radix-8 stages and one radix-4 or radix-2 stage when log2(n) is not a
// multiple of 3.  Each stage is done in place in one LDS buffer: every thread
// first loads the inputs of its butterflies into registers, the block
// synchronises, then every thread twiddles, transforms in registers and
// stores its outputs, and the block synchronises again.  The buffer holds
// `nrows` transforms of length n; element j of transform r lives at
// buf[r * rs + j * es] (rs and es powers of two, or any values below 2^24
// with PAD).  Threads walk the elements with the unit-stride
// index fastest (j when es == 1, r otherwise), so each wavefront reads and
// writes consecutive LDS words.
#pragma once

#include "internal.h"

// Row padding (in elements) for a buffer of rows of n points whose rows are
// transformed by lds_fft: with n / R butterflies per row a wavefront pass
// spans several rows, and rows a power of two apart share LDS banks.  n / 8
// extra elements per row put the rows of a pass n / 4 (FP32) or n / 2
// (FP64) banks apart: no conflicts for n = 64 and for the 16-butterfly stage
// of n = 128, at most two-way for n = 32; rows of 256 or more points fill a
// pass on their own.
__host__ __device__ inline int lds_row_pad(int n) { return (n >= 32 && n <= 128) ? n / 8 : 0; }

template <typename T>
__device__ __forceinline__ Cx<T> mul_i(Cx<T> a, int sign) {
  // multiply by -i (sign < 0) or +i (sign > 0)
  return sign < 0 ? Cx<T>{a.y, -a.x} : Cx<T>{-a.y, a.x};
}

template <typename T>
__device__ __forceinline__ void dft2(Cx<T>* x) {
  const Cx<T> a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft4(Cx<T>& x0, Cx<T>& x1, Cx<T>& x2, Cx<T>& x3, int sign) {
  const Cx<T> t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3);
  const Cx<T> t3 = mul_i(csub(x1, x3), sign);
  x0 = cadd(t0, t2);
  x1 = cadd(t1, t3);
  x2 = csub(t0, t2);
  x3 = csub(t1, t3);
}

// 8-point DFT: two 4-point DFTs of the even and odd samples, combined with
// the 8th roots of unity exp(sign * 2 pi i k / 8)
template <typename T>
__device__ __forceinline__ void dft8(Cx<T>* x, int sign) {
  Cx<T> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  Cx<T> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4(e0, e1, e2, e3, sign);
  dft4(o0, o1, o2, o3, sign);
  const T h = (T)0.70710678118654752440;
  // o1 *= w8^1, o2 *= w8^2, o3 *= w8^3
  if (sign < 0) {
    o1 = Cx<T>{h * (o1.x + o1.y), h * (o1.y - o1.x)};
    o3 = Cx<T>{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
  } else {
    o1 = Cx<T>{h * (o1.x - o1.y), h * (o1.x + o1.y)};
    o3 = Cx<T>{-h * (o3.x + o3.y), h * (o3.x - o3.y)};
  }
  o2 = mul_i(o2, sign);
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1);
  x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);
  x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);
  x[7] = csub(e3, o3);
}

// One Stockham stage of radix R (LR = log2 R) over all butterflies of the
// block; E is the compile-time bound on elements per thread
// (nrows * n <= E * blockDim).  n, the stage sizes and, for strided
// transforms (es != 1), nrows are powers of two passed as base-2 logarithms,
// so index arithmetic is shifts and masks: the vector ALU time of these
// kernels is comparable to their memory time.  With PAD the row and element
// strides rs and es are any values below 2^24 (24-bit multiplies), so that
// a caller can pad the rows of its buffer: with short rows a wavefront
// spans several rows, and rows a power of two apart fall into the same LDS
// banks; without PAD they are powers of two (shifts).  Row transforms
// (es == 1) take any nrows (the gradient pass transforms a halo row more).
template <typename T, int R, int LR, int E, bool PAD>
__device__ __forceinline__ void fft_stage(Cx<T>* buf, int log2n, int nrows, int log2nrows, int rs,
                                          int es, int log2ns, int sign,
                                          const Cx<T>* __restrict__ tw) {
  const int lrs = PAD ? 0 : __builtin_ctz((unsigned)rs), les = PAD ? 0 : __builtin_ctz((unsigned)es);
  auto at = [&](int row, int x) {
    return PAD ? __umul24(row, rs) + __umul24(x, es) : (row << lrs) + (x << les);
  };
  constexpr int BPT = (E / R) > 0 ? (E / R) : 1;  // butterflies per thread
  const int lnb = log2n - LR;                      // log2 of butterflies per transform
  const int total = nrows << lnb;
  const int ns = 1 << log2ns;
  const int ltw = log2n - log2ns - LR;             // twiddle stride n / (ns R)
  Cx<T> x[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int t = threadIdx.x + q * blockDim.x;
    if (t < total) {
      int row, j;
      if (es == 1) {
        row = t >> lnb;
        j = t & ((1 << lnb) - 1);
      } else {
        j = t >> log2nrows;
        row = t & ((1 << log2nrows) - 1);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) x[q][r] = buf[at(row, j + (r << lnb))];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int t = threadIdx.x + q * blockDim.x;
    if (t < total) {
      int row, j;
      if (es == 1) {
        row = t >> lnb;
        j = t & ((1 << lnb) - 1);
      } else {
        j = t >> log2nrows;
        row = t & ((1 << log2nrows) - 1);
      }
      const int k = j & (ns - 1);
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const Cx<T> w = tw[(r * k) << ltw];
          x[q][r] = sign < 0 ? cmul(x[q][r], w) : cmulc(x[q][r], w);
        }
      }
      if (R == 8) dft8(x[q], sign);
      else if (R == 4) dft4(x[q][0], x[q][1], x[q][2], x[q][3], sign);
      else dft2(x[q]);
      const int d = ((j - k) << LR) + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[at(row, d + (r << log2ns))] = x[q][r];
    }
  }
  __syncthreads();
}

// Full transform (sign -1 forward, +1 inverse, unnormalised), in place, of
// the nrows transforms of length n = 2^log2n (nrows a power of two when
// es != 1).
// tw[m] = exp(-2 pi i m / n), a table the caller has copied into LDS (every
// stage reads it, and a global-memory latency per stage would serialise the
// transform).  The caller synchronises before the call.
template <typename T, int E, bool PAD = false>
__device__ __forceinline__ void lds_fft(Cx<T>* buf, int n, int log2n, int nrows, int rs, int es,
                                        int sign, const Cx<T>* __restrict__ tw) {
  (void)n;
  const int log2nrows = es == 1 ? 0 : __builtin_ctz((unsigned)nrows);
  int log2ns = 0;
  int left = log2n;
  while (left > 0) {
    if (left >= 3 && left != 4) {
      fft_stage<T, 8, 3, E, PAD>(buf, log2n, nrows, log2nrows, rs, es, log2ns, sign, tw);
      log2ns += 3;
      left -= 3;
    } else if (left >= 2) {
      fft_stage<T, 4, 2, E, PAD>(buf, log2n, nrows, log2nrows, rs, es, log2ns, sign, tw);
      log2ns += 2;
      left -= 2;
    } else {
      fft_stage<T, 2, 1, E, PAD>(buf, log2n, nrows, log2nrows, rs, es, log2ns, sign, tw);
      log2ns += 1;
      left -= 1;
    }
  }
}
