// Compile-time Stockham transforms with register-resident first and last
// stages, for the row and column passes of the spectral Poisson solve (App. B.4,
// S11-S14).
//
// The plan is the one lds_fft follows (radix-8 stages, then radix-4 or
// radix-2 for the remainder), with the length, the number of transforms and
// the block size known at compile time, so every index is a shift or a mask
// of constants.  A forward transform and its inverse run back to back:
//   - the forward transform's first stage takes its inputs in registers
//     (the caller loads them straight from global memory: the inputs of
//     butterfly j are the points j + r N/R, consecutive across lanes);
//   - every stage but the last writes its outputs to LDS and the next stage
//     reads its inputs from there (one exchange per stage boundary);
//   - the forward transform's last stage leaves its outputs in registers at
//     the points j + r N/R, which are exactly the inputs of the first stage
//     of the inverse transform when the inverse takes the stages in reverse
//     order, so the pointwise multiplication in between happens in registers
//     and the two transforms share no LDS round trip;
//   - the inverse transform's last stage leaves its outputs in registers at
//     the points j + r N/R0 (R0 the radix of the forward first stage), the
//     caller's load pattern, for a direct store.
// Each thread holds 8 points: one radix-8 butterfly, two radix-4 or four
// radix-2 ones.  Two layouts of the 2^LOGT transforms:
//   - columns (ROWS false): consecutive lanes take consecutive transforms
//     (the columns of a row-major field, so global loads are row segments);
//     point y of transform t at LDS element (y << LOGT) + t + (y >> 3);
//   - rows (ROWS true): consecutive lanes take consecutive butterflies of
//     one transform (a row, read along x); point y of transform t at
//     t (N + N/8) + y + (y >> 3).
// The pad element every 8 points spreads the strided stage outputs over the
// LDS banks.
#pragma once

#include "fft_lds.h"

namespace fftreg {

constexpr int plan_lr(int logn, int s) {
  int left = logn;
  for (int i = 0;; ++i) {
    const int lr = (left >= 3 && left != 4) ? 3 : (left >= 2 ? 2 : 1);
    if (i == s) return lr;
    left -= lr;
  }
}

constexpr int plan_stages(int logn) {
  int left = logn, n = 0;
  while (left > 0) {
    left -= (left >= 3 && left != 4) ? 3 : (left >= 2 ? 2 : 1);
    ++n;
  }
  return n;
}

// radix log and log2(ns) of stage s, forward order (REV false) or reversed
constexpr int stage_lr(int logn, int s, bool rev) {
  return plan_lr(logn, rev ? plan_stages(logn) - 1 - s : s);
}
constexpr int stage_lns(int logn, int s, bool rev) {
  int a = 0;
  for (int i = 0; i < s; ++i) a += stage_lr(logn, i, rev);
  return a;
}

template <bool ROWS, int LOGN, int LOGT>
__device__ __forceinline__ int lds_at(int y, int t) {
  if constexpr (ROWS)
    return t * ((1 << LOGN) + ((1 << LOGN) >> 3)) + y + (y >> 3);
  else
    return (y << LOGT) + t + (y >> 3);
}

// LDS elements of a buffer of 2^LOGT transforms of length 2^LOGN
template <bool ROWS, int LOGN, int LOGT>
constexpr int lds_elems() {
  if constexpr (ROWS)
    return ((1 << LOGN) + ((1 << LOGN) >> 3)) << LOGT;
  else
    return ((1 << LOGN) << LOGT) + ((1 << LOGN) >> 3) + 1;
}

template <int R>
__device__ __forceinline__ void dft_r(Cx<float>* x, int sign) {
  if constexpr (R == 8)
    dft8(x, sign);
  else if constexpr (R == 4)
    dft4(x[0], x[1], x[2], x[3], sign);
  else
    dft2(x);
}

// butterfly q of the thread in a stage of radix 2^LR: its transform t and
// its index j among the transform's N / R butterflies
template <bool ROWS, int LOGN, int LOGT, int BLOCK, int LR>
__device__ __forceinline__ void bfly(int q, int& t, int& j) {
  const int b = (int)threadIdx.x + q * BLOCK;
  if constexpr (ROWS) {
    j = b & ((1 << (LOGN - LR)) - 1);
    t = b >> (LOGN - LR);
  } else {
    t = b & ((1 << LOGT) - 1);
    j = b >> LOGT;
  }
}

// twiddle and transform the thread's butterflies of stage (LR, LNS)
template <bool ROWS, int LOGN, int LOGT, int BLOCK, int LR, int LNS, int SIGN>
__device__ __forceinline__ void stage_compute(Cx<float> (&x)[8], const Cx<float>* __restrict__ tw) {
  constexpr int R = 1 << LR, BPT = 8 / R, NS = 1 << LNS, LTW = LOGN - LNS - LR;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    int t, j;
    bfly<ROWS, LOGN, LOGT, BLOCK, LR>(q, t, j);
    if constexpr (NS > 1) {
      const int k = j & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const Cx<float> w = tw[(r * k) << LTW];
        x[q * R + r] = SIGN < 0 ? cmul(x[q * R + r], w) : cmulc(x[q * R + r], w);
      }
    }
    dft_r<R>(&x[q * R], SIGN);
  }
}

template <bool ROWS, int LOGN, int LOGT, int BLOCK, int LR, int LNS>
__device__ __forceinline__ void stage_store(const Cx<float> (&x)[8], Cx<float>* A) {
  constexpr int R = 1 << LR, BPT = 8 / R, NS = 1 << LNS;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    int t, j;
    bfly<ROWS, LOGN, LOGT, BLOCK, LR>(q, t, j);
    const int k = j & (NS - 1);
    const int d = ((j - k) << LR) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) A[lds_at<ROWS, LOGN, LOGT>(d + r * NS, t)] = x[q * R + r];
  }
}

template <bool ROWS, int LOGN, int LOGT, int BLOCK, int LR>
__device__ __forceinline__ void stage_load(Cx<float> (&x)[8], const Cx<float>* A) {
  constexpr int R = 1 << LR, BPT = 8 / R, STRIDE = (1 << LOGN) >> LR;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    int t, j;
    bfly<ROWS, LOGN, LOGT, BLOCK, LR>(q, t, j);
#pragma unroll
    for (int r = 0; r < R; ++r) x[q * R + r] = A[lds_at<ROWS, LOGN, LOGT>(j + r * STRIDE, t)];
  }
}

// stages S0.. of a transform (REV: the stages in reverse order) on the
// thread's registers; the first stage's inputs and the last stage's outputs
// stay in registers
template <bool ROWS, int LOGN, int LOGT, int BLOCK, int SIGN, bool REV, int S0 = 0>
__device__ __forceinline__ void run(Cx<float> (&x)[8], Cx<float>* A, const Cx<float>* tw) {
  constexpr int S = plan_stages(LOGN);
  if constexpr (S0 < S) {
    constexpr int LR = stage_lr(LOGN, S0, REV), LNS = stage_lns(LOGN, S0, REV);
    stage_compute<ROWS, LOGN, LOGT, BLOCK, LR, LNS, SIGN>(x, tw);
    if constexpr (S0 + 1 < S) {
      stage_store<ROWS, LOGN, LOGT, BLOCK, LR, LNS>(x, A);
      __syncthreads();
      stage_load<ROWS, LOGN, LOGT, BLOCK, stage_lr(LOGN, S0 + 1, REV)>(x, A);
      __syncthreads();
      run<ROWS, LOGN, LOGT, BLOCK, SIGN, REV, S0 + 1>(x, A, tw);
    }
  }
}

// the points of butterfly q's element r in a stage of radix 2^LR whose
// inputs (first stage) or outputs (last stage) are in registers: point
// j + r N / R of transform t
template <bool ROWS, int LOGN, int LOGT, int BLOCK, int LR>
__device__ __forceinline__ void point(int q, int r, int& t, int& y) {
  int j;
  bfly<ROWS, LOGN, LOGT, BLOCK, LR>(q, t, j);
  y = j + r * ((1 << LOGN) >> LR);
}

}  // namespace fftreg
