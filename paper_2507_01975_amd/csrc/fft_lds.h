// In-LDS batched complex FFT used by the spectral Poisson solve (App. B.4,
// S11-S14).  Stockham autosort formulation with radix-4 stages and one
// radix-2 stage when log2(n) is odd, so the result comes out in natural
// order without a bit-reversal pass.  All threads of the block cooperate on
// `nrows` independent transforms of length n stored row-major in LDS.
#pragma once

#include "internal.h"

// tw[m] = exp(-2 pi i m / n), m in [0, n).  sign = -1 forward, +1 inverse
// (unnormalised).  Returns the buffer (a or b) holding the result.
template <typename T>
__device__ Cx<T>* lds_fft(Cx<T>* a, Cx<T>* b, int n, int log2n, int nrows, int sign,
                          const Cx<T>* __restrict__ tw) {
  int ns = 1;
  int left = log2n;
  while (left > 0) {
    const int radix = (left >= 2) ? 4 : 2;
    const int nb = n / radix;
    const int total = nb * nrows;
    const int twstep = n / (ns * radix);
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int row = t / nb;
      const int j = t - row * nb;
      const Cx<T>* in = a + row * n;
      Cx<T>* out = b + row * n;
      const int k = j & (ns - 1);
      const int d = (j - k) * radix + k;
      if (radix == 4) {
        Cx<T> x0 = in[j], x1 = in[j + nb], x2 = in[j + 2 * nb], x3 = in[j + 3 * nb];
        if (ns > 1) {
          const Cx<T> w1 = tw[k * twstep], w2 = tw[2 * k * twstep], w3 = tw[3 * k * twstep];
          if (sign < 0) {
            x1 = cmul(x1, w1); x2 = cmul(x2, w2); x3 = cmul(x3, w3);
          } else {
            x1 = cmulc(x1, w1); x2 = cmulc(x2, w2); x3 = cmulc(x3, w3);
          }
        }
        const Cx<T> t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3);
        const Cx<T> df = csub(x1, x3);
        // multiply by w^1 of the 4-point DFT: -i (forward) or +i (inverse)
        const Cx<T> t3 = (sign < 0) ? Cx<T>{df.y, -df.x} : Cx<T>{-df.y, df.x};
        out[d] = cadd(t0, t2);
        out[d + ns] = cadd(t1, t3);
        out[d + 2 * ns] = csub(t0, t2);
        out[d + 3 * ns] = csub(t1, t3);
      } else {
        Cx<T> x0 = in[j], x1 = in[j + nb];
        if (ns > 1) {
          const Cx<T> w1 = tw[k * twstep];
          x1 = (sign < 0) ? cmul(x1, w1) : cmulc(x1, w1);
        }
        out[d] = cadd(x0, x1);
        out[d + ns] = csub(x0, x1);
      }
    }
    __syncthreads();
    Cx<T>* tmp = a;
    a = b;
    b = tmp;
    ns *= radix;
    left -= (radix == 4) ? 2 : 1;
  }
  return a;
}
