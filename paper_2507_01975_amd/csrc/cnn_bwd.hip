// Backward pass of the coefficient network on gfx950 matrix cores.
//
// For a layer y = conv3x3(x, W) + b (circular padding) with output cotangent
// g and input x:
//   db[co]          = sum_p g[p][co]
//   dW[co][tap][ci] = sum_p g[p][co] * x[p + tap][ci]            (wgrad)
//   dx[p][ci]       = sum_{tap, co} g[p - tap][co] * W[co][tap][ci]
//                   = conv3x3(g, W')[p][ci],  W'[ci][t][co] = W[co][8 - t][ci]
// and through GELU dz = dx * GELU'(z) with the pre-activation z recomputed
// by a forward pass.  The data gradient reuses the forward implicit-GEMM
// kernel with the flipped, transposed weights and a GELU' epilogue.  The
// weight gradient is a GEMM with the pixels as the reduction dimension: per
// chunk of 32 pixels a workgroup stages g transposed ([co][pixel]) and the 9
// shifted copies of x transposed ([tap, ci][pixel]) in LDS, so both MFMA
// operands are contiguous 8-element pixel runs; each workgroup reduces a
// range of pixels in registers and writes one partial, and a second kernel
// sums the partials in a fixed order (deterministic, no atomics).  Cotangents
// are stored in bf16 between layers, products accumulate in FP32.  The first
// layer (2 input channels) runs on the vector ALUs.
#include "cnn_common.h"

namespace {
using namespace cnnk;

constexpr int kChunk = 32;        // pixels per MFMA K step in wgrad
constexpr int kTRow = kChunk + 8; // padded LDS row of transposed operands
constexpr int kK = 9 * kC;        // 576 = (tap, ci) columns of dW

// gout planar float [B][66][H][W] -> bf16 NHWC [P][96] (channels 66..95 zero),
// transposed through LDS: a workgroup takes 64 consecutive pixels (one
// trajectory's: the pixel count per trajectory is a power of two >= 64),
// reads each channel row of them coalesced and writes each pixel's 96
// channels as twelve 16-byte stores
constexpr int kTP = 64;  // pixels per workgroup
__global__ void __launch_bounds__(kBlock) k_gout_to_nhwc(const float* __restrict__ g,
                                                         uint16_t* __restrict__ G, int hw,
                                                         int total) {
  __shared__ float t[LDSV_NOUT][kTP + 1];
  const int p0 = blockIdx.x * kTP;
  const int b = p0 / hw, r0 = p0 - b * hw;
  const float* gb = g + (size_t)b * LDSV_NOUT * hw + r0;
  for (int i = threadIdx.x; i < LDSV_NOUT * kTP; i += kBlock) {
    const int c = i / kTP, px = i % kTP;
    t[c][px] = (p0 + px < total) ? gb[(size_t)c * hw + px] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTP * 12; i += kBlock) {
    const int px = i / 12, cg = i % 12;
    if (p0 + px >= total) continue;
    uint16_t h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = cg * 8 + j;
      h[j] = f32_to_bf16(c < LDSV_NOUT ? t[c][px] : 0.f);
    }
    uint4 v;
    v.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
    v.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
    v.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
    v.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
    *reinterpret_cast<uint4*>(G + (size_t)(p0 + px) * 96 + cg * 8) = v;
  }
}

// W [cout][9][64] -> W' [64][9][cpad] with W'[ci][t][co] = W[co][8 - t][ci]
__global__ void k_dgrad_weights(const uint16_t* __restrict__ W, uint16_t* __restrict__ Wp, int cout,
                                int cpad) {
  const int total = kC * 9 * cpad;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int ci = e / (9 * cpad);
    const int t = (e / cpad) % 9;
    const int co = e % cpad;
    Wp[e] = (co < cout) ? W[((size_t)co * 9 + (8 - t)) * kC + ci] : (uint16_t)0;
  }
}

// partial dW over the workgroup's pixel range; dz has CS channels, MT tiles.
// Per 32-pixel chunk every thread holds its share of the chunk's operands in
// registers (16-byte loads of 8 channels of one pixel; trip counts fixed at
// compile time, all loads of a chunk in flight together), stores them
// transposed into LDS, and issues the next chunk's loads before the current
// chunk's MFMAs, so that their latency is hidden behind the matrix work.
// Lanes walk the pixels fastest, so the transposing 2-byte LDS stores of a
// wavefront fill consecutive halfwords of one or two rows (rows 8 apart sit
// 32 banks apart): no bank conflicts.
template <int MT, int CS>
__global__ void __launch_bounds__(kBlock) k_wgrad(const uint16_t* __restrict__ dz,
                                                  const uint16_t* __restrict__ x, PixMap pm,
                                                  int wgpix, float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t gT[MT * 16 * kTRow];
  __shared__ __attribute__((aligned(16))) uint16_t xT[kK * kTRow];
  static_assert(MT * 16 <= CS, "the cotangent rows must exist");
  constexpr int kGE = kChunk * (MT * 16 / 8);  // 16-byte cotangent groups per chunk
  constexpr int kXE = kChunk * 9 * (kC / 8);   // 16-byte activation groups per chunk
  static_assert(kXE % kBlock == 0, "chunk staging must tile the block");
  constexpr int kGPer = (kGE + kBlock - 1) / kBlock, kXPer = kXE / kBlock;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  f32x4 acc[MT][9];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < 9; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int p_begin = blockIdx.x * wgpix;
  const int p_end = min(p_begin + wgpix, pm.total);
  uint4 gv[kGPer];
  uint4 xv[kXPer];
  auto load = [&](int p0) {
#pragma unroll
    for (int k = 0; k < kGPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      const int pl = e % kChunk, cq = e / kChunk;
      const int p = p0 + pl;
      gv[k] = uint4{0u, 0u, 0u, 0u};
      if (e < kGE && p < p_end)
        gv[k] = *reinterpret_cast<const uint4*>(dz + (size_t)p * CS + cq * 8);
    }
#pragma unroll
    for (int k = 0; k < kXPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      const int pl = e % kChunk, r = e / kChunk;
      const int tap = r / (kC / 8), q = r % (kC / 8);
      const int p = p0 + pl;
      xv[k] = uint4{0u, 0u, 0u, 0u};
      if (p < p_end) {
        const int src = pm.shift(p, tap / 3 - 1, tap % 3 - 1);
        xv[k] = *reinterpret_cast<const uint4*>(x + (size_t)src * kC + q * 8);
      }
    }
  };
  auto put8 = [](uint16_t* dst, const uint4 v) {
    const uint16_t h[8] = {(uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16),
                           (uint16_t)(v.y & 0xffff), (uint16_t)(v.y >> 16),
                           (uint16_t)(v.z & 0xffff), (uint16_t)(v.z >> 16),
                           (uint16_t)(v.w & 0xffff), (uint16_t)(v.w >> 16)};
#pragma unroll
    for (int i = 0; i < 8; ++i) dst[i * kTRow] = h[i];
  };
  if (p_begin < p_end) load(p_begin);
  for (int p0 = p_begin; p0 < p_end; p0 += kChunk) {
    __syncthreads();  // the previous chunk's fragment reads are done
#pragma unroll
    for (int k = 0; k < kGPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      if (e < kGE) put8(gT + (e / kChunk) * 8 * kTRow + e % kChunk, gv[k]);
    }
#pragma unroll
    for (int k = 0; k < kXPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      const int r = e / kChunk;  // tap * 8 + q: row block 8 r of xT
      put8(xT + r * 8 * kTRow + e % kChunk, xv[k]);
    }
    __syncthreads();
    if (p0 + kChunk < p_end) load(p0 + kChunk);  // in flight during the MFMAs below
    bf16x8 af[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
      af[m] = *reinterpret_cast<const bf16x8*>(gT + (m * 16 + col) * kTRow + kq * 8);
#pragma unroll
    for (int n = 0; n < 9; ++n) {
      const int kcol = (wave * 9 + n) * 16 + col;
      const bf16x8 bf = *reinterpret_cast<const bf16x8*>(xT + kcol * kTRow + kq * 8);
#pragma unroll
      for (int m = 0; m < MT; ++m)
        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m], bf, acc[m][n], 0, 0, 0);
    }
  }
  float* out = partial + (size_t)blockIdx.x * (MT * 16) * kK;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < 9; ++n)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[(size_t)(m * 16 + kq * 4 + i) * kK + (wave * 9 + n) * 16 + col] = acc[m][n][i];
}

// dW[co][k] += sum over partials, in a fixed order: S threads share each
// output, thread s summing the partials s, s + S, ... eight at a time into
// four interleaved running sums (eight loads in flight), and the S sums are
// added in order through LDS; rows of partial = rows.  Outputs per
// workgroup: kBlock / S.
template <int S>
__global__ void __launch_bounds__(kBlock) k_partial_reduce(const float* __restrict__ partial,
                                                           int nblk, int rows, int cout, int ncol,
                                                           float* __restrict__ dW) {
  constexpr int kO = kBlock / S;
  __shared__ float red[S][kO];
  const int o = threadIdx.x % kO, sp = threadIdx.x / kO;
  const int e = blockIdx.x * kO + o;
  float t = 0.f;
  if (e < cout * ncol) {
    const int co = e / ncol, k = e % ncol;
    const size_t stride = (size_t)rows * ncol;
    const float* src = partial + (size_t)co * ncol + k;
    float a[4] = {0.f, 0.f, 0.f, 0.f};
    int b = sp;
    for (; b + 7 * S < nblk; b += 8 * S) {
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i & 3] += src[(size_t)(b + i * S) * stride];
    }
    for (; b < nblk; b += S) a[0] += src[(size_t)b * stride];
    t = (a[0] + a[1]) + (a[2] + a[3]);
  }
  red[sp][o] = t;
  __syncthreads();
  if (sp == 0 && e < cout * ncol) {
    float r = 0.f;
#pragma unroll
    for (int q = 0; q < S; ++q) r += red[q][o];
    dW[e] += r;
  }
}

// launch the reduction of nblk partial blocks into cout x ncol outputs
inline void launch_partial_reduce(ldsv_handle* h, hipStream_t st, const float* part, int nblk,
                                  int rows, int cout, int ncol, float* dW) {
  const int n = cout * ncol;
  if (n >= 16384)
    LDSV_TLAUNCH(h, 7, k_partial_reduce<4>, dim3((n + kBlock / 4 - 1) / (kBlock / 4)),
                 dim3(kBlock), 0, st, part, nblk, rows, cout, ncol, dW);
  else
    LDSV_TLAUNCH(h, 7, k_partial_reduce<16>, dim3((n + kBlock / 16 - 1) / (kBlock / 16)),
                 dim3(kBlock), 0, st, part, nblk, rows, cout, ncol, dW);
}

// bias gradient partials from the bf16 NHWC cotangent of a 64-channel layer:
// a workgroup sums kBiasPix pixels; thread t accumulates channels
// 8 (t % 8) .. +7 (one 16-byte load per pixel) over pixels t / 8 + 32 k, and
// the 32 pixel lanes are then added in a fixed order through LDS
constexpr int kBiasPix = 512;
__global__ void __launch_bounds__(kBlock) k_bias_partial(const uint16_t* __restrict__ dz,
                                                         int total, float* __restrict__ partial) {
  __shared__ float red[32][kC + 1];
  const int q = threadIdx.x & 7, r = threadIdx.x >> 3;
  const int p0 = blockIdx.x * kBiasPix;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int p = p0 + r; p < min(p0 + kBiasPix, total); p += 32) {
    const uint4 v = *reinterpret_cast<const uint4*>(dz + (size_t)p * kC + q * 8);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s[2 * i] += bf16_to_f32((uint16_t)(w[i] & 0xffffu));
      s[2 * i + 1] += bf16_to_f32((uint16_t)(w[i] >> 16));
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) red[r][q * 8 + i] = s[i];
  __syncthreads();
  if (threadIdx.x < kC) {
    float t = 0.f;
    for (int k = 0; k < 32; ++k) t += red[k][threadIdx.x];
    partial[(size_t)blockIdx.x * kC + threadIdx.x] = t;
  }
}

// the same for the float planar network-output cotangent [B][66][H][W]:
// workgroup (x, c) sums pixels [x kBiasPix, ...) of channel c
__global__ void __launch_bounds__(kBlock) k_bias_partial_planar(const float* __restrict__ g,
                                                                int hw, int total,
                                                                float* __restrict__ partial) {
  __shared__ float red[kBlock];
  const int c = blockIdx.y;
  const int p0 = blockIdx.x * kBiasPix;
  float s = 0.f;
  for (int p = p0 + (int)threadIdx.x; p < min(p0 + kBiasPix, total); p += kBlock) {
    const int b = p / hw, rr = p - b * hw;
    s += g[((size_t)b * LDSV_NOUT + c) * hw + rr];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * LDSV_NOUT + c] = red[0];
}

// first layer: partial dW0[co][tap][ci] over a pixel range (VALU)
__global__ void __launch_bounds__(kBlock) k_wgrad_first(const uint16_t* __restrict__ dz1,
                                                        const float* __restrict__ u,
                                                        const float* __restrict__ v, PixMap pm,
                                                        int wgpix, float* __restrict__ partial) {
  __shared__ float sx[kChunk][18];
  __shared__ float sg[kChunk][kC];
  // staging as in k_wgrad: registers first (compile-time trip counts), the
  // next chunk's loads issued before the current chunk's products
  constexpr int kSX = kChunk * 18, kSXPer = (kSX + kBlock - 1) / kBlock;
  constexpr int kSG = kChunk * kC, kSGPer = kSG / kBlock;
  static_assert(kSG % kBlock == 0, "chunk staging must tile the block");
  const int p_begin = blockIdx.x * wgpix;
  const int p_end = min(p_begin + wgpix, pm.total);
  float xr[kSXPer];
  uint16_t gr[kSGPer];
  auto load = [&](int p0) {
#pragma unroll
    for (int k = 0; k < kSXPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      xr[k] = 0.f;
      if (e < kSX) {
        const int pl = e / 18, kk = e % 18;
        const int p = p0 + pl;
        if (p < p_end) {
          const int tap = kk / 2;
          const int src = pm.shift(p, tap / 3 - 1, tap % 3 - 1);
          xr[k] = bf16_to_f32(f32_to_bf16((kk & 1) ? v[src] : u[src]));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kSGPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      const int pl = e / kC, c = e % kC;
      const int p = p0 + pl;
      gr[k] = (p < p_end) ? dz1[(size_t)p * kC + c] : (uint16_t)0;
    }
  };
  // thread owns outputs e = threadIdx.x + k * 256 (< 64 * 18 = 1152)
  float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (p_begin < p_end) load(p_begin);
  for (int p0 = p_begin; p0 < p_end; p0 += kChunk) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSXPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      if (e < kSX) sx[e / 18][e % 18] = xr[k];
    }
#pragma unroll
    for (int k = 0; k < kSGPer; ++k) {
      const int e = k * kBlock + (int)threadIdx.x;
      sg[e / kC][e % kC] = bf16_to_f32(gr[k]);
    }
    __syncthreads();
    if (p0 + kChunk < p_end) load(p0 + kChunk);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e < kC * 18) {
        const int co = e / 18, kk = e % 18;
        float s = 0.f;
        for (int pl = 0; pl < kChunk; ++pl) s += sg[pl][co] * sx[pl][kk];
        acc[k] += s;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int e = threadIdx.x + k * kBlock;
    if (e < kC * 18) partial[(size_t)blockIdx.x * kC * 18 + e] = acc[k];
  }
}

// first layer data gradient: gu[p] = sum_{tap, co} dz1[p - tap][co] W1[co][tap][0]
__global__ void __launch_bounds__(kBlock) k_dgrad_first(const uint16_t* __restrict__ dz1,
                                                        const uint16_t* __restrict__ W1, PixMap pm,
                                                        float* __restrict__ gu, float* __restrict__ gv) {
  __shared__ float w[kC * 18];
  for (int e = threadIdx.x; e < kC * 18; e += blockDim.x) w[e] = bf16_to_f32(W1[e]);
  __syncthreads();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pm.total) return;
  float su = 0.f, sv = 0.f;
  for (int tap = 0; tap < 9; ++tap) {
    const int q = pm.shift(p, -(tap / 3 - 1), -(tap % 3 - 1));
    const uint16_t* g = dz1 + (size_t)q * kC;
    for (int co = 0; co < kC; ++co) {
      const float gg = bf16_to_f32(g[co]);
      su += gg * w[(co * 9 + tap) * 2];
      sv += gg * w[(co * 9 + tap) * 2 + 1];
    }
  }
  gu[p] = su;
  gv[p] = sv;
}

}  // namespace

int ldsv_launch_cnn_backward(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                             const float* gout, float* gu, float* gv, const ldsv_net_grad* dW,
                             hipStream_t st) {
  const size_t P = h->nstate;
  // weight-gradient workgroups: about one per CU, each reducing a range of
  // whole 32-pixel chunks
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int wgpix = (int)(((P + ncu - 1) / ncu + kChunk - 1) / kChunk * kChunk);
  const int nwg = (int)((P + wgpix - 1) / wgpix);
  const int nbias = (int)((P + kBiasPix - 1) / kBiasPix);
  const int npart = nwg > nbias ? nwg : nbias;
  // workspace: 5 pre-activation planes (float NHWC 64), G (bf16 96), two dz
  // buffers (bf16 64), W' (bf16 64 x 9 x 96), wgrad partials
  if (!h->zpre_blk) {
    const size_t bytes = 5 * P * kC * 4 + P * 96 * 2 + 2 * P * kC * 2 + (size_t)kC * 9 * 96 * 2 +
                         (size_t)npart * 80 * kK * 4 + 256;
    LDSV_TRY(ldsv_alloc(h, &h->zpre_blk, bytes, "network backward workspace"));
  }
  char* w = (char*)h->zpre_blk;
  float* zpre[5];
  for (int l = 0; l < 5; ++l) zpre[l] = (float*)(w + (size_t)l * P * kC * 4);
  uint16_t* G = (uint16_t*)(w + 5 * P * kC * 4);
  uint16_t* dzA = G + P * 96;
  uint16_t* dzB = dzA + P * kC;
  uint16_t* Wp = dzB + P * kC;
  float* part = (float*)((char*)(Wp + (size_t)kC * 9 * 96) + 0);
  part = (float*)(((uintptr_t)part + 255) & ~(uintptr_t)255);
  PixMap pm{h->g.ny, h->g.nx, (int)P};
  const int hw = (int)h->ncell;
  const int nblk_conv = (int)((P + kPixPerBlock - 1) / kPixPerBlock);

  // forward recompute with pre-activations
  LDSV_TRY(ldsv_launch_cnn(h, net, u, v, h->netout, zpre, st));
  // layer 6: bias from the float cotangent, G = bf16 NHWC copy
  hipLaunchKernelGGL(k_bias_partial_planar, dim3(nbias, LDSV_NOUT), dim3(kBlock), 0, st, gout, hw,
                     (int)P, part);
  launch_partial_reduce(h, st, part, nbias, LDSV_NOUT, LDSV_NOUT, 1, dW->b[5]);
  hipLaunchKernelGGL(k_gout_to_nhwc, dim3((unsigned)((P + kTP - 1) / kTP)), dim3(kBlock), 0, st,
                     gout, G, hw, (int)P);
  LDSV_LAUNCHED();
  {
    LDSV_TLAUNCH(h, 4, (k_wgrad<5, 96>), dim3(nwg), dim3(kBlock), 0, st, G, h->act[4], pm, wgpix,
                 part);
  }
  launch_partial_reduce(h, st, part, nwg, 80, LDSV_NOUT, kK, dW->w[5]);
  LDSV_TLAUNCH(h, 7, k_dgrad_weights, grid1d((size_t)kC * 9 * 96), dim3(kBlock), 0, st, net->w[5],
                     Wp, LDSV_NOUT, 96);
  LDSV_LAUNCHED();
  {
    LDSV_TLAUNCH(h, 4, (k_conv3x3_mfma<4, 2, 96>), dim3(nblk_conv), dim3(kBlock), 0, st, G, Wp,
                       (const float*)nullptr, kC, pm, dzA, zpre[4], (float*)nullptr);
  }
  LDSV_LAUNCHED();
  uint16_t* dz = dzA;
  uint16_t* dzn = dzB;
  // layers 5..2 (index 4..1): dz is the cotangent of layer index li's pre-activation
  for (int li = 4; li >= 1; --li) {
    LDSV_TLAUNCH(h, 7, k_bias_partial, dim3(nbias), dim3(kBlock), 0, st, dz, (int)P, part);
    launch_partial_reduce(h, st, part, nbias, kC, kC, 1, dW->b[li]);
    LDSV_TLAUNCH(h, 4, (k_wgrad<4, 64>), dim3(nwg), dim3(kBlock), 0, st, dz, h->act[li - 1], pm,
                 wgpix, part);
    launch_partial_reduce(h, st, part, nwg, 64, kC, kK, dW->w[li]);
    LDSV_TLAUNCH(h, 7, k_dgrad_weights, grid1d((size_t)kC * 9 * 64), dim3(kBlock), 0, st,
                       net->w[li], Wp, kC, 64);
    if (h->g.nx % 16 == 0 && h->g.ny % 16 == 0)
      LDSV_TRY(ldsv_launch_conv_tile(h, 4, 2, dz, Wp, nullptr, kC, dzn, zpre[li - 1], nullptr, st));
    else
      LDSV_TLAUNCH(h, 4, (k_conv3x3_mfma<4, 2, 64>), dim3(nblk_conv), dim3(kBlock), 0, st, dz, Wp,
                   (const float*)nullptr, kC, pm, dzn, zpre[li - 1], (float*)nullptr);
    LDSV_LAUNCHED();
    uint16_t* t = dz;
    dz = dzn;
    dzn = t;
  }
  // layer 1
  LDSV_TLAUNCH(h, 7, k_bias_partial, dim3(nbias), dim3(kBlock), 0, st, dz, (int)P, part);
  launch_partial_reduce(h, st, part, nbias, kC, kC, 1, dW->b[0]);
  {
    // its 1152 outputs are summed on the vector ALUs from LDS: four times
    // the workgroups of the MFMA layers, each over a quarter of the pixels,
    // so that more waves hide the LDS latency (the partials, nwg1 x 1152
    // floats, fit the buffer sized for nwg x 80 x 576)
    const int wgpix1 = wgpix / 4 > kChunk ? (wgpix / 4 + kChunk - 1) / kChunk * kChunk : kChunk;
    const int nwg1 = (int)((P + wgpix1 - 1) / wgpix1);
    LDSV_TLAUNCH(h, 7, k_wgrad_first, dim3(nwg1), dim3(kBlock), 0, st, dz, u, v, pm, wgpix1, part);
    launch_partial_reduce(h, st, part, nwg1, kC * 18, kC * 18, 1, dW->w[0]);
  }
  LDSV_LAUNCHED();
  if (gu && gv) {
    LDSV_TLAUNCH(h, 7, k_dgrad_first, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, dz, net->w[0], pm, gu, gv);
    LDSV_LAUNCHED();
  }
  return LDSV_OK;
}
