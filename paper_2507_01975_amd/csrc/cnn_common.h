// Device code shared by the forward and backward network kernels: bf16
// helpers, the periodic pixel map and the implicit-GEMM 3x3 convolution on
// v_mfma_f32_16x16x32_bf16 (see cnn.hip for the design).
#pragma once

#include "cnn.h"

namespace cnnk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 64;             // hidden channels
constexpr int kPixPerWave = 64;    // 4 pixel tiles of 16
constexpr int kPixPerBlock = 256;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// round-to-nearest-even float -> bf16 of two values, packed low | high << 16
// (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const bf16x2 b = __builtin_convertvector((f32x2{lo, hi}), bf16x2);
  return __builtin_bit_cast(uint32_t, b);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  return (uint16_t)(pack_bf16x2(f, 0.0f) & 0xffffu);
}

// the float value of f rounded to bf16 (the storage precision of the
// network's stencil-coefficient outputs)
__device__ __forceinline__ float round_to_bf16(float f) {
  return __uint_as_float(((uint32_t)f32_to_bf16(f)) << 16);
}

// erfc(x) for x >= 0 by the Chebyshev-fitted form of Press et al.,
// Numerical Recipes (sec. 6.2, erfcc): t exp(-x^2 + P(t)), t = 1/(1 + x/2),
// fractional error below 1.2e-7 in exact arithmetic; in float32 the error is
// dominated by the rounding of -x^2 + P(t), about 1e-6 relative for x < 6.
// Fewer than half the instructions of erff (used by the GELU derivative of
// the backward kernels).
__device__ __forceinline__ float erfc_pos(float x) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  return t * __expf(fmaf(-x, x, p));
}

// standard normal CDF Phi(z) = erfc(-z / sqrt 2) / 2
__device__ __forceinline__ float normal_cdf(float z) {
  const float e = 0.5f * erfc_pos(fabsf(z) * 0.70710678118654752f);
  return z >= 0.0f ? 1.0f - e : e;
}

// exact (erf) GELU: z Phi(z) = max(z, 0) - |z| Q(|z|), Q(a) = Phi(-a) the
// normal upper tail, taken as 2^P(a) with P the degree-10 least-squares
// Chebyshev fit of log2 Q on [0, 6] written in powers of a (the fit and its
// error: gen_gelu_poly.py beside this file): relative error of Q below
// 1.3e-6 for a < 3 and 4.4e-6 up to 6 in float32, |GELU error| below 7e-8;
// Q(6) ~ 1e-9 stands in beyond.  Ten FMAs, one exp2, two med3 clamps and
// one FMA: the forward epilogues' vector-ALU work is dominated by this
// function (the erfc form above costs a reciprocal, an exponential and
// eighteen more instructions).  Non-finite z gives a non-finite result.
__device__ __forceinline__ float gelu_exact(float z) {
  const float a = __builtin_amdgcn_fmed3f(fabsf(z), 0.0f, 6.0f);
  float p = -1.149826456e-08f;
  p = fmaf(p, a, 3.878143104e-07f);
  p = fmaf(p, a, -5.562967999e-06f);
  p = fmaf(p, a, 4.235186861e-05f);
  p = fmaf(p, a, -1.504010288e-04f);
  p = fmaf(p, a, -3.018268617e-04f);
  p = fmaf(p, a, 7.375738584e-03f);
  p = fmaf(p, a, -5.279443413e-02f);
  p = fmaf(p, a, -4.590685666e-01f);
  p = fmaf(p, a, -1.151131988e+00f);
  p = fmaf(p, a, -9.999987483e-01f);
  return fmaf(-fabsf(z), __builtin_amdgcn_exp2f(p), __builtin_amdgcn_fmed3f(z, 0.0f, 3.0e38f));
}

// d/dz of the exact GELU: Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_grad(float z) {
  return normal_cdf(z) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// Output channel computed by row r of 16 x 16 accumulator block m in the
// 64-output layers.  Blocks 0 and 1 hold channels 0..31 and blocks 2 and 3
// channels 32..63, interleaved in groups of four, so that the rows 4q..4q+3
// a lane holds in blocks 2h and 2h+1 are the eight consecutive channels
// 32h + 8q .. 32h + 8q + 7 of its pixel: one 16-byte store of bf16 values
// (two per pixel and lane, each pixel row written in 64-byte pieces).
__device__ __forceinline__ constexpr int out_chan(int m, int r) {
  return ((m >> 1) << 5) + ((r >> 2) << 3) + ((m & 1) << 2) + (r & 3);
}

struct PixMap {
  int H, W;   // powers of two
  int total;  // B * H * W
  // pixel p moved by (dy, dx) with periodic wrap within its trajectory;
  // trajectory, row and column by shifts and masks (no integer division)
  __device__ __forceinline__ int shift(int p, int dy, int dx) const {
    const int hw = H * W;
    const int lw = __builtin_ctz(W), lhw = __builtin_ctz(hw);
    const int y = (p & (hw - 1)) >> lw;
    const int x = p & (W - 1);
    return ((p >> lhw) << lhw) + ((y + dy) & (H - 1)) * W + ((x + dx) & (W - 1));
  }
};

// MT: output-channel tiles of 16.  CIN: input channels (multiple of 32).
// EPI 0: z = acc + bias -> gelu -> bf16 NHWC [P][64] (and z float NHWC if zout)
// EPI 1: z = acc + bias -> float planar [B][cout][H][W], channels below
//        LDSV_NCOEF rounded to bf16 values (the coefficient storage precision)
// EPI 3 (tiled kernel only): channels below LDSV_NCOEF -> bf16 in blocks of
//        8 channels Y [B][8][H][W][8], the rest -> float planar out_planar
// EPI 2: g = acc * gelu'(zin[p][c]) -> bf16 NHWC [P][64] (data gradient)
template <int MT, int EPI, int CIN>
__global__ void __launch_bounds__(kBlock) k_conv3x3_mfma(const uint16_t* __restrict__ X,
                                                         const uint16_t* __restrict__ Wt,
                                                         const float* __restrict__ bias, int cout,
                                                         PixMap pm, uint16_t* __restrict__ Y,
                                                         float* __restrict__ zio,
                                                         float* __restrict__ out_planar) {
  constexpr int kWRow = CIN + 8;  // padded LDS weight row (bf16 elements)
  __shared__ __attribute__((aligned(16))) uint16_t wl[MT * 16 * kWRow];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int pbase = blockIdx.x * kPixPerBlock + wave * kPixPerWave;
  const int col = lane & 15;   // pixel within a tile / channel row within an A tile
  const int kq = lane >> 4;    // which 8-wide K slice

  f32x4 acc[4][MT];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[t][m] = f32x4{0.f, 0.f, 0.f, 0.f};

  int pix[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int p = pbase + t * 16 + col;
    pix[t] = p < pm.total ? p : pm.total - 1;
  }

  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    __syncthreads();
    // stage W[:, tap, :] (cout x CIN bf16) into LDS rows of kWRow; rows past
    // cout are zero
    for (int e = threadIdx.x; e < MT * 16 * (CIN / 8); e += blockDim.x) {
      const int row = e / (CIN / 8), q = e - row * (CIN / 8);
      uint4 v = {0u, 0u, 0u, 0u};
      if (row < cout) v = *reinterpret_cast<const uint4*>(Wt + ((size_t)row * 9 + tap) * CIN + q * 8);
      *reinterpret_cast<uint4*>(wl + row * kWRow + q * 8) = v;
    }
    __syncthreads();
    int src[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) src[t] = pm.shift(pix[t], dy, dx);
#pragma unroll
    for (int half = 0; half < CIN / 32; ++half) {
      const int cbase = half * 32 + kq * 8;
      bf16x8 bfrag[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        bfrag[t] = *reinterpret_cast<const bf16x8*>(X + (size_t)src[t] * CIN + cbase);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const bf16x8 afrag = *reinterpret_cast<const bf16x8*>(wl + (m * 16 + col) * kWRow + cbase);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag[t], acc[t][m], 0, 0, 0);
      }
    }
  }

  // epilogue: lane holds channels m*16 + 4*kq + i of pixel pbase + t*16 + col
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int p = pbase + t * 16 + col;
    if (p >= pm.total) continue;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int c0 = m * 16 + kq * 4;
      if (EPI == 0 || EPI == 2) {
        float z[4];
        float h[4];
        if (EPI == 2) {
          const float4 zi = *reinterpret_cast<const float4*>(zio + (size_t)p * kC + c0);
          const float zz[4] = {zi.x, zi.y, zi.z, zi.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) h[i] = acc[t][m][i] * gelu_grad(zz[i]);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            z[i] = acc[t][m][i] + bias[c0 + i];
            h[i] = gelu_exact(z[i]);
          }
        }
        uint2 pk;
        pk.x = pack_bf16x2(h[0], h[1]);
        pk.y = pack_bf16x2(h[2], h[3]);
        *reinterpret_cast<uint2*>(Y + (size_t)p * kC + c0) = pk;
        if (EPI == 0 && zio)
          *reinterpret_cast<float4*>(zio + (size_t)p * kC + c0) = float4{z[0], z[1], z[2], z[3]};
      } else {
        const int hw = pm.H * pm.W;
        const int b = p / hw;
        const int r = p - b * hw;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = c0 + i;
          const float z = acc[t][m][i] + bias[c];
          if (c < cout)
            out_planar[((size_t)b * cout + c) * hw + r] = c < LDSV_NCOEF ? round_to_bf16(z) : z;
        }
      }
    }
  }
}

// Persistent loops: slot s = g + k G is the k-th tile of workgroup g (grid G).
// Workgroups reach the 8 XCDs round-robin by id, so the slot is renumbered to
// give XCD x = g % 8 the contiguous tile range [x T/8, (x+1) T/8): the tiles of one
// image, whose halos overlap, are then in flight on one XCD at the same time
// and the shared halo rows come from its L2 once.  A bijection of [0, T) (the
// identity unless 8 divides both T and G).
__device__ __forceinline__ int xcd_slot_tile(int s, int T, int G) {
  if ((T & 7) || (G & 7)) return s;
  const int g = s % G, k = s / G;
  return (g & 7) * (T >> 3) + k * (G >> 3) + (g >> 3);
}

// The same convolution for grids whose sides are multiples of 16, as a
// persistent kernel (used for the 66-output last layer; the 64-output layers
// use k_conv3x3_dma below): a workgroup first stages the layer's whole weight
// matrix (cout padded to 16 MT rows x 576 bf16) in
// LDS, then loops over 16-row pixel tiles TW pixels wide; for each tile it
// stages the tile with its 1-pixel periodic halo (18 x (TW + 2) pixels x 64
// channels) and runs all 9 taps from LDS.  In both LDS arrays 16-byte chunk
// c of row r sits at chunk position c ^ (r & 7), which puts the rows that
// one fragment read touches in distinct banks (row padding, 144-byte tile
// rows, measured 3.7e6 bank-conflict cycles per launch; the swizzle none).
// LDS: 132 KB for 80 padded outputs and 16-wide tiles, one workgroup per CU.  (32-wide tiles, which halve the weight-fragment traffic
// per pixel, need more than the 256 registers two wavefronts per SIMD allow
// and were slower.)
//
// Eight wavefronts, wavefront w computing tile rows 2w and 2w+1 for every
// output channel.  The epilogue (bias-initialised accumulators, bf16
// rounding and the scattered stores of the coefficient blocks and planes)
// costs vector-ALU time comparable to the tile's matrix-core time, so the wavefronts are split into two groups
// that share each SIMD (w and w + 4 run on the same SIMD): group 0
// accumulates tile k and then runs its epilogue, group 1 first runs the
// epilogue of tile k-1 (its accumulators carried across the tile barrier) and
// then accumulates tile k.  On every SIMD one wavefront's MFMAs overlap the
// other's vector work.
constexpr int kConvBlock = 512;
constexpr int kWRowAll = 9 * kC;       // weight row (bf16 elements), swizzled chunks
constexpr int kTileRow = kC;           // tile pixel row, swizzled chunks
constexpr int kTileH = 18;             // 16 rows + halo

// TW: tile width in pixels (16 or 32); the staged tile is 18 x (TW + 2)
template <int MT, int TW>
constexpr size_t conv_tile_lds_bytes() {
  return (size_t)(MT * 16 * kWRowAll + kTileH * (TW + 2) * kTileRow) * 2;
}

template <int MT, int EPI, int TW>
__global__ void __launch_bounds__(kConvBlock) k_conv3x3_tile(const uint16_t* __restrict__ X,
                                                             const uint16_t* __restrict__ Wt,
                                                             const float* __restrict__ bias,
                                                             int cout, PixMap pm,
                                                             uint16_t* __restrict__ Y,
                                                             float* __restrict__ zio,
                                                             float* __restrict__ out_planar) {
  static_assert(MT == 5 && (EPI == 1 || EPI == 3), "the 66-output last layer");
  // output channel of row r of accumulator block m: for the bf16 blocks
  // (EPI 3) the first 64 in the order of the 64-output layers, the rest in
  // order; in order for the float planes (EPI 1), whose stores are per
  // channel anyway
  auto chan = [](int m, int r) { return EPI == 3 && m < 4 ? out_chan(m, r) : m * 16 + r; };
  extern __shared__ __attribute__((aligned(16))) uint16_t lds_u16[];
  uint16_t* wl = lds_u16;
  uint16_t* xt = lds_u16 + MT * 16 * kWRowAll;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = wave >> 2;
  const int col = lane & 15;
  const int kq = lane >> 4;
  constexpr int kTW = TW + 2;        // staged tile width
  constexpr int kNX = TW / 16;       // 16-pixel groups per tile row
  constexpr int NT = 2 * kNX;        // pixel tiles of 16 per wavefront
  const int tiles_x = pm.W / TW, tiles_y = pm.H / 16;
  const int ntiles = (pm.total / (pm.H * pm.W)) * tiles_x * tiles_y;
  const int hw = pm.H * pm.W;
  // whole weight matrix, once; loads are issued in batches before the LDS
  // stores so their latencies overlap
  {
    constexpr int kChunks = MT * 16 * (9 * kC / 8);
    constexpr int kBatch = 4;
    for (int e0 = 0; e0 < kChunks; e0 += kBatch * kConvBlock) {
      uint4 v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int e = e0 + k * kConvBlock + (int)threadIdx.x;
        const int row = e / (9 * kC / 8), q = e - row * (9 * kC / 8);
        v[k] = uint4{0u, 0u, 0u, 0u};
        if (e < kChunks && row < cout)
          v[k] = *reinterpret_cast<const uint4*>(Wt + (size_t)row * 9 * kC + q * 8);
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int e = e0 + k * kConvBlock + (int)threadIdx.x;
        const int row = e / (9 * kC / 8), q = e - row * (9 * kC / 8);
        if (e < kChunks)
          *reinterpret_cast<uint4*>(wl + row * kWRowAll + ((q ^ (row & 7)) << 3)) = v[k];
      }
    }
  }
  // the tile with its halo is loaded into registers one tile ahead (the
  // loads of tile k+1 are in flight while tile k is computed), then stored
  // to LDS between two barriers
  constexpr int kTChunks = kTileH * kTW * (kC / 8);
  constexpr int kTPer = (kTChunks + kConvBlock - 1) / kConvBlock;
  uint4 tv[kTPer];
  auto load_tile = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y);
    const int tr = tile - b * tiles_x * tiles_y;
    const int y0 = (tr / tiles_x) * 16, x0 = (tr % tiles_x) * TW;
#pragma unroll
    for (int k = 0; k < kTPer; ++k) {
      const int e = k * kConvBlock + (int)threadIdx.x;
      tv[k] = uint4{0u, 0u, 0u, 0u};
      if (e < kTChunks) {
        const int px = e / (kC / 8), q = e - px * (kC / 8);
        const int ry = px / kTW, rx = px - ry * kTW;
        const int gy = (y0 - 1 + ry) & (pm.H - 1), gx = (x0 - 1 + rx) & (pm.W - 1);
        tv[k] = *reinterpret_cast<const uint4*>(X + ((size_t)b * hw + gy * pm.W + gx) * kC + q * 8);
      }
    }
  };
  f32x4 acc[NT][MT];
  // accumulate the staged tile: pixel tile t covers row 2 wave + t / kNX,
  // columns 16 (t % kNX) .. +15; bias-initialised (EPI 0, 1)
  auto mma = [&]() {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      f32x4 b0 = f32x4{0.f, 0.f, 0.f, 0.f};
      if (EPI != 2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = chan(m, kq * 4 + i);
          b0[i] = c < cout ? bias[c] : 0.f;
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][m] = b0;
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int q = half * 4 + kq;
        bf16x8 bfrag[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int ry = wave * 2 + t / kNX + 1 + dy, rx = (t % kNX) * 16 + col + 1 + dx;
          const int px = ry * kTW + rx;
          bfrag[t] = *reinterpret_cast<const bf16x8*>(xt + px * kTileRow + ((q ^ (px & 7)) << 3));
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const int row = chan(m, col);
          const bf16x8 afrag = *reinterpret_cast<const bf16x8*>(
              wl + row * kWRowAll + (((tap * 8 + q) ^ (row & 7)) << 3));
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[t][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag[t], acc[t][m], 0, 0, 0);
        }
      }
    }
  };
  auto epilogue = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y);
    const int tr = tile - b * tiles_x * tiles_y;
    const int y0 = (tr / tiles_x) * 16, x0 = (tr % tiles_x) * TW;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int y = y0 + wave * 2 + t / kNX, x = x0 + (t % kNX) * 16 + col;
      const int r = y * pm.W + x;
      if (EPI == 1) {
        // all 66 channels as float planes, the 64 stencil coefficients
        // rounded to bf16 values
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = chan(m, kq * 4 + i);
            const float z = acc[t][m][i];
            if (c < cout)
              out_planar[((size_t)b * cout + c) * hw + r] = c < LDSV_NCOEF ? round_to_bf16(z) : z;
          }
        }
      } else {
        // EPI 3: the 64 stencil coefficients in bf16, blocks of 8 channels
        // [B][8][H][W][8] (blocks 2hh and 2hh+1 give a lane the 8 channels
        // of one block entry: one 16-byte store), the 2 correction channels
        // as float planes [B][2][H][W]
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int c0 = hh * 32 + kq * 8;
          const f32x4 a0 = acc[t][2 * hh], a1 = acc[t][2 * hh + 1];
          uint4 pk;
          pk.x = pack_bf16x2(a0[0], a0[1]);
          pk.y = pack_bf16x2(a0[2], a0[3]);
          pk.z = pack_bf16x2(a1[0], a1[1]);
          pk.w = pack_bf16x2(a1[2], a1[3]);
          *reinterpret_cast<uint4*>(Y + (((size_t)b * 8 + (c0 >> 3)) * hw + r) * 8) = pk;
        }
#pragma unroll
        for (int m = 4; m < MT; ++m) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = m * 16 + kq * 4 + i;
            if (c >= LDSV_NCOEF && c < cout)
              out_planar[((size_t)b * (LDSV_NOUT - LDSV_NCOEF) + (c - LDSV_NCOEF)) * hw + r] =
                  acc[t][m][i];
          }
        }
      }
    }
  };
  const int G = gridDim.x;
  if ((int)blockIdx.x < ntiles) load_tile(xcd_slot_tile(blockIdx.x, ntiles, G));
  int prev = -1;
  for (int s = blockIdx.x; s < ntiles; s += G) {
    const int tile = xcd_slot_tile(s, ntiles, G);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTPer; ++k) {
      const int e = k * kConvBlock + (int)threadIdx.x;
      if (e < kTChunks) {
        const int px = e / (kC / 8), q = e - px * (kC / 8);
        *reinterpret_cast<uint4*>(xt + px * kTileRow + ((q ^ (px & 7)) << 3)) = tv[k];
      }
    }
    __syncthreads();
    if (s + G < ntiles) load_tile(xcd_slot_tile(s + G, ntiles, G));
    if (grp == 1 && prev >= 0) epilogue(prev);
    mma();
    if (grp == 0) epilogue(tile);
    prev = tile;
  }
  if (grp == 1 && prev >= 0) epilogue(prev);
}

// The 64-output layers (and their data gradients) with the tiles brought
// into LDS by the load-to-LDS path (global_load_lds_dwordx4: each lane's 16
// bytes go straight to LDS at the instruction's base + 16 x lane, no
// registers), double-buffered: while tile k is multiplied, tile k+1 is in
// flight.  Without the register staging of k_conv3x3_tile the loads of a
// tile overlap all of the previous tile's work and the loop needs one
// barrier per tile.  Eight wavefronts, rows 2w and 2w+1 of the tile each, in
// the same two phase-shifted groups as k_conv3x3_tile.  The LDS rows are not
// padded (two tiles and the weights must fit in 160 KB): 16-byte chunk c of
// row r sits at chunk position c ^ (r & 7), which spreads the 8 rows of every
// fragment read over all banks; the load-to-LDS path writes chunk positions
// in lane order, so the swizzle is applied to the source addresses.
// LDS: 72 KB weights + 2 x 40.5 KB tiles.
constexpr int kDmaTile = 18 * 18 * kC;  // bf16 elements per staged tile

constexpr size_t conv_dma_lds_bytes() { return (size_t)(kC * 9 * kC + 2 * kDmaTile) * 2; }

typedef __attribute__((address_space(3))) void lds_void;

//
// L1 (inference of the second layer): the staged tile is not read from the
// first layer's output but computed in place from u, v: the first layer
// (2 -> 64 channels, one K = 32 step per 16 halo pixels, bias, GELU, bf16
// rounding, the same operands and operations as k_conv_first, so the tile
// holds the same values bit for bit) evaluated on the tile's 18 x 18 halo
// pixels, its 16-byte chunks written to the swizzled LDS positions.  The
// first layer's activations then never go through HBM (33.5 MB written and
// read back at 64^2 x 64) and its launch disappears, for 27 % of recomputed
// halo pixels; X is unused.
template <int EPI, bool L1 = false>
__global__ void __launch_bounds__(kConvBlock) k_conv3x3_dma(const uint16_t* __restrict__ X,
                                                            const uint16_t* __restrict__ Wt,
                                                            const float* __restrict__ bias,
                                                            PixMap pm, uint16_t* __restrict__ Y,
                                                            float* __restrict__ zio,
                                                            const float* __restrict__ u1,
                                                            const float* __restrict__ v1,
                                                            const uint16_t* __restrict__ W1,
                                                            const float* __restrict__ b1) {
  static_assert(!L1 || EPI == 0, "the fused first layer is an inference forward");
  extern __shared__ __attribute__((aligned(16))) uint16_t lds_u16[];
  uint16_t* wl = lds_u16;                   // [64][576], swizzled chunks
  uint16_t* xbuf = lds_u16 + kC * 9 * kC;   // two tiles [18 * 18][64], swizzled
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = wave >> 2;
  const int col = lane & 15;
  const int kq = lane >> 4;
  const int tiles_x = pm.W / 16, tiles_y = pm.H / 16;
  const int ntiles = (pm.total / (pm.H * pm.W)) * tiles_x * tiles_y;
  const int hw = pm.H * pm.W;
  // weights: slot (row, pos) receives logical chunk pos ^ (row & 7);
  // 64 x 72 chunks = 72 instructions of 64 lanes, 9 per wavefront
  for (int i = wave; i < kC * 72 / 64; i += kConvBlock / 64) {
    const int e = i * 64 + lane;
    const int row = e / 72, pos = e - row * 72;
    const int c = pos ^ (row & 7);
    __builtin_amdgcn_global_load_lds((const void*)(Wt + ((size_t)row * 72 + c) * 8),
                                     (lds_void*)(wl + (size_t)i * 64 * 8), 16, 0, 0);
  }
  // tile t into buffer s: 18 x 18 pixels x 8 chunks = 2592 slots, 40.5
  // instructions of 64 lanes over the 8 wavefronts (lanes past the end idle)
  constexpr int kTChunks = 18 * 18 * 8;
  constexpr int kTInst = (kTChunks + 63) / 64;
  // first layer (L1): the weights of the lane's A rows (channel
  // out_chan(m, col), K entries 8 kq .. 8 kq + 7 of the 18) and the bias of
  // its accumulator rows, once
  bf16x8 a1[4];
  f32x4 bias1[4];
  if constexpr (L1) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int co = out_chan(m, col);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kq * 8 + e;
        a1[m][e] = __builtin_bit_cast(__bf16, k < 18 ? W1[co * 18 + k] : (uint16_t)0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) bias1[m][i] = b1[out_chan(m, kq * 4 + i)];
    }
  }
  // L1: the 21 groups of 16 of the tile's 324 halo pixels, groups w, w + 8,
  // w + 16 on wavefront w; each lane gathers the u, v of its K entries
  // (taps 4 kq .. 4 kq + 3) for its pixel of every group first, then
  // multiplies, applies GELU and writes its two 16-byte chunks
  constexpr int kL1Groups = (18 * 18 + 15) / 16;
  constexpr int kL1PerWave = (kL1Groups + kConvBlock / 64 - 1) / (kConvBlock / 64);
  auto make_tile = [&](int tile, int sbuf) {
    const int b = tile / (tiles_x * tiles_y);
    const int tr = tile - b * tiles_x * tiles_y;
    const int y0 = (tr / tiles_x) * 16, x0 = (tr % tiles_x) * 16;
    uint16_t* dst = xbuf + sbuf * kDmaTile;
    const float* ub = u1 + (size_t)b * hw;
    const float* vb = v1 + (size_t)b * hw;
    bf16x8 bf[kL1PerWave];
#pragma unroll
    for (int k = 0; k < kL1PerWave; ++k) {
      const int g = wave + k * (kConvBlock / 64);
      const int px = g * 16 + col;
      const int ry = px / 18, rx = px - ry * 18;
      const int gy = y0 - 1 + ry, gx = x0 - 1 + rx;
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const int tap = (kq * 8 + e) / 2;
        float a = 0.f, c = 0.f;
        if (g < kL1Groups && px < 18 * 18 && tap < 9) {
          const int q = ((gy + tap / 3 - 1) & (pm.H - 1)) * pm.W + ((gx + tap % 3 - 1) & (pm.W - 1));
          a = ub[q];
          c = vb[q];
        }
        const uint32_t pk = pack_bf16x2(a, c);
        bf[k][e] = __builtin_bit_cast(__bf16, (uint16_t)(pk & 0xffffu));
        bf[k][e + 1] = __builtin_bit_cast(__bf16, (uint16_t)(pk >> 16));
      }
    }
#pragma unroll
    for (int k = 0; k < kL1PerWave; ++k) {
      const int g = wave + k * (kConvBlock / 64);
      const int px = g * 16 + col;
      if (g >= kL1Groups) continue;  // uniform per wavefront
      f32x4 z[4];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        z[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[m], bf[k], bias1[m], 0, 0, 0);
      if (px < 18 * 18) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const f32x4 q0 = z[2 * hh], q1 = z[2 * hh + 1];
          uint4 pk;
          pk.x = pack_bf16x2(gelu_exact(q0[0]), gelu_exact(q0[1]));
          pk.y = pack_bf16x2(gelu_exact(q0[2]), gelu_exact(q0[3]));
          pk.z = pack_bf16x2(gelu_exact(q1[0]), gelu_exact(q1[1]));
          pk.w = pack_bf16x2(gelu_exact(q1[2]), gelu_exact(q1[3]));
          const int chunk = hh * 4 + kq;  // channels 8 chunk .. 8 chunk + 7
          *reinterpret_cast<uint4*>(dst + px * kC + ((chunk ^ (px & 7)) << 3)) = pk;
        }
      }
    }
  };
  auto issue_tile = [&](int tile, int sbuf) {
    if constexpr (L1) {
      [[clang::always_inline]] make_tile(tile, sbuf);
      return;
    }
    const int b = tile / (tiles_x * tiles_y);
    const int tr = tile - b * tiles_x * tiles_y;
    const int y0 = (tr / tiles_x) * 16, x0 = (tr % tiles_x) * 16;
    uint16_t* dst = xbuf + sbuf * kDmaTile;
    for (int i = wave; i < kTInst; i += kConvBlock / 64) {
      const int e = i * 64 + lane;
      if (e < kTChunks) {
        const int px = e >> 3, pos = e & 7;
        const int ry = px / 18, rx = px - ry * 18;
        const int gy = (y0 - 1 + ry) & (pm.H - 1), gx = (x0 - 1 + rx) & (pm.W - 1);
        const int q = pos ^ (px & 7);
        __builtin_amdgcn_global_load_lds(
            (const void*)(X + ((size_t)b * hw + gy * pm.W + gx) * kC + q * 8),
            (lds_void*)(dst + (size_t)i * 64 * 8), 16, 0, 0);
      }
    }
  };
  f32x4 acc[2][4];
  auto mma = [&](const uint16_t* xt) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      f32x4 b0 = f32x4{0.f, 0.f, 0.f, 0.f};
      if (EPI != 2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) b0[i] = bias[out_chan(m, kq * 4 + i)];
      }
      acc[0][m] = b0;
      acc[1][m] = b0;
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int q = half * 4 + kq;
        bf16x8 bfrag[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int px = (wave * 2 + t + 1 + dy) * 18 + col + 1 + dx;
          bfrag[t] = *reinterpret_cast<const bf16x8*>(xt + px * kC + ((q ^ (px & 7)) << 3));
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int row = out_chan(m, col);
          const int c = tap * 8 + q;
          const bf16x8 afrag =
              *reinterpret_cast<const bf16x8*>(wl + row * 576 + ((c ^ (row & 7)) << 3));
          acc[0][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag[0], acc[0][m], 0, 0, 0);
          acc[1][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag[1], acc[1][m], 0, 0, 0);
        }
      }
    }
  };
  auto epilogue = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y);
    const int tr = tile - b * tiles_x * tiles_y;
    const int y0 = (tr / tiles_x) * 16, x0 = (tr % tiles_x) * 16;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const size_t p = (size_t)b * hw + (size_t)(y0 + wave * 2 + t) * pm.W + x0 + col;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        // blocks 2hh and 2hh+1: channels c0 .. c0 + 7 (out_chan)
        const int c0 = hh * 32 + kq * 8;
        const f32x4 a0 = acc[t][2 * hh], a1 = acc[t][2 * hh + 1];
        const float z[8] = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        float h[8];
        if (EPI == 2) {
          const float4 zi0 = *reinterpret_cast<const float4*>(zio + p * kC + c0);
          const float4 zi1 = *reinterpret_cast<const float4*>(zio + p * kC + c0 + 4);
          const float zz[8] = {zi0.x, zi0.y, zi0.z, zi0.w, zi1.x, zi1.y, zi1.z, zi1.w};
#pragma unroll
          for (int i = 0; i < 8; ++i) h[i] = z[i] * gelu_grad(zz[i]);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) h[i] = gelu_exact(z[i]);
        }
        uint4 pk;
        pk.x = pack_bf16x2(h[0], h[1]);
        pk.y = pack_bf16x2(h[2], h[3]);
        pk.z = pack_bf16x2(h[4], h[5]);
        pk.w = pack_bf16x2(h[6], h[7]);
        *reinterpret_cast<uint4*>(Y + p * kC + c0) = pk;
        if (EPI == 0 && zio) {
          *reinterpret_cast<float4*>(zio + p * kC + c0) = float4{z[0], z[1], z[2], z[3]};
          *reinterpret_cast<float4*>(zio + p * kC + c0 + 4) = float4{z[4], z[5], z[6], z[7]};
        }
      }
    }
  };
  const int G = gridDim.x;
  int sbuf = 0;
  if ((int)blockIdx.x < ntiles) [[clang::always_inline]] issue_tile(xcd_slot_tile(blockIdx.x, ntiles, G), 0);
  int prev = -1;
  for (int s = blockIdx.x; s < ntiles; s += G) {
    const int tile = xcd_slot_tile(s, ntiles, G);
    // this wavefront's loads of the current tile (and, the first time, of
    // the weights) have landed; after the barrier everyone's have, and every
    // wavefront is done reading the other buffer
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const bool more = s + G < ntiles;
    const int next = more ? xcd_slot_tile(s + G, ntiles, G) : 0;
    if constexpr (!L1) {
      if (more) [[clang::always_inline]] issue_tile(next, sbuf ^ 1);
    }
    if (grp == 1 && prev >= 0) epilogue(prev);
    // L1: each group computes its share of the next tile while the other
    // group's wavefront on the same SIMD multiplies (group 1 before its
    // MFMAs, group 0 after its epilogue); the next barrier publishes it
    if constexpr (L1) {
      if (grp == 1 && more) [[clang::always_inline]] make_tile(next, sbuf ^ 1);
    }
    mma(xbuf + sbuf * kDmaTile);
    if (grp == 0) epilogue(tile);
    if constexpr (L1) {
      if (grp == 0 && more) [[clang::always_inline]] make_tile(next, sbuf ^ 1);
    }
    prev = tile;
    sbuf ^= 1;
  }
  if (grp == 1 && prev >= 0) epilogue(prev);
}

}  // namespace cnnk
