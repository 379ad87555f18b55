// The coefficient network on gfx950 matrix cores.
//
// Six 3x3 convolutions with circular padding (periodic BC padding, App. B.1),
// 2 -> 64 -> 64 -> 64 -> 64 -> 64 -> 66 channels, bias, exact GELU after the
// first five (the learnable part of the flux block in per-cell form, Sec.
// 3.4).  Activations are bf16 NHWC ([B][H][W][64], channels fastest); the
// output is float planar [B][66][H][W] (64 raw stencil values + 2 TC).
//
// Layers 2..6 are implicit GEMMs on v_mfma_f32_16x16x32_bf16 with the output
// channel as the M dimension, the pixel as N and (tap, input channel) as K:
//   A (16 x 32): weights W[co][tap][ci], 8 contiguous bf16 per lane
//   B (32 x 16): activations X[pixel + tap][ci], 8 contiguous bf16 per lane
//   D (16 x 16): lane l holds rows 4(l/16)..+3 of pixel l%16; in the
//                64-output layers row r of block m is channel out_chan(m, r),
//                so that a lane stores 8 consecutive channels (16 bytes) of
//                one NHWC pixel from two blocks.
// Kernels (cnn_common.h):
//   k_conv3x3_dma   64-output layers on grids whose sides are multiples of
//                   16: persistent, weights and two 16 x 16 halo tiles in LDS
//                   (tiles loaded straight to LDS, double-buffered)
//   k_conv3x3_tile  the 66-output last layer on such grids (80 padded rows)
//   k_conv3x3_mfma  any grid: 256 pixels per workgroup, the weight slice of
//                   each tap staged in LDS, activation fragments read from
//                   global memory (L1/L2), also the 96-channel data gradient
//                   of the last layer in the backward pass
// FP32 accumulation; bias, GELU and bf16 rounding (round to nearest even) in
// the epilogue.
//
// Layer 1 (2 input channels, K = 18) is a single zero-padded K = 32 step of
// the same instruction with the im2col gather done in registers.
#include "cnn_common.h"

namespace {
using namespace cnnk;

// pixel tiles of 16 per wavefront in layer 1: two keep the accumulators
// small enough for 4+ wavefronts per SIMD, which the GELU-bound epilogue needs
constexpr int kFirstTiles = 4;

// layer 1: 2 -> 64 as one K = 32 step of the same MFMA (K = 18 real
// entries: tap-major, channel-minor, as the weights are stored, zero-padded).
// Wavefront w owns kFirstTiles tiles of 16 pixels and all 64 channels:
// lane l gathers the 8 K entries 8(l/16)..+7 of pixel l%16 of each tile
// (bf16-rounded u, v of the taps), holds the matching 8 weights of 4 channel
// tiles, and the epilogue is the one of the other layers.
__global__ void __launch_bounds__(kBlock, 4) k_conv_first(const float* __restrict__ u,
                                                       const float* __restrict__ v,
                                                       const uint16_t* __restrict__ W1,
                                                       const float* __restrict__ b1, PixMap pm,
                                                       uint16_t* __restrict__ Y,
                                                       float* __restrict__ zout) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int kq = lane >> 4;
  const int pbase = (blockIdx.x * (kBlock / 64) + wave) * (kFirstTiles * 16);
  bf16x8 afrag[4];
  f32x4 acc[kFirstTiles][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int co = out_chan(m, col);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = kq * 8 + e;
      afrag[m][e] = __builtin_bit_cast(__bf16, k < 18 ? W1[co * 18 + k] : (uint16_t)0);
    }
    f32x4 b0;
#pragma unroll
    for (int i = 0; i < 4; ++i) b0[i] = b1[out_chan(m, kq * 4 + i)];
#pragma unroll
    for (int t = 0; t < kFirstTiles; ++t) acc[t][m] = b0;
  }
  // the grid sides are powers of two: trajectory, row and column of a pixel
  // by shifts and masks, once per pixel; the taps wrap periodically
  const int hw = pm.H * pm.W;
  const int lw = __builtin_ctz(pm.W), lhw = __builtin_ctz(hw);
#pragma unroll
  for (int t = 0; t < kFirstTiles; ++t) {
    int p = pbase + t * 16 + col;
    p = p < pm.total ? p : pm.total - 1;
    const int base = (p >> lhw) << lhw;
    const int y = (p & (hw - 1)) >> lw, x = p & (pm.W - 1);
    bf16x8 bfrag;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      const int tap = (kq * 8 + e) / 2;
      float a = 0.f, b = 0.f;
      if (tap < 9) {
        const int q = base + ((y + tap / 3 - 1) & (pm.H - 1)) * pm.W + ((x + tap % 3 - 1) & (pm.W - 1));
        a = u[q];
        b = v[q];
      }
      const uint32_t pk = pack_bf16x2(a, b);
      bfrag[e] = __builtin_bit_cast(__bf16, (uint16_t)(pk & 0xffffu));
      bfrag[e + 1] = __builtin_bit_cast(__bf16, (uint16_t)(pk >> 16));
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
      acc[t][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag[m], bfrag, acc[t][m], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < kFirstTiles; ++t) {
    const int p = pbase + t * 16 + col;
    if (p >= pm.total) continue;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      // blocks 2hh and 2hh+1: channels c0 .. c0 + 7 (out_chan)
      const int c0 = hh * 32 + kq * 8;
      const f32x4 a0 = acc[t][2 * hh], a1 = acc[t][2 * hh + 1];
      uint4 pk;
      pk.x = pack_bf16x2(gelu_exact(a0[0]), gelu_exact(a0[1]));
      pk.y = pack_bf16x2(gelu_exact(a0[2]), gelu_exact(a0[3]));
      pk.z = pack_bf16x2(gelu_exact(a1[0]), gelu_exact(a1[1]));
      pk.w = pack_bf16x2(gelu_exact(a1[2]), gelu_exact(a1[3]));
      *reinterpret_cast<uint4*>(Y + (size_t)p * kC + c0) = pk;
      if (zout) {
        *reinterpret_cast<float4*>(zout + (size_t)p * kC + c0) = float4{a0[0], a0[1], a0[2], a0[3]};
        *reinterpret_cast<float4*>(zout + (size_t)p * kC + c0 + 4) =
            float4{a1[0], a1[1], a1[2], a1[3]};
      }
    }
  }
}

}  // namespace

int ldsv_ensure_learned(ldsv_handle* h) {
  LDSV_REQUIRE(h->g.dtype == LDSV_F32 && h->g.layout == LDSV_MAC, LDSV_EDTYPE,
               "the learned path needs an F32 MAC grid");
  if (h->netout) return LDSV_OK;
  const size_t P = h->nstate;
  const size_t bytes = 5 * P * kC * sizeof(uint16_t) + P * LDSV_NOUT * sizeof(float) +
                       P * LDSV_NCOEF * sizeof(uint16_t) +
                       P * (LDSV_NOUT - LDSV_NCOEF) * sizeof(float);
  void* vblk = nullptr;
  LDSV_TRY(ldsv_alloc(h, &vblk, bytes, "learned workspace"));
  char* blk = (char*)vblk;
  for (int l = 0; l < 5; ++l) h->act[l] = (uint16_t*)(blk + (size_t)l * P * kC * sizeof(uint16_t));
  h->netout = (float*)(blk + 5 * P * kC * sizeof(uint16_t));
  h->coef16 = (uint16_t*)(h->netout + P * LDSV_NOUT);
  h->tcbuf = (float*)(h->coef16 + P * LDSV_NCOEF);
  return LDSV_OK;
}

int ldsv_check_net(const ldsv_net* net) {
  LDSV_REQUIRE(net, LDSV_EINVAL, "null network");
  for (int l = 0; l < LDSV_NLAYERS; ++l)
    LDSV_REQUIRE(net->w[l] && net->b[l], LDSV_EINVAL, "network layer %d: null pointer", l);
  for (int l = 1; l < LDSV_NLAYERS; ++l)
    LDSV_REQUIRE(((uintptr_t)net->w[l] & 15) == 0, LDSV_EINVAL,
                 "network layer %d: weights must be 16-byte aligned", l);
  return LDSV_OK;
}

namespace {

// layers 1 and 2 of an inference forward in one launch on grids whose sides
// are multiples of 16: the layer-2 tiles computed from u, v in LDS
int launch_conv12(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                  uint16_t* Y, hipStream_t st) {
  PixMap pm{h->g.ny, h->g.nx, (int)h->nstate};
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int ntiles = (int)(h->nstate / 256);
  const int grid = ntiles < ncu ? ntiles : ncu;
  const size_t lds = conv_dma_lds_bytes();
  LDSV_HIP(hipFuncSetAttribute((const void*)k_conv3x3_dma<0, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  LDSV_TLAUNCH(h, 4, (k_conv3x3_dma<0, true>), dim3(grid), dim3(kConvBlock), lds, st,
               (const uint16_t*)nullptr, net->w[1], net->b[1], pm, Y, (float*)nullptr, u, v,
               net->w[0], net->b[0]);
  return LDSV_OK;
}

}  // namespace

// forward through all layers; zpre (nullable): 5 float NHWC pre-activation
// buffers for the backward pass.  fuse_first without them, on grids whose
// sides are multiples of 16: layer 1 computed inside layer 2's tiles.
int ldsv_launch_cnn(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                    float* out, float* const* zpre, hipStream_t st, uint16_t* coef16, float* tc,
                    bool* bf16_out, bool fuse_first) {
  PixMap pm{h->g.ny, h->g.nx, (int)h->nstate};
  // 16 x 16 LDS tiles when both sides are multiples of 16
  const bool tiled = (h->g.nx % 16 == 0) && (h->g.ny % 16 == 0);
  const bool fuse12 = fuse_first && tiled && !zpre;
  if (fuse12) {
    LDSV_TRY(launch_conv12(h, net, u, v, h->act[1], st));
  } else {
    const int first_pix = (kBlock / 64) * kFirstTiles * 16;
    const int nblk_first = (int)((h->nstate + first_pix - 1) / first_pix);
    LDSV_TLAUNCH(h, 5, k_conv_first, dim3(nblk_first), dim3(kBlock), 0, st, u, v, net->w[0],
                 net->b[0], pm, h->act[0], zpre ? zpre[0] : nullptr);
  }
  LDSV_LAUNCHED();
  const int nblk = (int)((h->nstate + kPixPerBlock - 1) / kPixPerBlock);
  for (int l = fuse12 ? 2 : 1; l < 5; ++l) {
    if (tiled)
      LDSV_TRY(ldsv_launch_conv_tile(h, 4, 0, h->act[l - 1], net->w[l], net->b[l], kC, h->act[l],
                                     zpre ? zpre[l] : nullptr, nullptr, st));
    else
      LDSV_TLAUNCH(h, 4, (k_conv3x3_mfma<4, 0, 64>), dim3(nblk), dim3(kBlock), 0, st,
                   h->act[l - 1], net->w[l], net->b[l], kC, pm, h->act[l],
                   zpre ? zpre[l] : nullptr, (float*)nullptr);
    LDSV_LAUNCHED();
  }
  if (tiled)
    LDSV_TRY(coef16 ? ldsv_launch_conv_tile(h, 5, 3, h->act[4], net->w[5], net->b[5], LDSV_NOUT,
                                            coef16, nullptr, tc, st)
                    : ldsv_launch_conv_tile(h, 5, 1, h->act[4], net->w[5], net->b[5], LDSV_NOUT,
                                            nullptr, nullptr, out, st));
  else
    LDSV_TLAUNCH(h, 4, (k_conv3x3_mfma<5, 1, 64>), dim3(nblk), dim3(kBlock), 0, st, h->act[4],
                 net->w[5], net->b[5], LDSV_NOUT, pm, (uint16_t*)nullptr, (float*)nullptr, out);
  LDSV_LAUNCHED();
  if (bf16_out) *bf16_out = tiled && coef16;
  return LDSV_OK;
}

int ldsv_launch_conv_tile(ldsv_handle* h, int mt, int epi, const uint16_t* X, const uint16_t* W,
                          const float* bias, int cout, uint16_t* Y, float* zio, float* out,
                          hipStream_t st) {
  PixMap pm{h->g.ny, h->g.nx, (int)h->nstate};
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int ntiles = (int)(h->nstate / 256);
  const int grid = ntiles < ncu ? ntiles : ncu;
#define LDSV_CONV_TILE(MT_, EPI_, TW_)                                                          \
  {                                                                                            \
    const size_t lds = conv_tile_lds_bytes<MT_, TW_>();                                        \
    LDSV_HIP(hipFuncSetAttribute((const void*)k_conv3x3_tile<MT_, EPI_, TW_>,                   \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));       \
    LDSV_TLAUNCH(h, 4, (k_conv3x3_tile<MT_, EPI_, TW_>), dim3(grid), dim3(kConvBlock), lds, st, \
                 X, W, bias, cout, pm, Y, zio, out);                                           \
  }
#define LDSV_CONV_DMA(EPI_)                                                                   \
  {                                                                                          \
    const size_t lds = conv_dma_lds_bytes();                                                 \
    LDSV_HIP(hipFuncSetAttribute((const void*)k_conv3x3_dma<EPI_>,                            \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));     \
    LDSV_TLAUNCH(h, 4, (k_conv3x3_dma<EPI_>), dim3(grid), dim3(kConvBlock), lds, st, X, W,    \
                 bias, pm, Y, zio, (const float*)nullptr, (const float*)nullptr,             \
                 (const uint16_t*)nullptr, (const float*)nullptr);                           \
  }
  if (mt == 4 && epi == 0 && cout == kC) LDSV_CONV_DMA(0)
  else if (mt == 4 && epi == 2 && cout == kC) LDSV_CONV_DMA(2)
  else if (mt == 5 && epi == 1) LDSV_CONV_TILE(5, 1, 16)
  else if (mt == 5 && epi == 3) LDSV_CONV_TILE(5, 3, 16)
  else {
    ldsv_set_error("conv tile: unsupported configuration");
    return LDSV_EINVAL;
  }
#undef LDSV_CONV_TILE
#undef LDSV_CONV_DMA
  LDSV_LAUNCHED();
  return LDSV_OK;
}
