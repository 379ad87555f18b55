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
//   D (16 x 16): lane l holds channels 4(l/16)..+3 of pixel l%16, so a lane
//                stores 4 consecutive channels (8 bytes) of one NHWC pixel.
// A workgroup (4 wavefronts) owns 256 consecutive pixels and every output
// channel; per tap it stages that tap's weight slice in LDS (rows padded to
// 144 bytes so the 16 rows a fragment read touches fall in distinct banks),
// and each wavefront multiplies it against its 4 pixel tiles.  Activation
// fragments come straight from global memory (the 9 taps re-read each pixel
// from L1/L2).  FP32 accumulation; bias, GELU and bf16 rounding (round to
// nearest even) in the epilogue.
//
// Layer 1 (2 input channels, K = 18) is not a contraction worth the matrix
// cores; it runs on the vector ALUs with bf16-rounded inputs and weights and
// FP32 accumulation, the same arithmetic as the MFMA layers.
#include "cnn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 64;             // hidden channels
constexpr int kWRow = kC + 8;      // padded LDS weight row (bf16 elements)
constexpr int kPixPerWave = 64;    // 4 pixel tiles of 16
constexpr int kPixPerBlock = 256;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t x = __float_as_uint(f);
  if ((x & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((x >> 16) | 0x40u);
  x += 0x7fffu + ((x >> 16) & 1u);
  return (uint16_t)(x >> 16);
}

__device__ __forceinline__ float gelu_exact(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

struct PixMap {
  int H, W;
  int total;  // B * H * W
  __device__ __forceinline__ int shift(int p, int dy, int dx) const {
    const int hw = H * W;
    const int b = p / hw;
    const int r = p - b * hw;
    const int y = r / W;
    const int x = r - y * W;
    return b * hw + ((y + dy) & (H - 1)) * W + ((x + dx) & (W - 1));
  }
};

// MT: output-channel tiles of 16 (4 for 64 channels, 5 for 66 padded to 80).
// EPI 0: z = acc + bias -> gelu -> bf16 NHWC (and z float NHWC if zout)
// EPI 1: z = acc + bias -> float planar [B][cout][H][W]
template <int MT, int EPI>
__global__ void __launch_bounds__(kBlock) k_conv3x3_mfma(const uint16_t* __restrict__ X,
                                                         const uint16_t* __restrict__ Wt,
                                                         const float* __restrict__ bias, int cout,
                                                         PixMap pm, uint16_t* __restrict__ Y,
                                                         float* __restrict__ zout,
                                                         float* __restrict__ out_planar) {
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
    // stage W[:, tap, :] (cout x 64 bf16) into LDS rows of kWRow; rows past
    // cout are zero
    for (int e = threadIdx.x; e < MT * 16 * (kC / 8); e += blockDim.x) {
      const int row = e / (kC / 8), q = e - row * (kC / 8);
      uint4 v = {0u, 0u, 0u, 0u};
      if (row < cout) v = *reinterpret_cast<const uint4*>(Wt + ((size_t)row * 9 + tap) * kC + q * 8);
      *reinterpret_cast<uint4*>(wl + row * kWRow + q * 8) = v;
    }
    __syncthreads();
    int src[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) src[t] = pm.shift(pix[t], dy, dx);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int cbase = half * 32 + kq * 8;
      bf16x8 bfrag[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        bfrag[t] = *reinterpret_cast<const bf16x8*>(X + (size_t)src[t] * kC + cbase);
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
      if (EPI == 0) {
        float z[4];
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          z[i] = acc[t][m][i] + bias[c0 + i];
          h[i] = f32_to_bf16(gelu_exact(z[i]));
        }
        uint2 pk;
        pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        *reinterpret_cast<uint2*>(Y + (size_t)p * kC + c0) = pk;
        if (zout) *reinterpret_cast<float4*>(zout + (size_t)p * kC + c0) = float4{z[0], z[1], z[2], z[3]};
      } else {
        const int hw = pm.H * pm.W;
        const int b = p / hw;
        const int r = p - b * hw;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = c0 + i;
          if (c < cout) out_planar[((size_t)b * cout + c) * hw + r] = acc[t][m][i] + bias[c];
        }
      }
    }
  }
}

// layer 1: 2 -> 64 on the vector ALUs; one thread per pixel
__global__ void __launch_bounds__(kBlock) k_conv_first(const float* __restrict__ u,
                                                       const float* __restrict__ v,
                                                       const uint16_t* __restrict__ W1,
                                                       const float* __restrict__ b1, PixMap pm,
                                                       uint16_t* __restrict__ Y,
                                                       float* __restrict__ zout) {
  __shared__ float w[kC * 18];
  __shared__ float bb[kC];
  for (int e = threadIdx.x; e < kC * 18; e += blockDim.x) w[e] = bf16_to_f32(W1[e]);
  for (int e = threadIdx.x; e < kC; e += blockDim.x) bb[e] = b1[e];
  __syncthreads();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pm.total) return;
  float in[18];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int q = pm.shift(p, tap / 3 - 1, tap % 3 - 1);
    in[2 * tap] = bf16_to_f32(f32_to_bf16(u[q]));
    in[2 * tap + 1] = bf16_to_f32(f32_to_bf16(v[q]));
  }
  for (int c0 = 0; c0 < kC; c0 += 8) {
    uint16_t h[8];
    float z[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < 18; ++k) a += w[(c0 + i) * 18 + k] * in[k];
      z[i] = a + bb[c0 + i];
      h[i] = f32_to_bf16(gelu_exact(z[i]));
    }
    uint4 pk;
    pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
    pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
    pk.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
    pk.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
    *reinterpret_cast<uint4*>(Y + (size_t)p * kC + c0) = pk;
    if (zout) {
      *reinterpret_cast<float4*>(zout + (size_t)p * kC + c0) = float4{z[0], z[1], z[2], z[3]};
      *reinterpret_cast<float4*>(zout + (size_t)p * kC + c0 + 4) = float4{z[4], z[5], z[6], z[7]};
    }
  }
}

}  // namespace

int ldsv_ensure_learned(ldsv_handle* h) {
  LDSV_REQUIRE(h->g.dtype == LDSV_F32 && h->g.layout == LDSV_MAC, LDSV_EDTYPE,
               "the learned path needs an F32 MAC grid");
  if (h->netout) return LDSV_OK;
  const size_t P = h->nstate;
  const size_t bytes = 5 * P * kC * sizeof(uint16_t) + P * LDSV_NOUT * sizeof(float);
  void* vblk = nullptr;
  LDSV_TRY(ldsv_alloc(h, &vblk, bytes, "learned workspace"));
  char* blk = (char*)vblk;
  for (int l = 0; l < 5; ++l) h->act[l] = (uint16_t*)(blk + (size_t)l * P * kC * sizeof(uint16_t));
  h->netout = (float*)(blk + 5 * P * kC * sizeof(uint16_t));
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

// forward through all layers; zpre (nullable): 5 float NHWC pre-activation
// buffers for the backward pass
int ldsv_launch_cnn(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                    float* out, float* const* zpre, hipStream_t st) {
  PixMap pm{h->g.ny, h->g.nx, (int)h->nstate};
  const int nblk_first = (int)((h->nstate + kBlock - 1) / kBlock);
  {
    TimerScope ts(h, 5, st);
    hipLaunchKernelGGL(k_conv_first, dim3(nblk_first), dim3(kBlock), 0, st, u, v, net->w[0],
                       net->b[0], pm, h->act[0], zpre ? zpre[0] : nullptr);
  }
  LDSV_LAUNCHED();
  const int nblk = (int)((h->nstate + kPixPerBlock - 1) / kPixPerBlock);
  for (int l = 1; l < 5; ++l) {
    TimerScope ts(h, 4, st);
    hipLaunchKernelGGL((k_conv3x3_mfma<4, 0>), dim3(nblk), dim3(kBlock), 0, st, h->act[l - 1],
                       net->w[l], net->b[l], kC, pm, h->act[l], zpre ? zpre[l] : nullptr,
                       (float*)nullptr);
    LDSV_LAUNCHED();
  }
  {
    TimerScope ts(h, 4, st);
    hipLaunchKernelGGL((k_conv3x3_mfma<5, 1>), dim3(nblk), dim3(kBlock), 0, st, h->act[4],
                       net->w[5], net->b[5], LDSV_NOUT, pm, (uint16_t*)nullptr, (float*)nullptr,
                       out);
  }
  LDSV_LAUNCHED();
  return LDSV_OK;
}
