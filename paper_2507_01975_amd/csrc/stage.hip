// Fused finite-volume residual + Runge-Kutta stage kernels.
//
// MAC (incompressible NS, Sec. 3.3 Eqs. 3-4; App. B.2 S1-S7): for the u
// control volume centred at (i dx, (j+1/2) dy)
//   R_u = -(Phi^u_x[i] - Phi^u_x[i-1])/dx - (Phi^u_y[j] - Phi^u_y[j-1])/dy + f_x
// with face fluxes Phi = (advecting velocity)*(interpolated u) - nu*(face
// derivative of u).  The advecting velocity is the linear average of the
// normal velocity; the interpolated value is the physics stencil (midpoint
// average) or the learned 16-point stencil c = c_P + r - mean(r); the face
// derivative is the fourth-order [1, -27, 27, -1]/(24 h) kernel (S6).  The v
// equation mirrors it.  Forcing f = [A sin(k y) - d u, -d v] (App. C.1).
//
// Collocated (2D viscous Burgers, S25): flux form minus q*div with a
// second-order linear-upwind advected value and compact viscous term.
//
// Flux-block mode (Sec. 3.4, Eqs. 5-8): each interpolated value and each
// face derivative is O_P + O_L + O_F: the physics kernel, a spatially
// uniform learnable 5x4 kernel of the kind (20 weights, derivative weights
// scaled by 1/h) and a per-cell field of the kind added at the face the
// cell owns.
//
// One workgroup owns a TX x TY tile of cells.  It stages the stage state
// with a periodic halo of 2 cells in LDS, computes every face flux once
// (each face belongs to exactly one cell: the east face of the x-fluxes and
// the north face of the y-fluxes, so flux differences telescope and
// momentum is conserved), then forms R per cell and the RK combination in
// registers.  HBM traffic per cell: one read of the stage state, the base
// state and the accumulator as needed, one write of the outputs.
#include <type_traits>

#include "stage.h"

namespace {

constexpr int kMaxTX = 64;
constexpr int kMaxTY = 16;
constexpr int kH = 2;  // halo
constexpr int kSX = kMaxTX + 2 * kH;
constexpr int kSY = kMaxTY + 2 * kH;

// footprint point s: along-normal offset A_OFF[s], across offset B_OFF[s]
__constant__ int kAOff[16] = {-1, 0, 1, 2, -1, 0, 1, 2, -1, 0, 1, 2, 0, 1, 0, 1};
__constant__ int kBOff[16] = {-1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -2, -2, 2, 2};

// Physical constants, rounded to the kernel's type on the host (the same
// double-to-T roundings as before, without per-thread double divisions);
// the forcing keeps its FP64 inputs for the per-row sine.
template <typename T>
struct PhysT {
  T nu, drag, idx, idy, i24dx, i24dy, idx2, idy2;
  double amp, kf, dy;
  int mask;
};

template <typename T>
struct CombT {
  T alpha, beta, delta, eps, gamma, wacc;
  int need_un, need_acc;
};

// the 5x4 window of the uniform kernels: points 0..15 as above, then the
// four corners
__device__ __forceinline__ constexpr int a_off20(int s) {
  return s < 12 ? s % 4 - 1 : (s < 16 ? (s & 1) : (s & 1 ? 2 : -1));
}
__device__ __forceinline__ constexpr int b_off20(int s) {
  return s < 12 ? s / 4 - 1 : (s < 14 ? -2 : (s < 16 ? 2 : (s < 18 ? -2 : 2)));
}

template <typename T>
struct StagePtrs {
  const T* us;
  const T* vs;
  const T* un;
  const T* vn;
  const T* accu;
  const T* accv;
  T* ou;
  T* ov;
  T* oaccu;
  T* oaccv;
  const float* coef;
  size_t cbs;
  const uint16_t* coef16;
  size_t cbs16;
  const float* dcoef;
  const uint16_t* dcoef16;
  const float* tcu;
  const float* tcv;
  size_t tcbs;
  const float* fbw;  // flux block: [interp, deriv][kind][20] uniform weights
  const float* fbf;  // flux block: [B][8][Ny][Nx] fields (interp kinds, deriv kinds), nullable
  size_t fbs;
  const int* active;  // per-trajectory mask, nullable (MAC)
};

// One trajectory's plane addressed through a buffer resource: a uniform
// base in scalar registers and a 32-bit element offset per lane (one
// buffer_load/buffer_store with a vector offset instead of 64-bit address
// arithmetic per element); accesses past the plane return zero / are
// dropped by the hardware range check.
template <typename T>
struct PlaneBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ PlaneBuf(const T* base, unsigned n)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0,
                                            (int)(n * (unsigned)sizeof(T)), 0x00020000)) {}
  __device__ __forceinline__ T ld(unsigned i) const {
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, 0));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, 0));
  }
  __device__ __forceinline__ void st(unsigned i, T v) const {
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, i * 4u, 0, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b64(
          __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r,
          i * 8u, 0, 0);
  }
};

__device__ __forceinline__ float coef_value(const float* p) { return *p; }
__device__ __forceinline__ float coef_value(const uint16_t* p) {
  return __uint_as_float(((uint32_t)*p) << 16);  // bf16 -> float, exact
}

// The 16 raw values of kind K at the cell with in-plane offset off: float
// planes [64][Ny][Nx] (point s of kind K in plane 16K + s), or bf16 values
// in blocks of 8 channels [8][Ny][Nx][8] (channel c of a cell at block c / 8,
// position c % 8: a kind is two 16-byte loads, and the loads of consecutive
// cells are consecutive 16-byte chunks)
__device__ __forceinline__ void kind_values(const float* cb, int kind, size_t plane, size_t off,
                                            float (&r)[16]) {
#pragma unroll
  for (int s = 0; s < 16; ++s) r[s] = cb[(size_t)(16 * kind + s) * plane + off];
}
__device__ __forceinline__ void kind_values(const uint16_t* cb, int kind, size_t plane,
                                            size_t off, float (&r)[16]) {
  const uint4 a = *reinterpret_cast<const uint4*>(cb + ((size_t)(2 * kind) * plane + off) * 8);
  const uint4 b = *reinterpret_cast<const uint4*>(cb + ((size_t)(2 * kind + 1) * plane + off) * 8);
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    r[2 * k] = __uint_as_float(w[k] << 16);
    r[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
  }
}

// learned interpolation at a face owned by global cell (gi, gj), kind K;
// q(a, b) is the tile value at along offset a, across offset b; the raw
// coefficients are float planes or bf16 per-cell vectors (CT)
template <typename T, bool ALONG_X, int W, typename CT>
__device__ __forceinline__ T learned_face(const T (*S)[W], int lj, int li, const CT* cb,
                                          int kind, size_t plane, size_t off) {
  float rv[16];
  kind_values(cb, kind, plane, off, rv);
  T r[16];
  T m = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    r[s] = (T)rv[s];
    m += r[s];
  }
  m *= (T)(1.0 / 16.0);
  T acc = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const T q = ALONG_X ? S[lj + kBOff[s]][li + kAOff[s]] : S[lj + kAOff[s]][li + kBOff[s]];
    acc += (r[s] - m) * q;
  }
  const T q0 = S[lj][li];
  const T q1 = ALONG_X ? S[lj][li + 1] : S[lj + 1][li];
  return acc + (T)0.5 * (q0 + q1);
}

// learned face derivative (units of 1/h) at a face: the raw values r of kind
// K projected onto zero sum, unit normal and zero across first moment around
// the fourth-order kernel, w = w_P + r - mean(r) - x (x.r)/16 - b (b.r)/24,
// applied to the 16 footprint values: sum r q - mean(r) sum q - (x.r)/16
// sum x q - (b.r)/24 sum b q + the fourth-order part
template <typename T, bool ALONG_X, int W, typename CT>
__device__ __forceinline__ T learned_dface(const T (*S)[W], int lj, int li, const CT* cb, int kind,
                                           size_t plane, size_t off) {
  float rv[16];
  kind_values(cb, kind, plane, off, rv);
  T rq = 0, sr = 0, sxr = 0, sbr = 0, sq = 0, sxq = 0, sbq = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const T r = (T)rv[s];
    const int a = a_off20(s), bb = b_off20(s);
    const T q = ALONG_X ? S[lj + bb][li + a] : S[lj + a][li + bb];
    const T x = (T)a - (T)0.5;
    rq += r * q;
    sr += r;
    sxr += x * r;
    sbr += (T)bb * r;
    sq += q;
    sxq += x * q;
    sbq += (T)bb * q;
  }
  const T qm1 = ALONG_X ? S[lj][li - 1] : S[lj - 1][li];
  const T q0 = S[lj][li];
  const T q1 = ALONG_X ? S[lj][li + 1] : S[lj + 1][li];
  const T q2 = ALONG_X ? S[lj][li + 2] : S[lj + 2][li];
  return rq - sr * sq * (T)(1.0 / 16.0) - sxr * sxq * (T)(1.0 / 16.0) -
         sbr * sbq * (T)(1.0 / 24.0) + (qm1 - (T)27 * q0 + (T)27 * q1 - q2) * (T)(1.0 / 24.0);
}

// uniform 5x4 kernel w (20 weights) at the face owned by tile point (lj, li)
template <typename T, bool ALONG_X, int W>
__device__ __forceinline__ T uniform_face(const T (*S)[W], int lj, int li, const float* w) {
  T acc = 0;
#pragma unroll
  for (int s = 0; s < 20; ++s) {
    const T q = ALONG_X ? S[lj + b_off20(s)][li + a_off20(s)] : S[lj + a_off20(s)][li + b_off20(s)];
    acc += (T)w[s] * q;
  }
  return acc;
}

__device__ __forceinline__ float fb_field(const float* f, size_t plane, int ch, size_t off) {
  return f ? f[(size_t)ch * plane + off] : 0.f;
}

// COEF: 0 plain stencil, 1 float raw coefficients, 2 bf16 raw coefficients,
// 3 flux block (uniform kernels and fields), 4 and 5: as 1 and 2 plus the
// learned derivative values in the same form
// ALL: every physics term on (the mask known at compile time, no per-face
// tests of it).  RK: the stage's combination known at compile time (0: from
// cb at run time; 1: beta uc + eps R, accumulator wacc R, the first RK4
// stage; 2: alpha un + eps R, accumulator gamma acc + wacc R, the middle
// ones; 3: alpha un + eps R + delta acc, no accumulator, the last one), its
// zero terms and their loads dropped
template <typename T, int COEF, int TX, int TY, bool ALL = false, int RK = 0>
__global__ void __launch_bounds__(kBlock) k_stage_mac(StagePtrs<T> p, PhysT<T> ph, CombT<T> cb, int nx,
                                                      int ny) {
  constexpr int W = TX + 2 * kH, Hh = TY + 2 * kH;
  constexpr int kTile = W * Hh;
  constexpr int kTilePer = (kTile + kBlock - 1) / kBlock;
  constexpr int kCells = TX * TY;
  constexpr int kCellPer = (kCells + kBlock - 1) / kBlock;
  __shared__ T su[Hh][W];
  __shared__ T sv[Hh][W];
  __shared__ T fux[TY][TX + 1];
  __shared__ T fvx[TY][TX + 1];
  __shared__ T fuy[TY + 1][TX];
  __shared__ T fvy[TY + 1][TX];
  __shared__ T frow[TY];

  const int tilesx = nx / TX;
  const int tile = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int b = tile / gridDim.x;
  if (p.active && !p.active[b]) return;  // uniform per workgroup, before any barrier
  const int tp = tile - b * gridDim.x;
  const int i0 = (tp % tilesx) * TX;
  const int j0 = (tp / tilesx) * TY;
  const size_t plane = (size_t)nx * ny;
  const size_t boff = (size_t)b * plane;
  // the trajectory's planes as buffers: 32-bit offsets within a plane (at
  // most 2048^2 cells)
  const unsigned pl = (unsigned)plane;
  const PlaneBuf<T> usb(p.us + boff, pl), vsb(p.vs + boff, pl);

  // stage state with its periodic halo: every load of the thread in flight
  // before the LDS stores
  {
    T tu[kTilePer], tvv[kTilePer];
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kTile) {
        const int r = t / W, c = t - r * W;
        const int gj = (j0 - kH + r + ny) & (ny - 1);
        const int gi = (i0 - kH + c + nx) & (nx - 1);
        const unsigned g = (unsigned)gj * (unsigned)nx + (unsigned)gi;
        tu[k] = usb.ld(g);
        tvv[k] = vsb.ld(g);
      }
    }
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      const int t = k * kBlock + (int)threadIdx.x;
      if (t < kTile) {
        const int r = t / W, c = t - r * W;
        su[r][c] = tu[k];
        sv[r][c] = tvv[k];
      }
    }
  }
  if ((ALL || (ph.mask & LDSV_FORCING)) && threadIdx.x < TY)
    frow[threadIdx.x] =
        ph.amp != 0.0 ? (T)(ph.amp * sin(ph.kf * ((j0 + threadIdx.x) + 0.5) * ph.dy)) : (T)0;
  // operands of the RK combination, prefetched before the flux phases
  T pun[kCellPer], pvn[kCellPer], pau[kCellPer], pav[kCellPer];
  const bool need_un = RK == 0 ? (bool)cb.need_un : RK != 1;
  const bool need_acc = RK == 0 ? (bool)cb.need_acc : RK != 1;
#pragma unroll
  for (int k = 0; k < kCellPer; ++k) {
    const int t = k * kBlock + (int)threadIdx.x;
    pun[k] = pvn[k] = pau[k] = pav[k] = (T)0;
    if (t < kCells) {
      const int r = t / TX, c = t - r * TX;
      const unsigned g = (unsigned)(j0 + r) * (unsigned)nx + (unsigned)(i0 + c);
      if (need_un) {
        pun[k] = PlaneBuf<T>(p.un + boff, pl).ld(g);
        pvn[k] = PlaneBuf<T>(p.vn + boff, pl).ld(g);
      }
      if (need_acc) {
        pau[k] = PlaneBuf<T>(p.accu + boff, pl).ld(g);
        pav[k] = PlaneBuf<T>(p.accv + boff, pl).ld(g);
      }
    }
  }
  __syncthreads();

  const bool adv = ALL || (ph.mask & LDSV_ADVECTION);
  const bool visc = ALL || (ph.mask & LDSV_VISCOSITY);
  const T nu = ph.nu;
  const T i24dx = ph.i24dx, i24dy = ph.i24dy;
  constexpr int IC = COEF == 4 ? 1 : (COEF == 5 ? 2 : COEF);  // interpolation form
  constexpr bool LD = COEF >= 4;                                 // learned derivatives
  const float* cbf = IC == 1 ? p.coef + (size_t)b * p.cbs : nullptr;
  const uint16_t* cbh = IC == 2 ? p.coef16 + (size_t)b * p.cbs16 : nullptr;
  const float* dbf = COEF == 4 ? p.dcoef + (size_t)b * p.cbs : nullptr;
  const uint16_t* dbh = COEF == 5 ? p.dcoef16 + (size_t)b * p.cbs16 : nullptr;
  const float* fbf = COEF == 3 && p.fbf ? p.fbf + (size_t)b * p.fbs : nullptr;

  // x-faces: owners i in [i0-1, i0+TX-1], rows j in [j0, j0+TY-1]
  constexpr int kXF = TY * (TX + 1);
#pragma unroll
  for (int k = 0; k < (kXF + kBlock - 1) / kBlock; ++k) {
    const int t = k * kBlock + (int)threadIdx.x;
    if (t >= kXF) break;
    const int r = t / (TX + 1), c = t - r * (TX + 1);
    const int li = c + 1, lj = r + kH;
    [[maybe_unused]] const size_t xoff = (size_t)(j0 + r) * nx + ((i0 - 1 + c + nx) & (nx - 1));
    T fu = 0, fv = 0;
    if (adv) {
      const T ubar = (T)0.5 * (su[lj][li] + su[lj][li + 1]);
      const T ubar_e = (T)0.5 * (su[lj - 1][li + 1] + su[lj][li + 1]);
      T uf, vf;
      if constexpr (COEF == 3) {
        uf = (T)0.5 * (su[lj][li] + su[lj][li + 1]) + uniform_face<T, true, W>(su, lj, li, p.fbw) +
             (T)fb_field(fbf, plane, 0, xoff);
        vf = (T)0.5 * (sv[lj][li] + sv[lj][li + 1]) +
             uniform_face<T, true, W>(sv, lj, li, p.fbw + 40) + (T)fb_field(fbf, plane, 2, xoff);
      } else if constexpr (COEF != 0) {
        const int gi = (i0 - 1 + c + nx) & (nx - 1);
        const size_t off = (size_t)(j0 + r) * nx + gi;
        if constexpr (IC == 1) {
          uf = learned_face<T, true, W>(su, lj, li, cbf, 0, plane, off);
          vf = learned_face<T, true, W>(sv, lj, li, cbf, 2, plane, off);
        } else {
          uf = learned_face<T, true, W>(su, lj, li, cbh, 0, plane, off);
          vf = learned_face<T, true, W>(sv, lj, li, cbh, 2, plane, off);
        }
      } else {
        uf = (T)0.5 * (su[lj][li] + su[lj][li + 1]);
        vf = (T)0.5 * (sv[lj][li] + sv[lj][li + 1]);
      }
      fu = ubar * uf;
      fv = ubar_e * vf;
    }
    if (visc) {
      if constexpr (COEF == 3) {
        const T du = (su[lj][li - 1] - (T)27 * su[lj][li] + (T)27 * su[lj][li + 1] - su[lj][li + 2]) * i24dx +
                     uniform_face<T, true, W>(su, lj, li, p.fbw + 80) * ph.idx +
                     (T)fb_field(fbf, plane, 4, xoff);
        const T dv = (sv[lj][li - 1] - (T)27 * sv[lj][li] + (T)27 * sv[lj][li + 1] - sv[lj][li + 2]) * i24dx +
                     uniform_face<T, true, W>(sv, lj, li, p.fbw + 120) * ph.idx +
                     (T)fb_field(fbf, plane, 6, xoff);
        fu -= nu * du;
        fv -= nu * dv;
      } else if constexpr (LD) {
        if constexpr (COEF == 4) {
          fu -= nu * learned_dface<T, true, W>(su, lj, li, dbf, 0, plane, xoff) * ph.idx;
          fv -= nu * learned_dface<T, true, W>(sv, lj, li, dbf, 2, plane, xoff) * ph.idx;
        } else {
          fu -= nu * learned_dface<T, true, W>(su, lj, li, dbh, 0, plane, xoff) * ph.idx;
          fv -= nu * learned_dface<T, true, W>(sv, lj, li, dbh, 2, plane, xoff) * ph.idx;
        }
      } else {
        fu -= nu * (su[lj][li - 1] - (T)27 * su[lj][li] + (T)27 * su[lj][li + 1] - su[lj][li + 2]) * i24dx;
        fv -= nu * (sv[lj][li - 1] - (T)27 * sv[lj][li] + (T)27 * sv[lj][li + 1] - sv[lj][li + 2]) * i24dx;
      }
    }
    fux[r][c] = fu;
    fvx[r][c] = fv;
  }
  // y-faces: owners j in [j0-1, j0+TY-1], columns i in [i0, i0+TX-1]
  constexpr int kYF = (TY + 1) * TX;
  // the y-face loop numbers the threads from wavefront 1, so that its
  // partial last iteration and that of the x-face loop (which starts at
  // wavefront 0) fall on different wavefronts
  const int ty = ((int)threadIdx.x + kBlock - 64) & (kBlock - 1);
#pragma unroll
  for (int k = 0; k < (kYF + kBlock - 1) / kBlock; ++k) {
    const int t = k * kBlock + ty;
    if (t >= kYF) break;
    const int r = t / TX, c = t - r * TX;
    const int li = c + kH, lj = r + 1;
    [[maybe_unused]] const size_t yoff = (size_t)((j0 - 1 + r + ny) & (ny - 1)) * nx + (i0 + c);
    T fu = 0, fv = 0;
    if (adv) {
      const T vbar_n = (T)0.5 * (sv[lj + 1][li - 1] + sv[lj + 1][li]);
      const T vbar_c = (T)0.5 * (sv[lj][li] + sv[lj + 1][li]);
      T uf, vf;
      if constexpr (COEF == 3) {
        uf = (T)0.5 * (su[lj][li] + su[lj + 1][li]) +
             uniform_face<T, false, W>(su, lj, li, p.fbw + 20) + (T)fb_field(fbf, plane, 1, yoff);
        vf = (T)0.5 * (sv[lj][li] + sv[lj + 1][li]) +
             uniform_face<T, false, W>(sv, lj, li, p.fbw + 60) + (T)fb_field(fbf, plane, 3, yoff);
      } else if constexpr (COEF != 0) {
        const int gj = (j0 - 1 + r + ny) & (ny - 1);
        const size_t off = (size_t)gj * nx + (i0 + c);
        if constexpr (IC == 1) {
          uf = learned_face<T, false, W>(su, lj, li, cbf, 1, plane, off);
          vf = learned_face<T, false, W>(sv, lj, li, cbf, 3, plane, off);
        } else {
          uf = learned_face<T, false, W>(su, lj, li, cbh, 1, plane, off);
          vf = learned_face<T, false, W>(sv, lj, li, cbh, 3, plane, off);
        }
      } else {
        uf = (T)0.5 * (su[lj][li] + su[lj + 1][li]);
        vf = (T)0.5 * (sv[lj][li] + sv[lj + 1][li]);
      }
      fu = vbar_n * uf;
      fv = vbar_c * vf;
    }
    if (visc) {
      if constexpr (COEF == 3) {
        const T du = (su[lj - 1][li] - (T)27 * su[lj][li] + (T)27 * su[lj + 1][li] - su[lj + 2][li]) * i24dy +
                     uniform_face<T, false, W>(su, lj, li, p.fbw + 100) * ph.idy +
                     (T)fb_field(fbf, plane, 5, yoff);
        const T dv = (sv[lj - 1][li] - (T)27 * sv[lj][li] + (T)27 * sv[lj + 1][li] - sv[lj + 2][li]) * i24dy +
                     uniform_face<T, false, W>(sv, lj, li, p.fbw + 140) * ph.idy +
                     (T)fb_field(fbf, plane, 7, yoff);
        fu -= nu * du;
        fv -= nu * dv;
      } else if constexpr (LD) {
        if constexpr (COEF == 4) {
          fu -= nu * learned_dface<T, false, W>(su, lj, li, dbf, 1, plane, yoff) * ph.idy;
          fv -= nu * learned_dface<T, false, W>(sv, lj, li, dbf, 3, plane, yoff) * ph.idy;
        } else {
          fu -= nu * learned_dface<T, false, W>(su, lj, li, dbh, 1, plane, yoff) * ph.idy;
          fv -= nu * learned_dface<T, false, W>(sv, lj, li, dbh, 3, plane, yoff) * ph.idy;
        }
      } else {
        fu -= nu * (su[lj - 1][li] - (T)27 * su[lj][li] + (T)27 * su[lj + 1][li] - su[lj + 2][li]) * i24dy;
        fv -= nu * (sv[lj - 1][li] - (T)27 * sv[lj][li] + (T)27 * sv[lj + 1][li] - sv[lj + 2][li]) * i24dy;
      }
    }
    fuy[r][c] = fu;
    fvy[r][c] = fv;
  }
  __syncthreads();

  const T idx = ph.idx, idy = ph.idy;
  const T drag = ph.drag;
  const bool force = ALL || (ph.mask & LDSV_FORCING);
#pragma unroll
  for (int k = 0; k < kCellPer; ++k) {
    const int t = k * kBlock + (int)threadIdx.x;
    if (t >= kCells) break;
    const int r = t / TX, c = t - r * TX;
    const T uc = su[r + kH][c + kH], vc = sv[r + kH][c + kH];
    T ru = -(fux[r][c + 1] - fux[r][c]) * idx - (fuy[r + 1][c] - fuy[r][c]) * idy;
    T rv = -(fvx[r][c + 1] - fvx[r][c]) * idx - (fvy[r + 1][c] - fvy[r][c]) * idy;
    if (force) {
      ru += frow[r] - drag * uc;
      rv -= drag * vc;
    }
    const unsigned g = (unsigned)(j0 + r) * (unsigned)nx + (unsigned)(i0 + c);
    T ou, ov;
    if constexpr (RK == 1) {
      ou = cb.beta * uc + cb.eps * ru;
      ov = cb.beta * vc + cb.eps * rv;
    } else if constexpr (RK == 2) {
      ou = cb.alpha * pun[k] + cb.eps * ru;
      ov = cb.alpha * pvn[k] + cb.eps * rv;
    } else if constexpr (RK == 3) {
      ou = cb.alpha * pun[k] + cb.eps * ru + cb.delta * pau[k];
      ov = cb.alpha * pvn[k] + cb.eps * rv + cb.delta * pav[k];
    } else {
      ou = cb.beta * uc + cb.eps * ru + cb.alpha * pun[k] + cb.delta * pau[k];
      ov = cb.beta * vc + cb.eps * rv + cb.alpha * pvn[k] + cb.delta * pav[k];
    }
    if (p.tcu) {
      const size_t gt = (size_t)b * p.tcbs + (size_t)(j0 + r) * nx + (i0 + c);
      ou += (T)p.tcu[gt];
      ov += (T)p.tcv[gt];
    }
    PlaneBuf<T>(p.ou + boff, pl).st(g, ou);
    PlaneBuf<T>(p.ov + boff, pl).st(g, ov);
    if (RK == 1) {
      PlaneBuf<T>(p.oaccu + boff, pl).st(g, cb.wacc * ru);
      PlaneBuf<T>(p.oaccv + boff, pl).st(g, cb.wacc * rv);
    } else if (RK == 2 || (RK == 0 && p.oaccu)) {
      PlaneBuf<T>(p.oaccu + boff, pl).st(g, cb.gamma * pau[k] + cb.wacc * ru);
      PlaneBuf<T>(p.oaccv + boff, pl).st(g, cb.gamma * pav[k] + cb.wacc * rv);
    }
  }
}

// collocated tiles are at most 64 x 8 (six flux arrays instead of four)
constexpr int kMaxTYc = 8;
constexpr int kSYc = kMaxTYc + 2 * kH;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_stage_col(StagePtrs<T> p, PhysT<T> ph, CombT<T> cb, int nx,
                                                      int ny, int TX, int TY) {
  __shared__ T su[kSYc][kSX];
  __shared__ T sv[kSYc][kSX];
  __shared__ T ae[kMaxTYc][kMaxTX + 1];
  __shared__ T fue[kMaxTYc][kMaxTX + 1];
  __shared__ T fve[kMaxTYc][kMaxTX + 1];
  __shared__ T bn[kMaxTYc + 1][kMaxTX];
  __shared__ T fun[kMaxTYc + 1][kMaxTX];
  __shared__ T fvn[kMaxTYc + 1][kMaxTX];

  const int tilesx = nx / TX;
  const int tile = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int b = tile / gridDim.x;
  const int tp = tile - b * gridDim.x;
  const int i0 = (tp % tilesx) * TX;
  const int j0 = (tp / tilesx) * TY;
  const size_t plane = (size_t)nx * ny;
  const size_t boff = (size_t)b * plane;
  const int W = TX + 2 * kH, Hh = TY + 2 * kH;
  for (int t = threadIdx.x; t < W * Hh; t += blockDim.x) {
    const int r = t / W, c = t - r * W;
    const int gj = (j0 - kH + r + ny) & (ny - 1);
    const int gi = (i0 - kH + c + nx) & (nx - 1);
    const size_t g = boff + (size_t)gj * nx + gi;
    su[r][c] = p.us[g];
    sv[r][c] = p.vs[g];
  }
  __syncthreads();
  const bool adv = ph.mask & LDSV_ADVECTION;
  if (adv) {
    for (int t = threadIdx.x; t < TY * (TX + 1); t += blockDim.x) {
      const int r = t / (TX + 1), c = t - r * (TX + 1);
      const int li = c + 1, lj = r + kH;
      const T a = (T)0.5 * (su[lj][li] + su[lj][li + 1]);
      T qu, qv;
      if (a > (T)0) {
        qu = (T)-0.5 * su[lj][li - 1] + (T)1.5 * su[lj][li];
        qv = (T)-0.5 * sv[lj][li - 1] + (T)1.5 * sv[lj][li];
      } else {
        qu = (T)1.5 * su[lj][li + 1] - (T)0.5 * su[lj][li + 2];
        qv = (T)1.5 * sv[lj][li + 1] - (T)0.5 * sv[lj][li + 2];
      }
      ae[r][c] = a;
      fue[r][c] = a * qu;
      fve[r][c] = a * qv;
    }
    for (int t = threadIdx.x; t < (TY + 1) * TX; t += blockDim.x) {
      const int r = t / TX, c = t - r * TX;
      const int li = c + kH, lj = r + 1;
      const T bb = (T)0.5 * (sv[lj][li] + sv[lj + 1][li]);
      T qu, qv;
      if (bb > (T)0) {
        qu = (T)-0.5 * su[lj - 1][li] + (T)1.5 * su[lj][li];
        qv = (T)-0.5 * sv[lj - 1][li] + (T)1.5 * sv[lj][li];
      } else {
        qu = (T)1.5 * su[lj + 1][li] - (T)0.5 * su[lj + 2][li];
        qv = (T)1.5 * sv[lj + 1][li] - (T)0.5 * sv[lj + 2][li];
      }
      bn[r][c] = bb;
      fun[r][c] = bb * qu;
      fvn[r][c] = bb * qv;
    }
  }
  __syncthreads();
  const T idx = ph.idx, idy = ph.idy;
  const T idx2 = ph.idx2, idy2 = ph.idy2;
  const T nu = ph.nu;
  const bool visc = ph.mask & LDSV_VISCOSITY;
  for (int t = threadIdx.x; t < TY * TX; t += blockDim.x) {
    const int r = t / TX, c = t - r * TX;
    const int lj = r + kH, li = c + kH;
    const T uc = su[lj][li], vc = sv[lj][li];
    T ru = 0, rv = 0;
    if (adv) {
      const T dv = (ae[r][c + 1] - ae[r][c]) * idx + (bn[r + 1][c] - bn[r][c]) * idy;
      ru = -((fue[r][c + 1] - fue[r][c]) * idx + (fun[r + 1][c] - fun[r][c]) * idy) + uc * dv;
      rv = -((fve[r][c + 1] - fve[r][c]) * idx + (fvn[r + 1][c] - fvn[r][c]) * idy) + vc * dv;
    }
    if (visc) {
      ru += nu * ((su[lj][li + 1] - (T)2 * uc + su[lj][li - 1]) * idx2 +
                  (su[lj + 1][li] - (T)2 * uc + su[lj - 1][li]) * idy2);
      rv += nu * ((sv[lj][li + 1] - (T)2 * vc + sv[lj][li - 1]) * idx2 +
                  (sv[lj + 1][li] - (T)2 * vc + sv[lj - 1][li]) * idy2);
    }
    const size_t g = boff + (size_t)(j0 + r) * nx + (i0 + c);
    T ou = cb.beta * uc + cb.eps * ru;
    T ov = cb.beta * vc + cb.eps * rv;
    if (cb.need_un) {
      ou += cb.alpha * p.un[g];
      ov += cb.alpha * p.vn[g];
    }
    T au = 0, av = 0;
    if (cb.need_acc) {
      au = p.accu[g];
      av = p.accv[g];
      ou += cb.delta * au;
      ov += cb.delta * av;
    }
    p.ou[g] = ou;
    p.ov[g] = ov;
    if (p.oaccu) {
      p.oaccu[g] = cb.gamma * au + cb.wacc * ru;
      p.oaccv[g] = cb.gamma * av + cb.wacc * rv;
    }
  }
}

// the plain stage with every physics term on, its RK combination kind rk
// (see k_stage_mac) fixed at compile time
template <typename T, int TX, int TY>
void launch_plain_all(ldsv_handle* h, dim3 grid, hipStream_t st, const StagePtrs<T>& p,
                      const PhysT<T>& ph, const CombT<T>& cb, int nx, int ny, int rk) {
  if (rk == 1)
    LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 0, TX, TY, true, 1>), grid, dim3(kBlock), 0, st, p, ph, cb,
                 nx, ny);
  else if (rk == 2)
    LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 0, TX, TY, true, 2>), grid, dim3(kBlock), 0, st, p, ph, cb,
                 nx, ny);
  else if (rk == 3)
    LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 0, TX, TY, true, 3>), grid, dim3(kBlock), 0, st, p, ph, cb,
                 nx, ny);
  else
    LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 0, TX, TY, true>), grid, dim3(kBlock), 0, st, p, ph, cb, nx,
                 ny);
}

// the learned-derivative stage modes exist for FP32 states only (the
// learned path's precision)
template <typename T, int COEF, int TX, int TY, bool ALL = false>
int launch_learned_d(ldsv_handle* h, dim3 grid, hipStream_t st, const StagePtrs<T>& p,
                     const PhysT<T>& ph, const CombT<T>& cb, int nx, int ny) {
  if constexpr (std::is_same<T, float>::value) {
    LDSV_TLAUNCH(h, 0, (k_stage_mac<T, COEF, TX, TY, ALL>), grid, dim3(kBlock), 0, st, p, ph, cb,
                 nx, ny);
    return LDSV_OK;
  } else {
    ldsv_set_error("stage: learned derivative stencils need FP32 states");
    return LDSV_EDTYPE;
  }
}

template <typename T>
int launch_stage_t(ldsv_handle* h, const ldsv_params* prm, const StageArgs& a, hipStream_t st) {
  StagePtrs<T> p;
  p.us = (const T*)a.us;
  p.vs = (const T*)a.vs;
  p.un = (const T*)a.un;
  p.vn = (const T*)a.vn;
  p.accu = (const T*)a.accu;
  p.accv = (const T*)a.accv;
  p.ou = (T*)a.ou;
  p.ov = (T*)a.ov;
  p.oaccu = (T*)a.oaccu;
  p.oaccv = (T*)a.oaccv;
  p.coef = a.coef;
  p.cbs = a.coef_bstride;
  p.coef16 = a.coef16;
  p.cbs16 = a.coef16_bstride;
  p.dcoef = a.dcoef;
  p.dcoef16 = a.dcoef16;
  p.tcu = a.tcu;
  p.tcv = a.tcv;
  p.tcbs = a.tc_bstride;
  p.fbw = a.fbw;
  p.fbf = a.fbf;
  p.fbs = a.fb_bstride;
  p.active = a.active;
  const double dx = h->g.lx / h->g.nx, dy = h->g.ly / h->g.ny;
  PhysT<T> ph;
  ph.nu = (T)prm->nu;
  ph.drag = (T)prm->drag;
  ph.idx = (T)(1.0 / dx);
  ph.idy = (T)(1.0 / dy);
  ph.i24dx = (T)(1.0 / (24.0 * dx));
  ph.i24dy = (T)(1.0 / (24.0 * dy));
  ph.idx2 = ph.idx * ph.idx;
  ph.idy2 = ph.idy * ph.idy;
  ph.amp = prm->forcing_amp;
  ph.kf = prm->forcing_k;
  ph.dy = dy;
  ph.mask = prm->physics_mask;
  CombT<T> cb{(T)a.alpha, (T)a.beta, (T)a.delta, (T)a.eps, (T)a.gamma, (T)a.wacc,
              a.alpha != 0.0, a.delta != 0.0 || a.gamma != 0.0};
  const int nx = h->g.nx, ny = h->g.ny;
  if (h->g.layout == LDSV_COLLOCATED) {
    const int TX = nx < kMaxTX ? nx : kMaxTX;
    const int TYc = ny < kMaxTYc ? ny : kMaxTYc;
    dim3 gridc((nx / TX) * (ny / TYc), h->g.batch);
    LDSV_TLAUNCH(h, 0, k_stage_col<T>, gridc, dim3(kBlock), 0, st, p, ph, cb, nx, ny, TX, TYc);
    LDSV_LAUNCHED();
    return LDSV_OK;
  }
  // small grids: shrink the tile (64x16 -> 64x8 -> 32x8) until the launch
  // has at least 1024 workgroups, about four waves per SIMD, so that the
  // per-face coefficient loads have other waves to hide behind; each face
  // flux is computed the same way whatever the tile, so the result does not
  // depend on it
  int TX = nx < kMaxTX ? nx : kMaxTX;
  int TY = ny < kMaxTY ? ny : kMaxTY;
  auto wgs = [&](int tx, int ty) { return (long)(nx / tx) * (ny / ty) * h->g.batch; };
  while (wgs(TX, TY) < 1024 && (TY > 8 || TX > 32)) {
    if (TY > 8)
      TY = 8;
    else
      TX /= 2;
  }
  dim3 grid((nx / TX) * (ny / TY), h->g.batch);
  // every physics term on (all the configurations run so): the mask fixed at
  // compile time in every mode (the float- and bf16-coefficient forms of a
  // mode then compile to the same arithmetic and stay equal bit for bit)
  const bool all = ph.mask == LDSV_ALL_PHYSICS;
  // the RK4 stages' combination patterns (zero coefficients; SSP-RK3 and
  // the rest keep the general form)
  int rk = 0;
  {
    const bool acc_out = a.oaccu != nullptr;
    if (a.alpha == 0.0 && a.delta == 0.0 && a.gamma == 0.0 && acc_out)
      rk = 1;
    else if (a.beta == 0.0 && a.delta == 0.0 && a.alpha != 0.0 && a.gamma != 0.0 && acc_out)
      rk = 2;
    else if (a.beta == 0.0 && a.alpha != 0.0 && a.delta != 0.0 && !acc_out)
      rk = 3;
  }
#define LDSV_STAGE_CASE(tx, ty)                                                                   \
  if (TX == tx && TY == ty) {                                                                     \
    if (a.fbw && all)                                                                             \
      LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 3, tx, ty, true>), grid, dim3(kBlock), 0, st, p, ph, cb, \
                   nx, ny);                                                                       \
    else if (a.fbw)                                                                               \
      LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 3, tx, ty>), grid, dim3(kBlock), 0, st, p, ph, cb, nx,   \
                   ny);                                                                           \
    else if (a.coef16 && a.dcoef16 && all)                                                        \
      LDSV_TRY((launch_learned_d<T, 5, tx, ty, true>(h, grid, st, p, ph, cb, nx, ny)));           \
    else if (a.coef16 && a.dcoef16)                                                               \
      LDSV_TRY((launch_learned_d<T, 5, tx, ty>(h, grid, st, p, ph, cb, nx, ny)));                 \
    else if (a.coef16 && all)                                                                     \
      LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 2, tx, ty, true>), grid, dim3(kBlock), 0, st, p, ph, cb, \
                   nx, ny);                                                                       \
    else if (a.coef16)                                                                            \
      LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 2, tx, ty>), grid, dim3(kBlock), 0, st, p, ph, cb, nx,   \
                   ny);                                                                           \
    else if (a.coef && a.dcoef && all)                                                            \
      LDSV_TRY((launch_learned_d<T, 4, tx, ty, true>(h, grid, st, p, ph, cb, nx, ny)));           \
    else if (a.coef && a.dcoef)                                                                   \
      LDSV_TRY((launch_learned_d<T, 4, tx, ty>(h, grid, st, p, ph, cb, nx, ny)));                 \
    else if (a.coef && all)                                                                       \
      LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 1, tx, ty, true>), grid, dim3(kBlock), 0, st, p, ph, cb, \
                   nx, ny);                                                                       \
    else if (a.coef)                                                                              \
      LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 1, tx, ty>), grid, dim3(kBlock), 0, st, p, ph, cb, nx,   \
                   ny);                                                                           \
    else if (all)                                                                                 \
      launch_plain_all<T, tx, ty>(h, grid, st, p, ph, cb, nx, ny, rk);                            \
    else                                                                                          \
      LDSV_TLAUNCH(h, 0, (k_stage_mac<T, 0, tx, ty>), grid, dim3(kBlock), 0, st, p, ph, cb, nx,   \
                   ny);                                                                           \
  }
  LDSV_STAGE_CASE(64, 16)
  else LDSV_STAGE_CASE(32, 16) else LDSV_STAGE_CASE(16, 16) else LDSV_STAGE_CASE(8, 16)
  else LDSV_STAGE_CASE(64, 8) else LDSV_STAGE_CASE(32, 8) else LDSV_STAGE_CASE(16, 8)
  else LDSV_STAGE_CASE(8, 8)
  else {
    ldsv_set_error("stage: no tile for %d x %d", nx, ny);
    return LDSV_ESHAPE;
  }
#undef LDSV_STAGE_CASE
  LDSV_LAUNCHED();
  return LDSV_OK;
}

}  // namespace

int ldsv_launch_stage(ldsv_handle* h, const ldsv_params* prm, const StageArgs& a,
                      hipStream_t st) {
  if (h->g.dtype == LDSV_F64) return launch_stage_t<double>(h, prm, a, st);
  return launch_stage_t<float>(h, prm, a, st);
}
