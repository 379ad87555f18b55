// Support kernels: diagnostics and CFL reductions, fine-to-coarse face
// averaging, corner vorticity, per-snapshot Pearson correlation (App. D.1,
// S36), the MSE rollout loss gradient (Eq. 13), Adam, and bf16 rounding.
#include "reduce.h"
#include "stage.h"

namespace {

template <typename T>
struct DiagF {
  const T* u;
  const T* v;
  int nx, ny;
  double idx, idy;
  int mac;
  __device__ void operator()(int b, size_t i, double* out) const {
    const size_t n = (size_t)nx * ny;
    const T* ub = u + (size_t)b * n;
    const T* vb = v + (size_t)b * n;
    const double a = (double)ub[i], c = (double)vb[i];
    out[0] = fabs(a) + fabs(c);
    out[1] = 0.5 * (a * a + c * c);
    out[2] = a;
    out[3] = c;
    double d = 0.0;
    if (mac) {
      const int x = (int)(i % nx), y = (int)(i / nx);
      const int xp = (x + 1) & (nx - 1), yp = (y + 1) & (ny - 1);
      d = ((double)ub[(size_t)y * nx + xp] - a) * idx + ((double)vb[(size_t)yp * nx + x] - c) * idy;
    }
    out[4] = d * d;
    out[5] = (isfinite(a) && isfinite(c)) ? 0.0 : 1.0;
  }
};

template <typename T>
struct AbsSpeed {
  const T* u;
  const T* v;
  size_t n;
  __device__ void operator()(int b, size_t i, double* out) const {
    out[0] = fabs((double)u[(size_t)b * n + i]) + fabs((double)v[(size_t)b * n + i]);
  }
};

// diag[b][6]: max|u|+|v|, energy, mean u, mean v, ||Du||_2, finite flag
__global__ void k_diag_finish(const double* sums, const double* maxes, double* out, size_t n,
                              int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double* s = sums + (size_t)b * 6;
  const double* m = maxes + (size_t)b * 6;
  double* o = out + (size_t)b * 6;
  o[0] = m[0];
  o[1] = s[1] / (double)n;
  o[2] = s[2] / (double)n;
  o[3] = s[3] / (double)n;
  o[4] = sqrt(s[4]);
  o[5] = (m[5] > 0.0 || !isfinite(s[1])) ? 0.0 : 1.0;
}

template <typename T>
__global__ void k_downsample(const T* uf, const T* vf, T* uc, T* vc, int nxc, int nyc, int r,
                             int batch) {
  const size_t nc = (size_t)nxc * nyc;
  const size_t nf = nc * r * r;
  const int nxf = nxc * r;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nc * batch;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / nc);
    const size_t c = idx - (size_t)b * nc;
    const int I = (int)(c % nxc), J = (int)(c / nxc);
    const T* ub = uf + (size_t)b * nf;
    const T* vb = vf + (size_t)b * nf;
    double su = 0, sv = 0;
    for (int m = 0; m < r; ++m) {
      su += (double)ub[(size_t)(r * J + m) * nxf + r * I];
      sv += (double)vb[(size_t)(r * J) * nxf + r * I + m];
    }
    uc[idx] = (T)(su / r);
    vc[idx] = (T)(sv / r);
  }
}

template <typename T>
__global__ void k_vorticity(const T* u, const T* v, T* w, int nx, int ny, int batch, T idx_,
                            T idy_) {
  const size_t n = (size_t)nx * ny;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n * batch;
       g += (size_t)gridDim.x * blockDim.x) {
    const size_t base = (g / n) * n;
    const size_t c = g - base;
    const int i = (int)(c % nx), j = (int)(c / nx);
    const int im = (i - 1) & (nx - 1), jm = (j - 1) & (ny - 1);
    w[g] = (v[g] - v[base + (size_t)j * nx + im]) * idx_ - (u[g] - u[base + (size_t)jm * nx + i]) * idy_;
  }
}

template <typename T>
struct Moments {
  const T* a;
  const T* b;
  size_t n;
  __device__ void operator()(int t, size_t i, double* out) const {
    const double x = (double)a[(size_t)t * n + i], y = (double)b[(size_t)t * n + i];
    out[0] = x;
    out[1] = y;
    out[2] = x * x;
    out[3] = y * y;
    out[4] = x * y;
  }
};

__global__ void k_pcc_finish(const double* m, double* out, size_t n, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double* s = m + (size_t)b * 5;
  const double mx = s[0] / n, my = s[1] / n;
  const double cxx = s[2] / n - mx * mx, cyy = s[3] / n - my * my, cxy = s[4] / n - mx * my;
  out[b] = cxy / sqrt(cxx * cyy);
}

struct MseF {
  const float* u;
  const float* v;
  const float* lu;
  const float* lv;
  size_t n;
  __device__ void operator()(int b, size_t i, double* out) const {
    const size_t g = (size_t)b * n + i;
    const double du = (double)u[g] - (double)lu[g], dv = (double)v[g] - (double)lv[g];
    out[0] = du * du + dv * dv;
  }
};

__global__ void k_mse_grad(const float* u, const float* v, const float* lu, const float* lv,
                           float* gu, float* gv, size_t total, float s, int accumulate) {
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (size_t)gridDim.x * blockDim.x) {
    const float a = s * (u[g] - lu[g]), b = s * (v[g] - lv[g]);
    gu[g] = accumulate ? gu[g] + a : a;
    gv[g] = accumulate ? gv[g] + b : b;
  }
}

__global__ void k_mse_accum(const double* parts, int batch, double scale, double* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int b = 0; b < batch; ++b) s += parts[b];
    *loss += scale * s;
  }
}

// ob1 = 1 - b1 and ob2 = 1 - b2 come from the host in FP64 rounded once:
// formed here from the FP32 betas they would carry the betas' own rounding
// relative to their small difference (1 - 0.999f is 1.3e-5 away from 1e-3)
__global__ void k_adam(float* w, const float* g, float* m, float* v, size_t n, float b1, float ob1,
                       float b2, float ob2, float c1, float c2, float lr, float eps) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + ob1 * gi;
    const float vi = b2 * v[i] + ob2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// round-to-nearest-even float -> bf16 by the hardware conversion
// (v_cvt_pk_bf16_f32), the same instruction the network kernels use for
// their activations
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const bf16x2_t b = __builtin_convertvector((f32x2_t{f, 0.0f}), bf16x2_t);
  return (uint16_t)(__builtin_bit_cast(uint32_t, b) & 0xffffu);
}

__global__ void k_to_bf16(const float* s, uint16_t* d, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = f32_to_bf16_rne(s[i]);
}

template <typename T>
int diag_t(ldsv_handle* h, const void* u, const void* v, double* out, hipStream_t st) {
  const size_t n = h->ncell;
  const int B = h->g.batch;
  DiagF<T> f{(const T*)u, (const T*)v, h->g.nx, h->g.ny, h->g.nx / h->g.lx, h->g.ny / h->g.ly,
             h->g.layout == LDSV_MAC};
  double* sums = h->small;            // [B][6]
  double* maxes = h->small + 8 * B;   // [B][6]
  LDSV_TRY((reduce_per_traj<kRedSum, 6>(h, f, n, B, sums, st)));
  LDSV_TRY((reduce_per_traj<kRedMax, 6>(h, f, n, B, maxes, st)));
  hipLaunchKernelGGL(k_diag_finish, dim3((B + 63) / 64), dim3(64), 0, st, sums, maxes, out, n, B);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

}  // namespace

int ldsv_launch_diagnostics(ldsv_handle* h, const void* u, const void* v, double* out,
                            hipStream_t st) {
  if (h->g.dtype == LDSV_F64) return diag_t<double>(h, u, v, out, st);
  return diag_t<float>(h, u, v, out, st);
}

int ldsv_launch_maxspeed(ldsv_handle* h, const void* u, const void* v, double* out,
                         hipStream_t st) {
  if (h->g.dtype == LDSV_F64)
    return reduce_per_traj<kRedMax, 1>(h, AbsSpeed<double>{(const double*)u, (const double*)v, h->ncell},
                                       h->ncell, h->g.batch, out, st);
  return reduce_per_traj<kRedMax, 1>(h, AbsSpeed<float>{(const float*)u, (const float*)v, h->ncell},
                                     h->ncell, h->g.batch, out, st);
}

int ldsv_launch_downsample(ldsv_handle* h, int r, const float* uf, const float* vf, float* uc,
                           float* vc, hipStream_t st) {
  hipLaunchKernelGGL(k_downsample<float>, grid1d(h->nstate), dim3(kBlock), 0, st, uf, vf, uc, vc,
                     h->g.nx, h->g.ny, r, h->g.batch);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

int ldsv_launch_vorticity(ldsv_handle* h, const void* u, const void* v, void* w, hipStream_t st) {
  if (h->g.dtype == LDSV_F64)
    hipLaunchKernelGGL(k_vorticity<double>, grid1d(h->nstate), dim3(kBlock), 0, st,
                       (const double*)u, (const double*)v, (double*)w, h->g.nx, h->g.ny,
                       h->g.batch, h->g.nx / h->g.lx, h->g.ny / h->g.ly);
  else
    hipLaunchKernelGGL(k_vorticity<float>, grid1d(h->nstate), dim3(kBlock), 0, st,
                       (const float*)u, (const float*)v, (float*)w, h->g.nx, h->g.ny, h->g.batch,
                       (float)(h->g.nx / h->g.lx), (float)(h->g.ny / h->g.ly));
  LDSV_LAUNCHED();
  return LDSV_OK;
}

int ldsv_launch_pcc(ldsv_handle* h, const void* a, const void* b, double* out, hipStream_t st) {
  const size_t n = h->ncell;
  const int B = h->g.batch;
  if (h->g.dtype == LDSV_F64)
    LDSV_TRY((reduce_per_traj<kRedSum, 5>(h, Moments<double>{(const double*)a, (const double*)b, n},
                                          n, B, h->small, st)));
  else
    LDSV_TRY((reduce_per_traj<kRedSum, 5>(h, Moments<float>{(const float*)a, (const float*)b, n}, n,
                                          B, h->small, st)));
  hipLaunchKernelGGL(k_pcc_finish, dim3((B + 63) / 64), dim3(64), 0, st, h->small, out, n, B);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

int ldsv_launch_mse_grad(ldsv_handle* h, const float* u, const float* v, const float* lu,
                         const float* lv, double scale, float* gu, float* gv, double* loss,
                         hipStream_t st, int accumulate) {
  const size_t total = h->nstate;
  if (loss) {
    LDSV_TRY((reduce_per_traj<kRedSum, 1>(h, MseF{u, v, lu, lv, h->ncell}, h->ncell, h->g.batch,
                                          h->small, st)));
    hipLaunchKernelGGL(k_mse_accum, dim3(1), dim3(64), 0, st, h->small, h->g.batch,
                       0.5 * scale / (double)total, loss);
    LDSV_LAUNCHED();
  }
  if (gu && gv) {
    hipLaunchKernelGGL(k_mse_grad, grid1d(total), dim3(kBlock), 0, st, u, v, lu, lv, gu, gv, total,
                       (float)(scale / (double)total), accumulate);
    LDSV_LAUNCHED();
  }
  return LDSV_OK;
}

extern "C" int ldsv_adam_step(float* w, const float* g, float* m, float* v, size_t n, int t,
                              double lr, double beta1, double beta2, double eps, void* stream) {
  LDSV_REQUIRE(w && g && m && v && t >= 1, LDSV_EINVAL, "adam: null pointer or t < 1");
  const double c1 = 1.0 / (1.0 - pow(beta1, t));
  const double c2 = 1.0 / (1.0 - pow(beta2, t));
  hipLaunchKernelGGL(k_adam, grid1d(n), dim3(kBlock), 0, (hipStream_t)stream, w, g, m, v, n,
                     (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2),
                     (float)c1, (float)c2, (float)lr, (float)eps);
  LDSV_LAUNCHED();
  return LDSV_OK;
}

extern "C" int ldsv_to_bf16(const float* src, uint16_t* dst, size_t n, void* stream) {
  LDSV_REQUIRE(src && dst, LDSV_EINVAL, "to_bf16: null pointer");
  hipLaunchKernelGGL(k_to_bf16, grid1d(n), dim3(kBlock), 0, (hipStream_t)stream, src, dst, n);
  LDSV_LAUNCHED();
  return LDSV_OK;
}
