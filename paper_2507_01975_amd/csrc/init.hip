// Seeded initial conditions (App. C.1: random fields from fixed seeds;
// S30-S31: shear layers with a perturbation and random noise).
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) seeded
// seed + b * 0xD1B54A32D192ED03 for trajectory b, 53-bit uniforms and the
// Box-Muller transform, drawn on the host (a few thousand numbers).  The mode
// sums are evaluated on the device in FP64, then reduced (FP64,
// deterministic) for the normalisation, then cast to the grid dtype.
//
// Mode order over the half plane: kx = 0..K, ky = -K..K, keeping kx > 0 or
// ky > 0, and kx^2 + ky^2 <= K^2.
#include <cmath>
#include <vector>

#include "reduce.h"
#include "stage.h"

namespace {

struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

struct Normals {
  SplitMix64 g;
  bool have = false;
  double spare = 0;
  Normals(uint64_t seed, int b) { g.s = seed + (uint64_t)b * 0xD1B54A32D192ED03ull; }
  double next() {
    if (have) {
      have = false;
      return spare;
    }
    const double u1 = 1.0 - g.uniform();
    const double u2 = g.uniform();
    const double r = std::sqrt(-2.0 * std::log(u1));
    const double two_pi = 6.283185307179586476925286766559;
    spare = r * std::sin(two_pi * u2);
    have = true;
    return r * std::cos(two_pi * u2);
  }
};

std::vector<int> half_plane(int K) {
  std::vector<int> m;
  for (int kx = 0; kx <= K; ++kx)
    for (int ky = -K; ky <= K; ++ky)
      if ((kx > 0 || ky > 0) && kx * kx + ky * ky <= K * K) {
        m.push_back(kx);
        m.push_back(ky);
      }
  return m;
}

// phase 2 pi (kx X + ky Y) with X = (2i + off)/(2 nx), reduced exactly
__device__ __forceinline__ void phase_sc(int kx, int ky, int i, int j, int off, int nx, int ny,
                                         double* s, double* c) {
  const long long period = 2LL * nx * ny;
  long long m = ((long long)kx * (2 * i + off) * ny + (long long)ky * (2 * j + off) * nx) % period;
  if (m < 0) m += period;
  sincospi(2.0 * (double)m / (double)period, s, c);
}

// sum over modes of a1 cos + a2 sin at corners (off = 0) or centres (off = 1)
// amps layout: [B][ncomp][nmodes][2]; out: [B][ncomp][ny][nx] doubles
__global__ void k_mode_sum(const int* modes, int nmodes, const double* amps, int ncomp, int nx,
                           int ny, int off, int batch, double* out) {
  const size_t n = (size_t)nx * ny;
  const int b = blockIdx.y;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % nx), j = (int)(idx / nx);
    for (int comp = 0; comp < ncomp; ++comp) {
      const double* a = amps + ((size_t)b * ncomp + comp) * nmodes * 2;
      double acc = 0;
      for (int m = 0; m < nmodes; ++m) {
        double s, c;
        phase_sc(modes[2 * m], modes[2 * m + 1], i, j, off, nx, ny, &s, &c);
        acc += a[2 * m] * c + a[2 * m + 1] * s;
      }
      out[((size_t)b * ncomp + comp) * n + idx] = acc;
    }
  }
}

// psi at corners -> u = dpsi/dy at u-points, v = -dpsi/dx at v-points
__global__ void k_vel_from_psi(const double* psi, double* u, double* v, int nx, int ny,
                               double idx_, double idy_) {
  const size_t n = (size_t)nx * ny;
  const int b = blockIdx.y;
  const double* p = psi + (size_t)b * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % nx), j = (int)(idx / nx);
    const int ip = (i + 1) & (nx - 1), jp = (j + 1) & (ny - 1);
    u[(size_t)b * n + idx] = (p[(size_t)jp * nx + i] - p[idx]) * idy_;
    v[(size_t)b * n + idx] = -(p[(size_t)j * nx + ip] - p[idx]) * idx_;
  }
}

struct SqSum {
  const double* u;
  const double* v;
  size_t n;
  __device__ void operator()(int b, size_t i, double* out) const {
    const double a = u[(size_t)b * n + i], c = v[(size_t)b * n + i];
    out[0] = a * a + c * c;
  }
};

struct AbsMax2 {
  const double* u;  // [B][2][n]
  size_t n;
  __device__ void operator()(int b, size_t i, double* out) const {
    out[0] = fmax(fabs(u[((size_t)b * 2) * n + i]), fabs(u[((size_t)b * 2 + 1) * n + i]));
  }
};

// out = scale[b] * (a) (+ profile), cast to T.  mode 0: scale = 1/sqrt(e/(2n)) (unit energy),
// mode 1: scale = 1/max, mode 2: shear: u = prof(y) + s*a, v = pert sin + s*c with
// s = rms_target / sqrt(e/(2n))
template <typename T>
__global__ void k_finalize(const double* a, const double* c, const double* red, int mode,
                           size_t astride, int nx, int ny, double ly, double lx, double delta,
                           double pert, double target, T* u, T* v) {
  const size_t n = (size_t)nx * ny;
  const int b = blockIdx.y;
  double s;
  if (mode == 1) s = 1.0 / red[b];
  else s = target / sqrt(red[b] / (2.0 * (double)n));
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    double uu = s * a[(size_t)b * astride + idx];
    double vv = s * c[(size_t)b * astride + idx];
    if (mode == 2) {
      const int i = (int)(idx % nx), j = (int)(idx / nx);
      const double y = (j + 0.5) * ly / ny;
      const double prof = (y <= 0.5 * ly) ? tanh((y - 0.25 * ly) / delta) : -tanh((y - 0.75 * ly) / delta);
      const double x = (i + 0.5) * lx / nx;
      uu += prof;
      vv += pert * sin(2.0 * 2.0 * 3.14159265358979323846 * x / lx);
    }
    u[(size_t)b * n + idx] = (T)uu;
    v[(size_t)b * n + idx] = (T)vv;
  }
}

template <typename T>
__global__ void k_tgv(T* u, T* v, int nx, int ny, double amp, int k) {
  const size_t n = (size_t)nx * ny;
  const int b = blockIdx.y;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % nx), j = (int)(idx / nx);
    // u at (i, j+1/2), v at (i+1/2, j), arguments in units of pi
    const double xu = 2.0 * k * (double)i / nx, yu = 2.0 * k * (j + 0.5) / ny;
    const double xv = 2.0 * k * (i + 0.5) / nx, yv = 2.0 * k * (double)j / ny;
    u[(size_t)b * n + idx] = (T)(amp * sinpi(xu) * cospi(yu));
    v[(size_t)b * n + idx] = (T)(-amp * cospi(xv) * sinpi(yv));
  }
}

template <typename T>
int init_t(ldsv_handle* h, int kind, uint64_t seed, const ldsv_ic_args& ar, void* u, void* v,
           hipStream_t st) {
  const int nx = h->g.nx, ny = h->g.ny, B = h->g.batch;
  const size_t n = (size_t)nx * ny;
  const dim3 grid((unsigned)((n + kBlock - 1) / kBlock > 4096 ? 4096 : (n + kBlock - 1) / kBlock),
                  B);
  if (kind == LDSV_IC_TGV) {
    hipLaunchKernelGGL(k_tgv<T>, grid, dim3(kBlock), 0, st, (T*)u, (T*)v, nx, ny, ar.amp,
                       (int)ar.k);
    LDSV_LAUNCHED();
    return LDSV_OK;
  }
  // FP64 scratch: up to 3 * B * n doubles in the handle's state buffers
  // (8 contiguous state-sized arrays, at least 4 * B * n doubles).
  double* D = (double*)h->ws_u;
  const size_t Bn = (size_t)B * n;
  std::vector<int> modes;
  std::vector<double> amps;
  if (kind == LDSV_IC_FOURIER_MODES) {
    modes = half_plane(4);
    const int nm = (int)modes.size() / 2;
    amps.resize((size_t)B * 2 * nm * 2);
    for (int b = 0; b < B; ++b) {
      Normals g(seed, b);
      for (size_t q = 0; q < (size_t)2 * nm * 2; ++q) amps[(size_t)b * 2 * nm * 2 + q] = g.next();
    }
  } else {
    int K = 8;
    if (kind == LDSV_IC_GRF_PEAK) {
      K = std::min(16, std::min(nx, ny) / 2 - 1);
      if (K < 1) K = 1;
    }
    modes = half_plane(K);
    const int nm = (int)modes.size() / 2;
    amps.resize((size_t)B * nm * 2);
    for (int b = 0; b < B; ++b) {
      Normals g(seed, b);
      for (int m = 0; m < nm; ++m) {
        double a = 1.0;
        if (kind == LDSV_IC_GRF_PEAK) {
          const double kk = std::sqrt((double)(modes[2 * m] * modes[2 * m] +
                                               modes[2 * m + 1] * modes[2 * m + 1]));
          const double e = std::pow(kk, 4.0) * std::exp(-2.0 * (kk / ar.kpeak) * (kk / ar.kpeak));
          a = std::sqrt(e / (kk * kk * kk));
        }
        const double g1 = g.next();
        const double g2 = g.next();
        amps[((size_t)b * nm + m) * 2] = a * g1;
        amps[((size_t)b * nm + m) * 2 + 1] = a * g2;
      }
    }
  }
  const int nm = (int)modes.size() / 2;
  int* dmodes = nullptr;
  double* damps = nullptr;
  LDSV_HIP(hipMalloc(&dmodes, modes.size() * sizeof(int)));
  LDSV_HIP(hipMalloc(&damps, amps.size() * sizeof(double)));
  LDSV_HIP(hipMemcpyAsync(dmodes, modes.data(), modes.size() * sizeof(int),
                          hipMemcpyHostToDevice, st));
  LDSV_HIP(hipMemcpyAsync(damps, amps.data(), amps.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
  int rc = LDSV_OK;
  if (kind == LDSV_IC_FOURIER_MODES) {
    // trajectory b: u at D[(2b) n], v at D[(2b+1) n], cell centres
    hipLaunchKernelGGL(k_mode_sum, grid, dim3(kBlock), 0, st, dmodes, nm, damps, 2, nx, ny, 1, B, D);
    rc = reduce_per_traj<kRedMax, 1>(h, AbsMax2{D, n}, n, B, h->small, st);
    if (rc == LDSV_OK)
      hipLaunchKernelGGL(k_finalize<T>, grid, dim3(kBlock), 0, st, D, D + n, h->small, 1, 2 * n,
                         nx, ny, h->g.ly, h->g.lx, 0.0, 0.0, 1.0, (T*)u, (T*)v);
  } else {
    // streamfunction at corners -> exactly divergence-free MAC velocities
    hipLaunchKernelGGL(k_mode_sum, grid, dim3(kBlock), 0, st, dmodes, nm, damps, 1, nx, ny, 0, B, D);
    hipLaunchKernelGGL(k_vel_from_psi, grid, dim3(kBlock), 0, st, D, D + Bn, D + 2 * Bn, nx, ny,
                       nx / h->g.lx, ny / h->g.ly);
    rc = reduce_per_traj<kRedSum, 1>(h, SqSum{D + Bn, D + 2 * Bn, n}, n, B, h->small, st);
    if (rc == LDSV_OK) {
      if (kind == LDSV_IC_GRF_PEAK)
        hipLaunchKernelGGL(k_finalize<T>, grid, dim3(kBlock), 0, st, D + Bn, D + 2 * Bn, h->small,
                           0, n, nx, ny, h->g.ly, h->g.lx, 0.0, 0.0, 1.0, (T*)u, (T*)v);
      else
        hipLaunchKernelGGL(k_finalize<T>, grid, dim3(kBlock), 0, st, D + Bn, D + 2 * Bn, h->small,
                           2, n, nx, ny, h->g.ly, h->g.lx, ar.delta, ar.pert, ar.noise_rms,
                           (T*)u, (T*)v);
    }
  }
  hipError_t le = hipGetLastError();
  hipError_t se = hipStreamSynchronize(st);
  hipFree(dmodes);
  hipFree(damps);
  LDSV_HIP(le);
  LDSV_HIP(se);
  return rc;
}

}  // namespace

int ldsv_launch_init(ldsv_handle* h, int kind, uint64_t seed, const ldsv_ic_args* args, void* u,
                     void* v, hipStream_t st) {
  ldsv_ic_args ar{1.0, 1.0, 1.0 / 30.0, 0.05, 1e-3, 4.0};
  if (args) ar = *args;
  if (h->g.dtype == LDSV_F64) return init_t<double>(h, kind, seed, ar, u, v, st);
  return init_t<float>(h, kind, seed, ar, u, v, st);
}
