// Pressure projection on the periodic MAC grid (App. B.3, S8-S10; App. B.4,
// S11-S14).
//
//   d = D u*   (compact MAC divergence, cell centres)
//   p = (D G)^+ d  by FFT: p_hat = -d_hat / lambda_h(k), p_hat(0) = 0,
//       lambda_h = (2/dx)^2 sin^2(pi kx/Nx) + (2/dy)^2 sin^2(pi ky/Ny)
//   u = u* - G p
//
// Two trajectories are packed into one complex field z = d_b + i d_{b+1}.
// The Poisson multiplier is real and even in k, so the real and imaginary
// parts stay independent through forward FFT, division and inverse FFT;
// this halves the transform work compared with one complex FFT per
// trajectory and needs no real-to-complex unpacking.
//
// Three passes, each one HBM sweep:
//   k_div_rowfft     reads u*, v*; forms d for the pair; FFT along x; writes z
//   k_col_solve      FFT along y, FP64 division (with the 1/(Nx Ny) inverse
//                    normalisation folded in), inverse FFT along y, in place
//   k_rowifft_grad   inverse FFT along x for rows j-1..j+R-1, then
//                    u = u* - (p - p[i-1])/dx, v = v* - (p - p[j-1])/dy
#include "fft_lds.h"

namespace {

template <typename T>
__global__ void __launch_bounds__(kBlock) k_div_rowfft(const T* __restrict__ us,
                                                       const T* __restrict__ vs,
                                                       Cx<T>* __restrict__ z,
                                                       const Cx<T>* __restrict__ twx, int nx,
                                                       int ny, int log2nx, int batch, int rows,
                                                       T idx, T idy) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* A = reinterpret_cast<Cx<T>*>(smem_raw);
  Cx<T>* Bf = A + rows * nx;
  const int pair = blockIdx.y;
  const int b0 = 2 * pair;
  const bool has1 = (b0 + 1) < batch;
  const int j0 = blockIdx.x * rows;
  const size_t plane = (size_t)nx * ny;
  const T* u0 = us + (size_t)b0 * plane;
  const T* v0 = vs + (size_t)b0 * plane;
  const T* u1 = u0 + plane;
  const T* v1 = v0 + plane;
  for (int t = threadIdx.x; t < rows * nx; t += blockDim.x) {
    const int r = t / nx;
    const int i = t - r * nx;
    const int j = j0 + r;
    const int ip = (i + 1) & (nx - 1);
    const int jp = (j + 1) & (ny - 1);
    const size_t c = (size_t)j * nx + i;
    const T d0 = (u0[(size_t)j * nx + ip] - u0[c]) * idx + (v0[(size_t)jp * nx + i] - v0[c]) * idy;
    T d1 = 0;
    if (has1) d1 = (u1[(size_t)j * nx + ip] - u1[c]) * idx + (v1[(size_t)jp * nx + i] - v1[c]) * idy;
    A[t] = Cx<T>{d0, d1};
  }
  __syncthreads();
  Cx<T>* res = lds_fft<T>(A, Bf, nx, log2nx, rows, -1, twx);
  Cx<T>* zo = z + (size_t)pair * plane + (size_t)j0 * nx;
  for (int t = threadIdx.x; t < rows * nx; t += blockDim.x) zo[t] = res[t];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_col_solve(Cx<T>* __restrict__ z,
                                                      const Cx<T>* __restrict__ twy, int nx,
                                                      int ny, int log2ny, int cols, double dx,
                                                      double dy) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* A = reinterpret_cast<Cx<T>*>(smem_raw);
  Cx<T>* Bf = A + cols * ny;
  const int pair = blockIdx.y;
  const int x0 = blockIdx.x * cols;
  Cx<T>* zp = z + (size_t)pair * nx * ny;
  // load columns x0..x0+cols-1 (row segments are contiguous), transpose into LDS
  for (int t = threadIdx.x; t < cols * ny; t += blockDim.x) {
    const int y = t / cols;
    const int c = t - y * cols;
    A[c * ny + y] = zp[(size_t)y * nx + x0 + c];
  }
  __syncthreads();
  Cx<T>* fwd = lds_fft<T>(A, Bf, ny, log2ny, cols, -1, twy);
  Cx<T>* other = (fwd == A) ? Bf : A;
  const double pi = 3.14159265358979323846;
  const double cx = 4.0 / (dx * dx), cy = 4.0 / (dy * dy);
  const double norm = 1.0 / ((double)nx * (double)ny);
  for (int t = threadIdx.x; t < cols * ny; t += blockDim.x) {
    const int c = t / ny;
    const int ky = t - c * ny;
    const int kx = x0 + c;
    const double sx = sin(pi * kx / nx), sy = sin(pi * ky / ny);
    const double lam = cx * sx * sx + cy * sy * sy;
    const double s = (lam > 0.0) ? -norm / lam : 0.0;
    const Cx<T> v = fwd[t];
    fwd[t] = Cx<T>{(T)((double)v.x * s), (T)((double)v.y * s)};
  }
  __syncthreads();
  Cx<T>* inv = lds_fft<T>(fwd, other, ny, log2ny, cols, +1, twy);
  for (int t = threadIdx.x; t < cols * ny; t += blockDim.x) {
    const int y = t / cols;
    const int c = t - y * cols;
    zp[(size_t)y * nx + x0 + c] = inv[c * ny + y];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_rowifft_grad(const Cx<T>* __restrict__ z,
                                                         const Cx<T>* __restrict__ twx,
                                                         const T* __restrict__ us,
                                                         const T* __restrict__ vs,
                                                         T* __restrict__ uo, T* __restrict__ vo,
                                                         T* __restrict__ po, int nx, int ny,
                                                         int log2nx, int batch, int rows, T idx,
                                                         T idy) {
  extern __shared__ unsigned char smem_raw[];
  const int nr = rows + 1;
  Cx<T>* A = reinterpret_cast<Cx<T>*>(smem_raw);
  Cx<T>* Bf = A + nr * nx;
  const int pair = blockIdx.y;
  const int b0 = 2 * pair;
  const bool has1 = (b0 + 1) < batch;
  const int j0 = blockIdx.x * rows;
  const size_t plane = (size_t)nx * ny;
  const Cx<T>* zp = z + (size_t)pair * plane;
  for (int t = threadIdx.x; t < nr * nx; t += blockDim.x) {
    const int r = t / nx;
    const int i = t - r * nx;
    const int j = (j0 - 1 + r + ny) & (ny - 1);
    A[t] = zp[(size_t)j * nx + i];
  }
  __syncthreads();
  const Cx<T>* P = lds_fft<T>(A, Bf, nx, log2nx, nr, +1, twx);
  for (int t = threadIdx.x; t < rows * nx; t += blockDim.x) {
    const int r = t / nx;
    const int i = t - r * nx;
    const int j = j0 + r;
    const int im = (i - 1) & (nx - 1);
    const Cx<T> pc = P[(r + 1) * nx + i];
    const Cx<T> pw = P[(r + 1) * nx + im];
    const Cx<T> ps = P[r * nx + i];
    const size_t c0 = (size_t)b0 * plane + (size_t)j * nx + i;
    uo[c0] = us[c0] - (pc.x - pw.x) * idx;
    vo[c0] = vs[c0] - (pc.x - ps.x) * idy;
    if (po) po[c0] = pc.x;
    if (has1) {
      const size_t c1 = c0 + plane;
      uo[c1] = us[c1] - (pc.y - pw.y) * idx;
      vo[c1] = vs[c1] - (pc.y - ps.y) * idy;
      if (po) po[c1] = pc.y;
    }
  }
}

template <typename T>
int project_impl(ldsv_handle* h, const void* us, const void* vs, void* uo, void* vo, void* po,
                 hipStream_t st) {
  const int nx = h->g.nx, ny = h->g.ny, B = h->g.batch;
  const T idx = (T)(nx / h->g.lx), idy = (T)(ny / h->g.ly);
  const size_t cs = sizeof(Cx<T>);
  // every pass keeps its two LDS buffers within 64 KB
  const size_t kLds = 65536;
  // pass 1 and 3: rows per block (power of two dividing ny) with up to 2048
  // values per block and room for one halo row in pass 3
  int rows = 2048 / nx;
  if (rows < 1) rows = 1;
  if (rows > ny) rows = ny;
  while (rows > 1 && 2 * (size_t)(rows + 1) * nx * cs > kLds) rows >>= 1;
  LDSV_REQUIRE(2 * (size_t)(rows + 1) * nx * cs <= kLds, LDSV_ESHAPE,
               "project: nx=%d too large for the LDS row transform", nx);
  size_t lds = 2 * (size_t)rows * nx * cs;
  LDSV_HIP(hipFuncSetAttribute((const void*)k_div_rowfft<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
  LDSV_TLAUNCH(h, 1, k_div_rowfft<T>, dim3(ny / rows, h->npairs), dim3(kBlock), lds, st,
                     (const T*)us, (const T*)vs, (Cx<T>*)h->zspec, (const Cx<T>*)h->twx, nx, ny,
                     h->log2nx, B, rows, idx, idy);
  }
  LDSV_LAUNCHED();
  // pass 2: columns per block within the LDS budget
  int cols = (int)(kLds / (2 * (size_t)ny * cs));
  LDSV_REQUIRE(cols >= 1, LDSV_ESHAPE, "project: ny=%d too large for the LDS column transform", ny);
  if (cols > nx) cols = nx;
  while (nx % cols) cols >>= 1;
  lds = 2 * (size_t)cols * ny * cs;
  LDSV_HIP(hipFuncSetAttribute((const void*)k_col_solve<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
  LDSV_TLAUNCH(h, 2, k_col_solve<T>, dim3(nx / cols, h->npairs), dim3(kBlock), lds, st,
                     (Cx<T>*)h->zspec, (const Cx<T>*)h->twy, nx, ny, h->log2ny, cols, h->g.lx / nx,
                     h->g.ly / ny);
  }
  LDSV_LAUNCHED();
  // pass 3 (same rows as pass 1)
  lds = 2 * (size_t)(rows + 1) * nx * cs;
  LDSV_HIP(hipFuncSetAttribute((const void*)k_rowifft_grad<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
  LDSV_TLAUNCH(h, 3, k_rowifft_grad<T>, dim3(ny / rows, h->npairs), dim3(kBlock), lds, st,
                     (const Cx<T>*)h->zspec, (const Cx<T>*)h->twx, (const T*)us, (const T*)vs,
                     (T*)uo, (T*)vo, (T*)po, nx, ny, h->log2nx, B, rows, idx, idy);
  }
  LDSV_LAUNCHED();
  return LDSV_OK;
}

}  // namespace

// u*, v* -> projected u, v (may alias u*, v* only if the caller accepts that
// pass 3 reads u*[c] before writing out[c] at the same index, which it does).
int ldsv_launch_project(ldsv_handle* h, const void* us, const void* vs, void* uo, void* vo,
                        void* po, hipStream_t st) {
  if (h->g.dtype == LDSV_F64) return project_impl<double>(h, us, vs, uo, vo, po, st);
  return project_impl<float>(h, us, vs, uo, vo, po, st);
}
