// ldsv_fv_step_noalloc: the plain/coefficient FV step of ldsv_fv_step for
// callers that cannot allocate device memory.  Every intermediate of the step
// (RK stage states, accumulator, pre-projection state, spectrum, twiddle and
// Poisson-factor tables) lives in `scratch`, a fixed device array of this
// translation unit; the call makes no hipMalloc/hipFree and no allocating
// library call.  The kernels are the ones ldsv_fv_step launches: a handle
// object on the host stack carries the grid's shape and points its
// workspace fields into the array.
#include <cmath>
#include <algorithm>
#include <mutex>

#include "internal.h"

int ldsv_check_grid(const ldsv_grid* g, const char* who);
int ldsv_handle_shape(ldsv_handle* h, const ldsv_grid* g);
int ldsv_check_fv_step(const ldsv_handle* h, const ldsv_params* prm, const float* coef,
                       const void* u_in, const void* v_in, const void* u_out,
                       const void* v_out, int nsteps, const char* who);
int ldsv_internal_step(ldsv_handle* h, const ldsv_params* p, const float* coef, size_t cbs,
                       const void* su, const void* sv, void* du, void* dv, const float* tcu,
                       const float* tcv, size_t tcbs, hipStream_t st);

namespace {

// One copy per device, held until the process ends.  In host code the name
// is only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress (scratch_base below) and is the only form ever passed
// to a kernel or a copy.
__device__ __align__(256) unsigned char scratch[LDSV_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_base[kMaxDevices] = {nullptr};
hipError_t g_base_err[kMaxDevices] = {hipSuccess};

// the array's address on the current device (looked up once per device,
// with that device current)
int scratch_base(void** base) {
  int dev = -1;
  LDSV_HIP(hipGetDevice(&dev));
  LDSV_REQUIRE(dev >= 0 && dev < kMaxDevices, LDSV_EINVAL, "fv_step_noalloc: device %d", dev);
  std::call_once(g_once[dev], [dev] {
    void* p = nullptr;
    g_base_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_base[dev] = (g_base_err[dev] == hipSuccess) ? p : nullptr;
  });
  if (g_base_err[dev] != hipSuccess || !g_base[dev]) {
    (void)hipGetLastError();
    ldsv_set_error("fv_step_noalloc: hipGetSymbolAddress of the scratch array failed: %d (%s)",
                   (int)g_base_err[dev], hipGetErrorString(g_base_err[dev]));
    return LDSV_EHIP;
  }
  *base = g_base[dev];
  return LDSV_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// The tables ldsv_create writes from the host: twiddles exp(-2 pi i m / n) of
// the grid dtype, and the FP64 Poisson factors -1 / (lambda_h Nx Ny) with
// lambda_h = (2/dx)^2 sin^2(pi kx/Nx) + (2/dy)^2 sin^2(pi ky/Ny), zero mode 0.
template <typename T>
__global__ void k_noalloc_tables(Cx<T>* twx, Cx<T>* twy, double* pinv, int nx, int ny, double dx,
                                 double dy) {
  const double two_pi = 6.283185307179586476925286766559;
  const double pi = 3.14159265358979323846;
  const size_t n = (size_t)nx * ny;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + nx + ny;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < (size_t)nx) {
      const double a = two_pi * (double)i / (double)nx;
      twx[i] = Cx<T>{(T)cos(a), (T)(-sin(a))};
    } else if (i < (size_t)(nx + ny)) {
      const int m = (int)(i - nx);
      const double a = two_pi * (double)m / (double)ny;
      twy[m] = Cx<T>{(T)cos(a), (T)(-sin(a))};
    } else if (pinv) {
      const size_t c = i - nx - ny;
      const int kx = (int)(c % nx), ky = (int)(c / nx);
      const double sy = sin(pi * ky / ny);
      const double sx = sin(pi * kx / nx);
      const double lam = 4.0 / (dx * dx) * sx * sx + 4.0 / (dy * dy) * sy * sy;
      pinv[c] = (kx == 0 && ky == 0) ? 0.0 : -(1.0 / ((double)nx * (double)ny)) / lam;
    }
  }
}

// Lays the workspace of grid h->g out in the array starting at base; returns
// the bytes it needs (nothing is written when base is null).
size_t layout_scratch(ldsv_handle* h, char* base) {
  const size_t sb = align256(h->nstate * h->esize);
  const bool mac = h->g.layout == LDSV_MAC;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  h->twx = take((size_t)h->g.nx * 2 * h->esize);
  h->twy = take((size_t)h->g.ny * 2 * h->esize);
  h->pinv = mac ? (double*)take(h->ncell * sizeof(double)) : nullptr;
  h->zspec = mac ? take((size_t)h->npairs * h->ncell * 2 * h->esize) : nullptr;
  h->ws_u = take(sb);
  h->ws_v = take(sb);
  h->st_u = take(sb);
  h->st_v = take(sb);
  h->acc_u = take(sb);
  h->acc_v = take(sb);
  return off;
}

}  // namespace

extern "C" int ldsv_fv_step_noalloc(const ldsv_grid* g, const ldsv_params* prm, const float* coef,
                                    const void* u_in, const void* v_in, void* u_out, void* v_out,
                                    int nsteps, void* stream) {
  LDSV_REQUIRE(g != nullptr, LDSV_EINVAL, "fv_step_noalloc: null grid");
  LDSV_TRY(ldsv_check_grid(g, "fv_step_noalloc"));
  ldsv_handle h;  // shape and workspace pointers only; owns nothing
  LDSV_TRY(ldsv_handle_shape(&h, g));
  LDSV_TRY(ldsv_check_fv_step(&h, prm, coef, u_in, v_in, u_out, v_out, nsteps,
                              "fv_step_noalloc"));
  const size_t need = layout_scratch(&h, nullptr);
  LDSV_REQUIRE(need <= (size_t)LDSV_NOALLOC_SCRATCH_BYTES, LDSV_ESHAPE,
               "fv_step_noalloc: a %dx%d grid of %d trajectories needs %zu bytes of workspace, "
               "more than the %zu-byte scratch array (use ldsv_fv_step)",
               g->nx, g->ny, g->batch, need, (size_t)LDSV_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  LDSV_TRY(scratch_base(&base));
  layout_scratch(&h, (char*)base);
  const hipStream_t st = (hipStream_t)stream;
  // the tables are rewritten on every call: the array keeps whatever the
  // last call on this device left in it
  const size_t nt = h.ncell + g->nx + g->ny;
  const double dx = g->lx / g->nx, dy = g->ly / g->ny;
  const dim3 tg((unsigned)std::min<size_t>((nt + kBlock - 1) / kBlock, 4096));
  if (g->dtype == LDSV_F64)
    hipLaunchKernelGGL(k_noalloc_tables<double>, tg, dim3(kBlock), 0, st, (Cx<double>*)h.twx,
                       (Cx<double>*)h.twy, h.pinv, g->nx, g->ny, dx, dy);
  else
    hipLaunchKernelGGL(k_noalloc_tables<float>, tg, dim3(kBlock), 0, st, (Cx<float>*)h.twx,
                       (Cx<float>*)h.twy, h.pinv, g->nx, g->ny, dx, dy);
  LDSV_LAUNCHED();
  const size_t cbs = (size_t)LDSV_NCOEF * h.ncell;
  for (int k = 0; k < nsteps; ++k) {
    const void* su = (k == 0) ? u_in : u_out;
    const void* sv = (k == 0) ? v_in : v_out;
    LDSV_TRY(ldsv_internal_step(&h, prm, coef, cbs, su, sv, u_out, v_out, nullptr, nullptr, 0,
                                st));
  }
  return LDSV_OK;
}
