// Internal declarations of libldsv: the handle, error reporting, complex
// arithmetic and the launch helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldsv.h"

// ---------------------------------------------------------------- errors
void ldsv_set_error(const char* fmt, ...);

#define LDSV_REQUIRE(cond, code, ...)      \
  do {                                     \
    if (!(cond)) {                         \
      ldsv_set_error(__VA_ARGS__);         \
      return (code);                       \
    }                                      \
  } while (0)

#define LDSV_HIP(call)                                                          \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ldsv_set_error("HIP error %d (%s) at %s:%d", (int)e_, hipGetErrorString(e_), \
                     __FILE__, __LINE__);                                       \
      return LDSV_EHIP;                                                         \
    }                                                                           \
  } while (0)

#define LDSV_LAUNCHED() LDSV_HIP(hipGetLastError())

#define LDSV_TRY(expr)          \
  do {                          \
    int s_ = (expr);            \
    if (s_ != LDSV_OK) return s_; \
  } while (0)

// ---------------------------------------------------------------- complex
template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// ---------------------------------------------------------------- timing
// Optional per-kernel-class timing with HIP events recorded on the launch
// stream around each launch (used by the benchmark to measure the dominant
// kernel's average duration inside its timed region).
constexpr int kTimerClasses = 10;
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> ev[kTimerClasses];  // start/stop pairs
  std::vector<hipEvent_t> pool;
};

// ---------------------------------------------------------------- handle
struct ldsv_handle {
  ldsv_grid g;
  int device;
  int log2nx, log2ny;
  size_t ncell;    // nx * ny
  size_t nstate;   // batch * nx * ny
  int npairs;      // ceil(batch / 2): trajectories packed two per complex FFT
  size_t esize;    // sizeof element (4 or 8)

  // workspace (element type = grid dtype)
  void* ws_u = nullptr;   // RK stage state
  void* ws_v = nullptr;
  void* st_u = nullptr;   // pre-projection state u*
  void* st_v = nullptr;
  void* acc_u = nullptr;  // RK accumulator (acc_v follows acc_u contiguously)
  void* acc_v = nullptr;
  void* base_u = nullptr; // copy of u_n when a step runs in place
  void* base_v = nullptr;
  void* zspec = nullptr;  // complex spectrum [npairs][ny][nx]
  void* twx = nullptr;    // exp(-2 pi i m / nx), complex of dtype
  void* twy = nullptr;
  double* pinv = nullptr; // FP64 Poisson factors -1/(lambda_h Nx Ny) [ny][nx] (MAC)
  double* red = nullptr;  // reduction partials
  size_t red_len = 0;
  double* small = nullptr;  // reduction results, 16 doubles per trajectory
  double* small_host = nullptr;  // pinned host mirror of `small`
  int* flag_dev = nullptr;

  // learned-path workspace (F32 MAC grids only)
  uint16_t* act[6] = {nullptr};  // bf16 activations [B][Ny][Nx][64] (input of layer l+1)
  float* pre[5] = {nullptr};     // unused unless backward: pre-activation cache
  float* netout = nullptr;       // [B][66][Ny][Nx]
  uint16_t* coef16 = nullptr;    // bf16 stencil coefficients [B][64][Ny][Nx] (inference)
  float* tcbuf = nullptr;        // temporal correction [B][2][Ny][Nx] (inference)
  float* gnet = nullptr;         // [B][66][Ny][Nx] gradient of network output
  // the derivative-stencil network (allocated on first use): its output in
  // the same two forms, its unused correction planes, its output gradient
  float* dnetout = nullptr;      // [B][66][Ny][Nx]
  uint16_t* dcoef16 = nullptr;   // [B][64][Ny][Nx]
  float* dtcbuf = nullptr;       // [B][2][Ny][Nx]
  float* gdnet = nullptr;        // [B][66][Ny][Nx]
  float* gact = nullptr;         // [B][Ny][Nx][64] float gradient buffers
  float* gact2 = nullptr;
  void* stage_keep = nullptr;    // forward stage states for the adjoint (4 x 2 x state)
  void* adj_u = nullptr;         // adjoint work arrays (2 x state each)
  void* adj_k = nullptr;
  void* adj_g = nullptr;
  void* save_u = nullptr;        // rollout fallback copy of u_{k-1}
  // rollout guard: while speed_out is set, the last projection of an RK4
  // step that runs the one-trajectory kernel (all trajectories active)
  // writes max(|u| + |v|) of each trajectory's new state there (infinity if
  // a value is not finite) and sets speed_written; speed_now is the target
  // the step hands to its last projection
  double* speed_out = nullptr;
  double* speed_now = nullptr;
  bool speed_written = false;
  void* zpre_blk = nullptr;      // network backward workspace
  void* roll_blk = nullptr;      // rollout-backward checkpoints and segment states
  size_t roll_bytes = 0;
  // flux-block workspace (Sec. 3.4 O_L + O_F): per-tile partial sums of the
  // uniform-kernel gradient, the FNO fields of a step and the FNO buffers
  void* fb_part = nullptr;       // [B x tiles][160] of the grid dtype
  float* fb_fields = nullptr;    // [B][8][Ny][Nx]
  float* fb_gfields = nullptr;   // [B][8][Ny][Nx] gradient of the fields
  float* fb_tc = nullptr;        // temporal correction: 2 planes [B][Ny][Nx]
  float* fb_gtc = nullptr;       // its gradient
  float* fb_tmp = nullptr;       // 2 state-sized scratch planes
  void* sc_ws = nullptr;         // passive scalar: two stage states + accumulator
  void* fno_blk = nullptr;       // FNO buffers (fno.hip), fno_bytes long
  size_t fno_bytes = 0;
  size_t bytes = 0;
  std::vector<void*> allocs;     // base pointers of every device allocation owned
  KernelTimer timer;
};

// device allocation owned by the handle (freed by ldsv_destroy)
int ldsv_alloc(ldsv_handle* h, void** p, size_t bytes, const char* what);

// When timing is enabled on the handle, hands out a start/stop event pair
// recorded for kernel class cls and returns true.
bool ldsv_timer_pair(ldsv_handle* h, int cls, hipEvent_t* e0, hipEvent_t* e1);

// Launch a kernel; when the handle's timer is on, the launch carries a pair of
// events that the runtime stamps with that kernel's own start and end.
#define LDSV_TLAUNCH(h, cls, kern, grid, block, shm, st, ...)                        \
  do {                                                                              \
    hipEvent_t e0_, e1_;                                                            \
    if (ldsv_timer_pair((h), (cls), &e0_, &e1_))                                    \
      hipExtLaunchKernelGGL(kern, grid, block, shm, st, e0_, e1_, 0, __VA_ARGS__);   \
    else                                                                            \
      hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);                  \
  } while (0)

int ldsv_check_handle(const ldsv_handle* h);

// device-wide block size
constexpr int kBlock = 256;

// Workgroups are dispatched to the 8 XCDs of the chip round-robin by linear
// workgroup id, and each XCD has its own L2.  For tiled kernels whose tiles
// read halos of their neighbours, renumber the workgroups so that XCD x
// walks the contiguous tile range [x n/8, (x+1) n/8): neighbouring tiles then
// run on the same XCD close together in time and the halo lines are L2 hits
// instead of a second fetch from memory.  The renumbering is a bijection of
// [0, n) (the identity when 8 does not divide n).
__device__ __forceinline__ int xcd_contiguous(int lid, int n) {
  constexpr int kXcd = 8;
  if (n % kXcd) return lid;
  return (lid % kXcd) * (n / kXcd) + lid / kXcd;
}

inline dim3 grid1d(size_t n, int block = kBlock) {
  size_t g = (n + block - 1) / block;
  if (g > 65535u * 64u) g = 65535u * 64u;
  return dim3((unsigned)g);
}
