// Shared device/host helpers for the SBD library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "../../include/sbd.h"

namespace sbd {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename T> using cplx = typename cplx_of<T>::type;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T x, T y) { cplx<T> r; r.x = x; r.y = y; return r; }
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by (dir * i): dir = -1 gives -i, +1 gives +i
template <typename T>
__device__ __forceinline__ cplx<T> cmuli(cplx<T> a, int dir) {
  return dir < 0 ? mk<T>(a.y, -a.x) : mk<T>(-a.y, a.x);
}

#define SBD_HIP_TRY(expr)                                                   \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess) {                                                 \
      sbd::set_last_error(hipGetErrorString(_e), __FILE__, __LINE__);       \
      return SBD_EHIP;                                                      \
    }                                                                       \
  } while (0)

void set_last_error(const char* what, const char* file, int line);

// Record `msg` as the thread's last error and return `st`.
sbd_status fail_with(sbd_status st, const char* msg);

// Optional per-launch timing: when a recorder is installed on this thread,
// every launch site records a HIP event on the launch stream after enqueueing
// its kernel, labelled with the kernel it follows.
struct LaunchMarks;
void mark_launch(const char* name, hipStream_t st, double bytes);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// True if the plan records per-launch timing events (sbd_options.timing / sbd_set_timing).
bool plan_timing(sbd_plan_t plan);
// The plan's permutation (device, [n]: sorted position -> input index of the sources).
const int32_t* plan_perm(sbd_plan_t plan);

// Device memory of the library.  While an AllocStream scope is active on the calling
// thread (sbd_plan runs inside one, on its stream), allocations are stream-ordered
// (hipMallocAsync / hipFreeAsync on that stream) and host uploads are ordered on it too,
// so building a plan never waits for kernels that other streams have in flight (hipFree
// synchronises the whole device).  Outside a scope they are plain hipMalloc / hipFree /
// hipMemcpy.
// Blocks of 32 MiB and more go through the large-block cache while sbd_set_cache_limit holds
// a positive limit.
hipError_t dev_malloc(void** p, size_t bytes);
void dev_free(void* p);
hipError_t dev_upload(void* dst, const void* src, size_t bytes);
struct AllocStream {
  explicit AllocStream(hipStream_t st);
  ~AllocStream();
  hipStream_t prev;
  bool prev_set;
};

}  // namespace sbd
