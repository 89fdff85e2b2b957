// Shared internals of the gfx950 library: error reporting, workspace carving,
// complex helpers, launch geometry and FP64 block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>

#include "../../include/purimi.h"

namespace pr {

void set_error(const char* fmt, ...);
void clear_error();

#define PR_TRY_HIP(call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      ::pr::set_error("%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return PR_EHIP;                                                                 \
    }                                                                                 \
  } while (0)

#define PR_TRY_LAUNCH() PR_TRY_HIP(hipGetLastError())

#define PR_TRY(expr)          \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ != PR_OK) return rc_; \
  } while (0)

#define PR_NONNULL(ptr)                                  \
  do {                                                   \
    if (!(ptr)) {                                        \
      ::pr::set_error("%s: %s is NULL", __func__, #ptr); \
      return PR_EINVAL;                                  \
    }                                                    \
  } while (0)

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// A kernel fault from earlier work is reported before new work is queued.
inline int check_sticky() {
  hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("pending HIP error: %s", hipGetErrorString(e));
    return PR_EHIP;
  }
  return PR_OK;
}

// Calls that copy to or from host memory and wait for the stream refuse a
// stream under graph capture: a captured copy would replay into whatever the
// host address holds later (a stack frame or a freed buffer).
inline int no_capture(hipStream_t s, const char* what) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(s, &st);
  if (e != hipSuccess) {
    set_error("%s: hipStreamIsCapturing: %s", what, hipGetErrorString(e));
    return PR_EHIP;
  }
  if (st != hipStreamCaptureStatusNone) {
    set_error("%s reads results back to the host: not allowed on a stream under graph capture", what);
    return PR_EINVAL;
  }
  return PR_OK;
}

// Bump allocator over a caller-provided workspace. With base == nullptr it
// only measures, so size queries and carving share one code path.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (off + 255) & ~size_t(255); }
};

inline bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

// Pointers read from a table in device memory are generic to the compiler,
// which then emits flat loads and stores; those also count against the LDS
// wait counter, so each wait on an LDS read would wait for memory as well.
// The tables hold global-memory pointers: read them as such. (A kernel that
// chose at run time between such a pointer and a kernel argument would make
// the argument generic too: the kernels that take tables are separate
// instances.)
template <typename T>
__device__ __forceinline__ T* global_ptr_at(T* const* slot) {
  using G = __attribute__((address_space(1))) T*;
  const G g = (G)(*reinterpret_cast<const uintptr_t*>(slot));
  return (T*)g;
}

template <typename R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };
template <typename R> using cx_t = typename Cx<R>::T;

template <typename C> struct CxOf;
template <> struct CxOf<float2> { using R = float; };
template <> struct CxOf<double2> { using R = double; };

template <typename C>
__host__ __device__ inline C cmk(typename CxOf<C>::R re, typename CxOf<C>::R im) {
  C c;
  c.x = re;
  c.y = im;
  return c;
}
template <typename C> __device__ inline C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ inline C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ inline C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ inline C cconj(C a) { return cmk<C>(a.x, -a.y); }
template <typename C> __device__ inline C cscale(C a, typename CxOf<C>::R s) { return cmk<C>(a.x * s, a.y * s); }

// Launch geometry: the chip has 256 compute units in 8 XCDs.
constexpr int kComputeUnits = 256;
constexpr int kXcds = 8;

inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<int>(b);
}

// Deterministic block reduction of one double per thread (fixed tree).
// `sh` must hold blockDim.x doubles. Returns the sum in thread 0.
__device__ inline double block_sum_f64(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

}  // namespace pr
