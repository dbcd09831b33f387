// hip/hip_runtime.h for the host-emulation build of the HIP library sources.
//
// The library's kernels and host runtime are compiled as plain C++ for the
// CPU with this header in place of HIP's, so that the same sources run under
// array-bounds checks and with guard pages around every "device" buffer.  A
// kernel launch runs its blocks one after the other; the threads of a block
// run as host threads that meet at __syncthreads (a block barrier) and at the
// wave operations (__ballot, __shfl: a barrier of the 64 lanes of a wave).
// Device memory is host memory; streams, events and copies are synchronous.
// This is a checking tool for the tests: the library built with it is never
// the product.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __host__
// block memory: one section, which the runtime fills with a poison pattern
// before every block (LDS holds no defined value when a block starts)
#define __shared__ static __attribute__((section("hostemu_lds")))
#define __constant__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define __restrict__ __restrict

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct int2 {
  int x, y;
};
struct float4 {
  float x, y, z, w;
};

namespace hostemu {
struct Idx {
  unsigned x = 0, y = 0, z = 0;
};
int lane_index();
int block_threads();
void block_barrier();
int block_or(int p);
unsigned long long wave_ballot(int p);
unsigned long long wave_exchange(unsigned long long v, int src_lane);
void wave_gather(unsigned long long v, unsigned long long* all64);
void run_kernel(dim3 grid, dim3 block, void (*body)(void*), void* ctx);
[[noreturn]] void unsupported(const char* what);

template <class F>
void launch(dim3 grid, dim3 block, F f) {
  run_kernel(grid, block, [](void* p) { (*static_cast<F*>(p))(); }, &f);
}

template <class T>
unsigned long long to_bits(T v) {
  static_assert(sizeof(T) <= 8, "exchange of at most 8 bytes");
  unsigned long long u = 0;
  memcpy(&u, &v, sizeof(T));
  return u;
}
template <class T>
T from_bits(unsigned long long u) {
  T v;
  memcpy(&v, &u, sizeof(T));
  return v;
}
}  // namespace hostemu

extern thread_local hostemu::Idx threadIdx, blockIdx, blockDim, gridDim;

// --- block and wave operations ------------------------------------------------
inline void __syncthreads() { hostemu::block_barrier(); }
inline int __syncthreads_or(int p) { return hostemu::block_or(p); }
inline unsigned long long __ballot(int p) { return hostemu::wave_ballot(p); }
template <class T>
inline T __shfl(T v, int src, int width = 64) {
  const int lane = hostemu::lane_index();
  const int base = lane - lane % width;
  return hostemu::from_bits<T>(hostemu::wave_exchange(hostemu::to_bits(v), base + ((src % width) + width) % width));
}
template <class T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  const int lane = hostemu::lane_index();
  int src = lane ^ mask;
  if (src / width != lane / width) src = lane;
  return hostemu::from_bits<T>(hostemu::wave_exchange(hostemu::to_bits(v), src));
}
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline int __ffs(int v) { return __builtin_ffs(v); }
inline int __clzll(long long v) { return v ? __builtin_clzll((unsigned long long)v) : 64; }
inline unsigned __umulhi(unsigned a, unsigned b) { return (unsigned)(((unsigned long long)a * b) >> 32); }
inline unsigned long long __umul64hi(unsigned long long a, unsigned long long b) {
  return (unsigned long long)(((unsigned __int128)a * b) >> 64);
}

// --- atomics (on any address: "LDS" and "global" memory are host memory) --------
template <class T>
inline T atomicAdd(T* p, T v) {
  if constexpr (std::is_integral<T>::value) {
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
  } else {
    using U = typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned>::type;
    U* q = reinterpret_cast<U*>(p);
    U old = __atomic_load_n(q, __ATOMIC_SEQ_CST);
    for (;;) {
      T f;
      memcpy(&f, &old, sizeof(T));
      T g = f + v;
      U nw;
      memcpy(&nw, &g, sizeof(T));
      if (__atomic_compare_exchange_n(q, &old, nw, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) return f;
    }
  }
}
template <class T>
inline T atomicSub(T* p, T v) { return __atomic_fetch_sub(p, v, __ATOMIC_SEQ_CST); }
template <class T>
inline T atomicCAS(T* p, T cmp, T v) {
  __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
template <class T>
inline T atomicMax(T* p, T v) {
  T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (old < v && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return old;
}
template <class T>
inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline double unsafeAtomicAdd(double* p, double v) { return atomicAdd(p, v); }
inline float unsafeAtomicAdd(float* p, float v) { return atomicAdd(p, v); }
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
inline void __threadfence_block() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }

// --- bit casts and integer helpers ---------------------------------------------
inline unsigned __float_as_uint(float f) { return hostemu::from_bits<unsigned>(hostemu::to_bits(f)); }
inline float __uint_as_float(unsigned u) { return hostemu::from_bits<float>(u); }
inline int __float_as_int(float f) { return hostemu::from_bits<int>(hostemu::to_bits(f)); }
inline float __int_as_float(int u) { return hostemu::from_bits<float>((unsigned)u); }
inline long long __double_as_longlong(double d) { return (long long)hostemu::to_bits(d); }
inline double __longlong_as_double(long long u) { return hostemu::from_bits<double>((unsigned long long)u); }

template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b) {
  typedef typename std::common_type<A, B>::type C;
  return (C)a < (C)b ? (C)a : (C)b;
}
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b) {
  typedef typename std::common_type<A, B>::type C;
  return (C)a < (C)b ? (C)b : (C)a;
}

// --- matrix core: v_mfma_f32_16x16x16bf16_1k on one wave ------------------------
// Lane l holds A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16] (j = 0..3)
// and receives D[4 (l / 16) + j][l % 16] = C + sum_k A[.][k] B[k][.].
namespace hostemu {
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
inline float bf16_to_float(short b) {
  unsigned u = ((unsigned)(unsigned short)b) << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
inline f32x4 mfma_16x16x16_bf16(bf16x4 a, bf16x4 b, f32x4 c, int, int, int) {
  const int lane = lane_index();
  unsigned long long ab = 0, bb = 0;
  memcpy(&ab, &a, 8);
  memcpy(&bb, &b, 8);
  float A[16][16], B[16][16];
  unsigned long long va[64], vb[64];
  wave_gather(ab, va);
  wave_gather(bb, vb);
  for (int l = 0; l < 64; l++) {
    short sa[4], sb[4];
    memcpy(sa, &va[l], 8);
    memcpy(sb, &vb[l], 8);
    for (int j = 0; j < 4; j++) {
      A[l % 16][4 * (l / 16) + j] = bf16_to_float(sa[j]);
      B[4 * (l / 16) + j][l % 16] = bf16_to_float(sb[j]);
    }
  }
  f32x4 d = c;
  for (int j = 0; j < 4; j++) {
    const int row = 4 * (lane / 16) + j, col = lane % 16;
    float s = 0.0f;
    for (int k = 0; k < 16; k++) s += A[row][k] * B[k][col];
    d[j] = c[j] + s;
  }
  return d;
}
}  // namespace hostemu
#define __builtin_amdgcn_mfma_f32_16x16x16bf16_1k hostemu::mfma_16x16x16_bf16

// --- runtime API ------------------------------------------------------------------
typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotSupported = 801,
  hipErrorInvalidSymbol = 13,
  hipErrorUnknown = 999,
} hipError_t;
typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;
typedef enum hipStreamCaptureStatus {
  hipStreamCaptureStatusNone = 0,
  hipStreamCaptureStatusActive = 1,
  hipStreamCaptureStatusInvalidated = 2
} hipStreamCaptureStatus;
typedef enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;
struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph;
struct hipGraphExec;
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;
typedef ihipGraph* hipGraph_t;
typedef hipGraphExec* hipGraphExec_t;
typedef struct ihipGraphNode* hipGraphNode_t;
struct hipDeviceProp_t {
  char name[256];
  int multiProcessorCount;
  size_t totalGlobalMem;
  int warpSize;
};
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
#define HIP_SYMBOL(x) (x)

hipError_t hipMalloc(void** p, size_t n);
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc(reinterpret_cast<void**>(p), n); }
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemset(void* p, int v, size_t n);
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t s);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* n, char* log, size_t sz);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
template <class T>
inline hipError_t hipGetSymbolAddress(void** p, const T& sym) {
  *p = (void*)&sym;
  return hipSuccess;
}

#define hipLaunchKernelGGL(K, G, B, S, ST, ...) \
  ::hostemu::launch(dim3(G), dim3(B), [=]() { K(__VA_ARGS__); })
