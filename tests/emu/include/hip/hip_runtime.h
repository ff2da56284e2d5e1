// CPU stand-in for the part of the HIP runtime and device language that the
// library's sources use, so that the very same kernel sources can be built
// as host code and checked on a CPU: test infrastructure, not a second
// implementation (nothing here computes anything of the method).
//
// Execution model (emu_fiber.cpp): each workgroup runs on one OS thread,
// its GPU threads are fibers that switch at every workgroup barrier and at
// every wavefront-level exchange (shuffles, votes, DPP moves, readlane,
// wave barriers); a workgroup barrier is released only when every live
// thread of the workgroup waits at it, a wavefront exchange when every live
// lane of the wavefront does, and threads waiting at different barriers are
// reported as an error.  Workgroups of a grid run in parallel over a few OS
// threads.  Function-scope __shared__ objects are thread_local statics (one
// copy per OS thread, i.e. per running workgroup); the dynamic LDS array is
// a heap block of exactly the launch's size, filled with NaN bytes when a
// workgroup starts.  Device memory is host heap memory allocated with its
// exact size, so that AddressSanitizer reports any access outside an
// allocation.
#pragma once
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>
#include <stdio.h>
#include <math.h>
#include <cmath>
#include <algorithm>
#include <atomic>
#include <functional>
#include <tuple>
#include <utility>
#include <type_traits>

#define __global__
#define __device__
#define __host__
#define __shared__ static thread_local
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx { unsigned x, y, z; };
extern thread_local EmuIdx threadIdx;
extern thread_local EmuIdx blockIdx;
extern EmuIdx blockDim, gridDim;

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotSupported = 801,
  hipErrorUnknown = 999
} hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef void* hipGraph_t;
typedef void* hipGraphExec_t;
typedef void* hipGraphNode_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal,
                            hipStreamCaptureModeRelaxed };

hipError_t hipMalloc(void** p, size_t n);
template <typename T> inline hipError_t hipMalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), n);
}
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipMemset(void* d, int v, size_t n);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetDevice(int* d);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipGetSymbolAddress(void** p, const void* sym);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* n, char* log, size_t sz);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
template <typename K>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, size_t) {
  *n = 1;
  return hipSuccess;
}

// ---- device side
namespace emu {
void syncthreads();
void wave_sync();
uint64_t wave_exchange(uint64_t v, int src_lane);
int wave_all(int pred);
int lane();
void run_grid(dim3 g, dim3 b, size_t shmem, const std::function<void()>& fn);
}  // namespace emu
extern thread_local char* emu_dyn_lds;   // the launch's dynamic LDS

inline void __syncthreads() { emu::syncthreads(); }
// The lanes of a wavefront execute a fence together on the GPU, so a fence
// orders one lane's stores before other lanes' later loads of the same
// wavefront (the library relies on this after its sweeps' stores); here a
// fence also waits for the rest of the wavefront.  The library's fences are
// reached by every lane of the wavefront.
inline void __threadfence_block() {
  emu::wave_sync();
  std::atomic_thread_fence(std::memory_order_seq_cst);
}
inline void __threadfence() {
  emu::wave_sync();
  std::atomic_thread_fence(std::memory_order_seq_cst);
}

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  static_assert(sizeof(T) <= 8, "shuffle of a value wider than 8 bytes");
  uint64_t b = 0;
  memcpy(&b, &v, sizeof(T));
  const int l = emu::lane();
  const int src = (l & ~(width - 1)) | ((l ^ mask) & (width - 1));
  b = emu::wave_exchange(b, src);
  T r;
  memcpy(&r, &b, sizeof(T));
  return r;
}
inline int __all(int p) { return emu::wave_all(p); }

inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicAdd(unsigned* p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline double atomicAdd(double* p, double v) {
  double old;
  uint64_t ob, nb;
  do {
    old = *p;
    memcpy(&ob, &old, 8);
    const double nv = old + v;
    memcpy(&nb, &nv, 8);
  } while (!__atomic_compare_exchange_n(reinterpret_cast<uint64_t*>(p), &ob, nb, false,
                                        __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST));
  return old;
}
inline float atomicAdd(float* p, float v) {
  uint32_t ob, nb;
  float old;
  do {
    old = *p;
    memcpy(&ob, &old, 4);
    const float nv = old + v;
    memcpy(&nb, &nv, 4);
  } while (!__atomic_compare_exchange_n(reinterpret_cast<uint32_t*>(p), &ob, nb, false,
                                        __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST));
  return old;
}

inline double __hiloint2double(int hi, int lo) {
  const uint64_t b = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  double d;
  memcpy(&d, &b, 8);
  return d;
}
inline int __double2hiint(double d) {
  uint64_t b;
  memcpy(&b, &d, 8);
  return (int)(uint32_t)(b >> 32);
}
inline int __double2loint(double d) {
  uint64_t b;
  memcpy(&b, &d, 8);
  return (int)(uint32_t)b;
}
inline float __int_as_float(int i) {
  float f;
  memcpy(&f, &i, 4);
  return f;
}
inline int __float_as_int(float f) {
  int i;
  memcpy(&i, &f, 4);
  return i;
}

// The library applies readfirstlane to wavefront-uniform values only, so it
// is the identity here.
template <typename T> inline T emu_readfirstlane(T v) { return v; }
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane(v)
inline int emu_readlane(int v, int l) { return (int)emu::wave_exchange((uint32_t)v, l); }
#define __builtin_amdgcn_readlane(v, l) emu_readlane((v), (l))
// The DPP lane moves the library uses: 0x130 wave_shl:1 (lane i reads i + 1),
// 0x134 wave_rol:1 (i reads (i + 1) mod 64), 0x138 wave_shr:1 (i reads i - 1),
// 0x13C wave_ror:1 (i reads (i - 1) mod 64); a source lane outside the
// wavefront gives 0 with bound_ctrl set, else the lane's own old value.
inline int emu_mov_dpp(int v, int ctrl, int, int, bool bound_ctrl) {
  const int l = emu::lane();
  int src = l;
  bool wrap = false;
  switch (ctrl) {
    case 0x130: src = l + 1; break;
    case 0x134: src = l + 1; wrap = true; break;
    case 0x138: src = l - 1; break;
    case 0x13C: src = l - 1; wrap = true; break;
    default: fprintf(stderr, "emu: unsupported dpp control 0x%x\n", ctrl); abort();
  }
  if (wrap) src = (src + 64) % 64;
  const bool out = src < 0 || src > 63;
  const uint32_t r = (uint32_t)emu::wave_exchange((uint32_t)v, out ? 0 : src);
  if (out) return bound_ctrl ? 0 : v;
  return (int)r;
}
#define __builtin_amdgcn_mov_dpp(v, c, rm, bm, bc) emu_mov_dpp((v), (c), (rm), (bm), (bc))
inline void emu_wave_barrier() { emu::wave_sync(); }
#define __builtin_amdgcn_wave_barrier() emu_wave_barrier()
#define __builtin_amdgcn_sched_barrier(m) ((void)0)
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)
inline double emu_rcp(double x) { return 1.0 / x; }
inline float emu_rcp(float x) { return 1.0f / x; }
#define __builtin_amdgcn_rcp(x) emu_rcp(x)
#define __builtin_amdgcn_rcpf(x) emu_rcp(x)

// min / max as HIP's device headers provide them (unqualified)
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }
inline unsigned long min(unsigned long a, unsigned long b) { return a < b ? a : b; }
inline unsigned long max(unsigned long a, unsigned long b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline float min(float a, float b) { return fminf(a, b); }
inline float max(float a, float b) { return fmaxf(a, b); }
inline double min(double a, double b) { return fmin(a, b); }
inline double max(double a, double b) { return fmax(a, b); }
using std::isfinite;
using std::isnan;
using std::isinf;

template <typename... P, typename... A>
inline void emu_launch(void (*k)(P...), dim3 g, dim3 b, size_t shmem, hipStream_t, A&&... args) {
  std::tuple<typename std::decay<P>::type...> params(std::forward<A>(args)...);
  emu::run_grid(g, b, shmem, [&]() { std::apply(k, params); });
}
#define hipLaunchKernelGGL(...) emu_launch(__VA_ARGS__)
