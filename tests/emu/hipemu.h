// CPU emulation of the small HIP subset used by the library's sources, for
// host-side testing only (logic and bounds checks under AddressSanitizer).
// Never part of the product: the shipped library is built by hipcc for
// gfx950.  Each block runs as blockDim host threads; __syncthreads is a
// barrier over them; blocks run one after another; "device" memory is host
// memory.  Wave operations (__shfl_down/__shfl_xor) assume 64-lane waves
// and wave-uniform control flow: every live lane of the wave reaches them.
#pragma once

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
// Static LDS variables: build_emu.py adds HIPEMU_LDS(name) after each
// declaration; the first thread of a block to pass it fills the variable
// with 0xff bytes (NaN as doubles), since on the device LDS holds whatever
// an earlier kernel left there.
#define HIPEMU_LDS(x) hipemu::lds_fresh((void*)&(x), sizeof(x))
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) ((const void*)&(x))
#define HIP_DYNAMIC_SHARED(type, name) type* name = (type*)hipemu::dyn_lds()

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum {
  hipSuccess = 0,
  hipErrorOutOfMemory = 2,
  hipErrorMemoryAllocation = 2,
  hipErrorInvalidValue = 1,
};
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
#define hipHostMallocDefault 0

namespace hipemu {
extern thread_local dim3 tl_threadIdx, tl_blockIdx;
extern dim3 g_blockDim, g_gridDim;
void barrier();
double shfl_down(double v, int off);
double shfl_xor(double v, int mask);
double quad_perm(double v, int ctrl);
unsigned long long ballot(int pred);
int readlane(int x, int lane);
void wave_sync();
double wave_reduce_add(double v);
typedef double d4 __attribute__((vector_size(4 * sizeof(double))));
d4 mfma_f64_16x16x4(double a, double b, d4 c);
void* dyn_lds();
void lds_fresh(void* p, size_t n);
void launch(dim3 grid, dim3 block, size_t shmem, const std::function<void()>& body);
extern long long g_fail_alloc_after;  // failure injection: fail the k-th allocation (-1: never)
}  // namespace hipemu

#define threadIdx (hipemu::tl_threadIdx)
#define blockIdx (hipemu::tl_blockIdx)
#define blockDim (hipemu::g_blockDim)
#define gridDim (hipemu::g_gridDim)

inline void __syncthreads() { hipemu::barrier(); }
inline void __threadfence_block() {}
inline void __threadfence() {}
// blocks run one after another here, so a plain add is atomic
inline int atomicAdd(int* p, int v) {
  const int o = *p;
  *p = o + v;
  return o;
}
inline double __shfl_down(double v, int off, int = 64) { return hipemu::shfl_down(v, off); }
inline double __shfl_xor(double v, int mask, int = 64) { return hipemu::shfl_xor(v, mask); }
inline unsigned long long __ballot(int pred) { return hipemu::ballot(pred); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
extern "C" double __ockl_wfred_add_f64(double v);
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
// only ever applied to wave-uniform values in the kernels
inline int __builtin_amdgcn_readfirstlane(int x) { return x; }
// every live lane of the wave reaches this point before any goes on
// (wave-synchronous LDS exchanges)
inline void __builtin_amdgcn_wave_barrier() { hipemu::wave_sync(); }
// ordering of memory operations within the wave: the emulated lanes share
// memory directly, so there is nothing to order
inline void __builtin_amdgcn_fence(int, const char*) {}
// value of x in lane `lane` of the wave (lane uniform over the wave)
inline int __builtin_amdgcn_readlane(int x, int lane) { return hipemu::readlane(x, lane); }
// DPP move: quad permutations (dpp_ctrl < 0x100, lane reads lane
// 4*(l/4) + ((ctrl >> 2*(l%4)) & 3) of its wave), row_mirror (0x140) and
// row_half_mirror (0x141)
inline int __builtin_amdgcn_mov_dpp(int src, int ctrl, int, int, bool) {
  return (int)hipemu::quad_perm((double)src, ctrl);
}
inline long long __double_as_longlong(double x) {
  long long r;
  memcpy(&r, &x, 8);
  return r;
}
inline double __longlong_as_double(long long x) {
  double r;
  memcpy(&r, &x, 8);
  return r;
}
// clang's 4 x double vector type, as GCC's generic vector of the same size
// (the kernels only use it for FP64 MFMA accumulators)
#define ext_vector_type(n) vector_size((n) * sizeof(double))
// a cache hint only: a plain load on the host
template <typename T>
inline T __builtin_nontemporal_load(const T* p) {
  return *p;
}
// FP64 16x16x4 matrix FMA over the 64 lanes of a wave: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[l / 16 + 4 i][l % 16]
inline hipemu::d4 __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, hipemu::d4 c, int, int, int) {
  return hipemu::mfma_f64_16x16x4(a, b, c);
}
using std::floor;
using std::copysign;
using std::sin;
using std::fmin;
using std::fmax;

using std::fma;
using std::fabs;
using std::sqrt;
using std::isfinite;
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }

#define hipLaunchKernelGGL(kern, grid, block, shmem, stream, ...) \
  hipemu::launch((grid), (block), (shmem), [&]() { kern(__VA_ARGS__); })
// launch bracketed by two events (recorded on the host clock here)
#define hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, ev0, ev1, flags, ...) \
  do {                                                                                \
    if (ev0) (void)hipEventRecord((ev0), (stream));                                  \
    hipemu::launch((grid), (block), (shmem), [&]() { kern(__VA_ARGS__); });           \
    if (ev1) (void)hipEventRecord((ev1), (stream));                                  \
  } while (0)

hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                            size_t height, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreate(hipStream_t* s);
#define hipStreamNonBlocking 1
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute a, int v);
// a __device__ variable is host memory here: its address is the symbol's
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e);
#define hipEventDisableTiming 2
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags = 0);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
template <typename T>
hipError_t hipMalloc(T** p, size_t n) {
  return hipMalloc((void**)p, n);
}
template <typename T>
hipError_t hipHostMalloc(T** p, size_t n, unsigned flags) {
  return hipHostMalloc((void**)p, n, flags);
}
