// Host stand-in for <hip/hip_runtime.h>, used only by the CPU check of the pilot-search kernel
// logic (tests/emu).  It runs one 64-lane wavefront as 64 coroutines of one host thread: a
// collective (ballot, shuffle, lane read, wavefront fence) records the lane's value and switches
// back to a scheduler, which resumes every other lane before any lane passes the collective, so the
// kernel code sees the values a wavefront would.  Host API calls and launches are no-ops.
#pragma once
#include <ucontext.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__
#define __align__(x) alignas(x)
#define HIP_SYMBOL(x) x

struct EmuIdx {
  unsigned x = 0, y = 0, z = 0;
};
extern EmuIdx threadIdx, blockIdx, blockDim, gridDim;
struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint2 {
  uint32_t x, y;
};
struct uint4 {
  uint32_t x, y, z, w;
};
typedef int hipError_t;
typedef void* hipStream_t;
enum {
  hipSuccess = 0,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidConfiguration = 9,
  hipDeviceAttributeMultiprocessorCount = 1,
  hipFuncAttributeMaxDynamicSharedMemorySize = 2,
  hipDeviceAttributeMaxSharedMemoryPerBlock = 3
};
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 256; return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, int, int) { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "host emulation"; }
inline hipError_t hipFreeAsync(void*, hipStream_t) { return hipSuccess; }
#define hipLaunchKernelGGL(...) ((void)0)

// The wavefront: one context per lane, the scheduler's context, and one exchange slot per lane.
struct EmuWave {
  ucontext_t sched, lane[64];
  uint64_t slot[64];
};
extern EmuWave* emu_wave;
inline void emu_sync() { swapcontext(&emu_wave->lane[threadIdx.x & 63], &emu_wave->sched); }
template <typename T>
inline T emu_exchange(T v, unsigned src) {
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  emu_wave->slot[threadIdx.x & 63] = u;
  emu_sync();
  const uint64_t r = emu_wave->slot[src & 63];
  emu_sync();
  T out;
  std::memcpy(&out, &r, sizeof(T));
  return out;
}
inline uint64_t __ballot(int pred) {
  emu_wave->slot[threadIdx.x & 63] = pred ? 1 : 0;
  emu_sync();
  uint64_t m = 0;
  for (int l = 0; l < 64; l++) m |= emu_wave->slot[l] << l;
  emu_sync();
  return m;
}
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  (void)width;
  return emu_exchange(v, (unsigned)src);
}
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  (void)width;
  return emu_exchange(v, (threadIdx.x & 63) ^ (unsigned)mask);
}
inline uint32_t emu_readfirstlane(uint32_t v) { return emu_exchange(v, 0); }
inline uint32_t emu_readlane(uint32_t v, uint32_t l) {
  if (l > 63) {
    std::fprintf(stderr, "lane read out of range: %u\n", l);
    std::abort();
  }
  return emu_exchange(v, l);
}
inline uint32_t emu_alignbit(uint32_t a, uint32_t b, uint32_t c) {
  return (uint32_t)((((uint64_t)a << 32) | b) >> (c & 31));
}
#define __builtin_amdgcn_readfirstlane emu_readfirstlane
#define __builtin_amdgcn_readlane emu_readlane
#define __builtin_amdgcn_alignbit emu_alignbit
#define __builtin_amdgcn_fence(...) emu_sync()
#define __builtin_amdgcn_wave_barrier() ((void)0)
inline void __syncthreads() {}
inline void __threadfence_block() {}
inline void __threadfence() {}
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __ffs(int x) { return __builtin_ffs(x); }
inline int __popc(uint32_t x) { return __builtin_popcount(x); }
inline int __popcll(uint64_t x) { return __builtin_popcountll(x); }
inline int __clzll(long long x) { return x ? __builtin_clzll(x) : 64; }
inline float __expf(float x) { return std::exp(x); }
inline float __log2f(float x) { return std::log2(x); }
inline float __logf(float x) { return std::log(x); }
inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
// one host thread runs every lane, so plain read-modify-writes are atomic
template <typename T> inline T atomicAnd(T* p, T v) { T o = *p; *p = o & v; return o; }
template <typename T> inline T atomicOr(T* p, T v) { T o = *p; *p = o | v; return o; }
template <typename T> inline T atomicAdd(T* p, T v) { T o = *p; *p = o + v; return o; }
template <typename T> inline T atomicMin(T* p, T v) { T o = *p; if (v < o) *p = v; return o; }
template <typename T> inline T min(T a, T b) { return a < b ? a : b; }
template <typename T> inline T max(T a, T b) { return a > b ? a : b; }
