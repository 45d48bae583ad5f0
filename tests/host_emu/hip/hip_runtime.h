// Host stand-in for the few HIP names the lean scan's device code uses, so that
// tests can compile that code with g++ and run it on the CPU: one std::thread
// per lane of a 64-lane wave, __ballot over a barrier of the 64 threads.  Test
// infrastructure only (the library itself is built with hipcc for gfx950).
#pragma once
#include <stdint.h>
#include <stdlib.h>
#include <barrier>
#include <atomic>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(x)
enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef void* hipStream_t;
struct uint4 { uint32_t x, y, z, w; };
struct dim3_ { unsigned x, y, z; };
extern thread_local dim3_ threadIdx;
extern std::barrier<>* g_bar;
extern bool g_pred[64];
inline uint64_t __ballot(bool p) {
  g_pred[threadIdx.x & 63] = p;
  g_bar->arrive_and_wait();
  uint64_t m = 0;
  for (int k = 0; k < 64; ++k) m |= (uint64_t)g_pred[k] << k;
  g_bar->arrive_and_wait();
  return m;
}
inline int __popcll(uint64_t v) { return __builtin_popcountll(v); }
template <class T> T __shfl_xor(T, int) { abort(); }
template <class T> T __shfl_up(T, int) { abort(); }
template <class T> T __shfl(T, int) { abort(); }
inline unsigned long long atomicMin(unsigned long long* p, unsigned long long v) {
  unsigned long long o = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (v < o && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {}
  return o;
}
#define __HIP_MEMORY_SCOPE_AGENT 0
template <class T> T __hip_atomic_load(const T* p, int, int) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
template <class T> void __hip_atomic_store(T* p, T v, int, int) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
