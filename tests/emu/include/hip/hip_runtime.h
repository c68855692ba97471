// CPU stand-in for the few HIP device facilities that the batched solver's body logic uses,
// so that isb_body.hpp can be compiled with g++ and run by host threads as one workgroup.
// Test infrastructure only: __syncthreads is a barrier over the workgroup's threads, wavefront
// shuffles go through a per-wave buffer and barrier, and atomics take a mutex.
#pragma once

#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __restrict__

typedef void* hipStream_t;

struct isb_emu_dim3 {
  unsigned x = 0, y = 0, z = 0;
};

extern thread_local isb_emu_dim3 threadIdx;
extern isb_emu_dim3 blockDim;
extern isb_emu_dim3 blockIdx;
extern isb_emu_dim3 gridDim;

namespace isb_emu {
struct Workgroup {
  std::barrier<>* all = nullptr;
  std::vector<std::barrier<>*> waves;
  std::vector<double> buf;
  std::mutex mu;
};
extern Workgroup* g_wg;
}  // namespace isb_emu

inline void __syncthreads() { isb_emu::g_wg->all->arrive_and_wait(); }

inline double __shfl_down(double v, int o, int width) {
  (void)width;
  const unsigned t = threadIdx.x, lane = t & 63, wave = t >> 6;
  auto* wg = isb_emu::g_wg;
  wg->buf[t] = v;
  wg->waves[wave]->arrive_and_wait();
  const double r = (lane + (unsigned)o < 64u) ? wg->buf[wave * 64 + lane + o] : v;
  wg->waves[wave]->arrive_and_wait();
  return r;
}

inline void unsafeAtomicAdd(double* p, double v) {
  std::lock_guard<std::mutex> g(isb_emu::g_wg->mu);
  *p += v;
}

inline int atomicAdd(int* p, int v) {
  std::lock_guard<std::mutex> g(isb_emu::g_wg->mu);
  const int old = *p;
  *p += v;
  return old;
}

using std::fabs;
using std::fmax;
using std::fmin;
using std::isfinite;
using std::sqrt;

// every emulated thread already holds the workgroup-uniform value
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
inline long long __double_as_longlong(double v) {
  long long b;
  std::memcpy(&b, &v, sizeof b);
  return b;
}
inline double __longlong_as_double(long long b) {
  double v;
  std::memcpy(&v, &b, sizeof v);
  return v;
}
