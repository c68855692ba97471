// CPU stand-in for the few HIP device facilities that the batched solver's body logic uses,
// so that isb_body.hpp can be compiled with g++ and run by host threads as one workgroup.
// Test infrastructure only: __syncthreads is a barrier over the workgroup's threads, wavefront
// shuffles and DPP moves go through per-wave buffers and one wave barrier each (two buffers used
// alternately: a lane can only overwrite a buffer after every lane has passed the barrier of the
// operation in between, so after every lane has read it), and atomics take a mutex.
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
typedef int hipError_t;  // only named by declarations of the library's launch functions

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
  std::vector<int> ibuf;
  std::mutex mu;
};
extern Workgroup* g_wg;
extern thread_local unsigned wave_phase;  // wave operations done by this thread (selects the buffer)
}  // namespace isb_emu

inline void __syncthreads() { isb_emu::g_wg->all->arrive_and_wait(); }

inline double __shfl_down(double v, int o, int width) {
  (void)width;
  const unsigned t = threadIdx.x, lane = t & 63, wave = t >> 6;
  auto* wg = isb_emu::g_wg;
  double* b = wg->buf.data() + (isb_emu::wave_phase++ & 1) * blockDim.x;
  b[t] = v;
  wg->waves[wave]->arrive_and_wait();
  return (lane + (unsigned)o < 64u) ? b[wave * 64 + lane + o] : v;
}

// DPP move within a wave of 64 (all lanes active): quad_perm (ctrl <= 0xFF), row_ror:n
// (0x121..0x12F, lane i of a row takes lane i - n of the row), row_bcast:15 (0x142, the last lane
// of the previous row) and row_bcast:31 (0x143, lane 31); lanes in rows outside row_mask keep old
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  (void)bank_mask;
  (void)bound_ctrl;
  const unsigned t = threadIdx.x, lane = t & 63, wave = t >> 6;
  auto* wg = isb_emu::g_wg;
  int* buf = wg->ibuf.data() + (isb_emu::wave_phase++ & 1) * blockDim.x;
  buf[t] = src;
  wg->waves[wave]->arrive_and_wait();
  int r = old;
  const unsigned row = lane >> 4;
  if ((row_mask >> row) & 1) {
    unsigned sl;
    if (ctrl <= 0xFF)
      sl = (lane & ~3u) | ((unsigned)(ctrl >> (2 * (lane & 3))) & 3u);
    else if (ctrl >= 0x121 && ctrl <= 0x12F)
      sl = (lane & ~15u) | ((lane - (unsigned)(ctrl - 0x120)) & 15u);
    else if (ctrl == 0x142)
      sl = row * 16 - 1;
    else if (ctrl == 0x143)
      sl = 31;
    else
      sl = lane;  // not used by the solver
    r = buf[wave * 64 + sl];
  }
  return r;
}

inline int __builtin_amdgcn_readlane(int v, int l) {
  const unsigned t = threadIdx.x, wave = t >> 6;
  auto* wg = isb_emu::g_wg;
  int* buf = wg->ibuf.data() + (isb_emu::wave_phase++ & 1) * blockDim.x;
  buf[t] = v;
  wg->waves[wave]->arrive_and_wait();
  return buf[wave * 64 + l];
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
