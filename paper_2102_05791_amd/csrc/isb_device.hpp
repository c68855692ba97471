// Device helpers shared by the grid-wide kernels and the persistent batched solver:
// wavefront/block reductions, SoA loads of the element rest data, edge-matrix gathers from the
// [n_v][D] vertex arrays, scatter primitives and the per-vertex energy terms.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "isb_elem.hpp"
#include "isb_internal.hpp"

namespace isb {

// Index checks of the debug build (-DISB_DEBUG; the CPU emulator of the batched solver is built
// with it): an index outside [0, n) stores the number of the check that saw it in g_isb_debug_site
// and reads as 0, so that the code goes on in bounds and the caller can report the site. Without
// ISB_DEBUG a check is the index itself.
#ifdef ISB_DEBUG
__device__ inline int g_isb_debug_site = 0;
__device__ __forceinline__ int isb_checked(int i, int n, int site) {
  if (i < 0 || i >= n) {
    __atomic_store_n(&g_isb_debug_site, site, __ATOMIC_RELAXED);
    return 0;
  }
  return i;
}
#define ISB_CHECKED(i, n, site) ::isb::isb_checked((i), (n), (site))
#else
#define ISB_CHECKED(i, n, site) (i)
#endif

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// sum over the block (blockDim.x == kBlock); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_min(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = v;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) r = fmin(r, sh[w]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ int elem_id(const ERange& r, int k) { return r.list ? r.list[k] : k; }

template <int D>
__device__ __forceinline__ void load_conn(const DevMesh& m, int e, int v[D + 1]) {
#pragma unroll
  for (int k = 0; k <= D; ++k) v[k] = m.conn[(size_t)k * m.n_e + e];
}

// Rest data of element e in the element precision T. CR: the compact record (m.axis >= 0): Dm^-1 and
// W only, the W-scaled material from the mesh's uniform scalars and the fibre vector Dm^-1 d = column
// m.axis of Dm^-1 (in FP64 the same values the general record holds).
template <int D, typename T, bool CR = false>
__device__ __forceinline__ void load_rest(const DevMesh& m, int e, ElemRest<D, T>& R) {
  const size_t ne = (size_t)m.n_e;
  if constexpr (CR) {
    constexpr bool F64 = std::is_same<T, double>::value;
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int c = 0; c < D; ++c)
        R.Dinv[j][c] = F64 ? T(m.Dinv[(size_t)(j * D + c) * ne + e]) : T(m.Dinv32[(size_t)(j * D + c) * ne + e]);
    const T w = F64 ? T(m.W[e]) : T(m.W32[e]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T g = R.Dinv[j][0];
#pragma unroll
      for (int c = 1; c < D; ++c) g = m.axis == c ? R.Dinv[j][c] : g;
      R.gf[j] = g;
    }
    R.wmu = w * T(m.mu_u);
    R.wlam = w * T(m.lam_u);
    R.wkf = w * T(m.kf_u);
  } else if constexpr (std::is_same<T, double>::value) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int c = 0; c < D; ++c) R.Dinv[j][c] = m.Dinv[(size_t)(j * D + c) * ne + e];
      R.gf[j] = m.gf[(size_t)j * ne + e];
    }
    R.wmu = m.wmu[e];
    R.wlam = m.wlam[e];
    R.wkf = m.wkf[e];
  } else {
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int c = 0; c < D; ++c) R.Dinv[j][c] = m.Dinv32[(size_t)(j * D + c) * ne + e];
      R.gf[j] = m.gf32[(size_t)j * ne + e];
    }
    R.wmu = m.wmu32[e];
    R.wlam = m.wlam32[e];
    R.wkf = m.wkf32[e];
  }
}

// Ds[c][j] = x_{v[j+1]} - x_{v[0]}, differences taken in f64 before rounding to T
template <int D, typename T>
__device__ __forceinline__ void gather_edges(const double* __restrict__ x, const int v[D + 1], T Ds[D][D]) {
  double b[D];
#pragma unroll
  for (int c = 0; c < D; ++c) b[c] = x[(size_t)v[0] * D + c];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int c = 0; c < D; ++c) Ds[c][j] = T(x[(size_t)v[j + 1] * D + c] - b[c]);
}

// edges of x + alpha dx
template <int D>
__device__ __forceinline__ void gather_edges_step(const double* __restrict__ x, const double* __restrict__ dx,
                                                  double alpha, const int v[D + 1], double Ds[D][D]) {
  double b[D];
#pragma unroll
  for (int c = 0; c < D; ++c) b[c] = x[(size_t)v[0] * D + c] + alpha * dx[(size_t)v[0] * D + c];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const size_t i = (size_t)v[j + 1] * D + c;
      Ds[c][j] = (x[i] + alpha * dx[i]) - b[c];
    }
}

template <bool ATOMIC>
__device__ __forceinline__ void scatter_add(double* dst, size_t i, double val) {
  if constexpr (ATOMIC)
    unsafeAtomicAdd(dst + i, val);
  else
    dst[i] += val;
}

template <int D, bool ATOMIC, typename T>
__device__ __forceinline__ void scatter_vertices(double* dst, const int v[D + 1], const T out[D + 1][D], double scale) {
#pragma unroll
  for (int k = 0; k <= D; ++k)
#pragma unroll
    for (int c = 0; c < D; ++c) scatter_add<ATOMIC>(dst, (size_t)v[k] * D + c, scale * double(out[k][c]));
}

// per-vertex part of the step objective: s_pot (m g y + k_c ReLU(-y)^2 + k_fr cv |v_t|^2) + 1/2 m |x - xhat|^2
template <int D>
__device__ __forceinline__ double vertex_energy_vals(const DevScene& sc, double mv, double cv, const double* xv,
                                                     const double* x0v, const double* xhv) {
  const double y = xv[1];
  double e = mv * sc.grav * y;
  const double pen = fmax(-y, 0.0);
  e += sc.kc * pen * pen;
  if (sc.kfr != 0.0) {
    double dt2 = 0.0;  // |x_t - x0_t|^2 = h^2 |v_t|^2
#pragma unroll
    for (int c = 0; c < D; ++c)
      if (c != 1) {
        const double dt = xv[c] - x0v[c];
        dt2 += dt * dt;
      }
    e += sc.kfr * cv * dt2 * sc.ih2;
  }
  e *= sc.s_pot;
  if (sc.be) {
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double d = xv[c] - xhv[c];
      d2 += d * d;
    }
    e += 0.5 * mv * d2;
  }
  return e;
}

template <int D>
__device__ __forceinline__ double vertex_energy(const DevMesh& m, const DevScene& sc, int v, const double* xv,
                                                const double* x0, const double* xhat, const double* cv) {
  double x0v[D], xhv[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x0v[c] = x0[(size_t)v * D + c];
    xhv[c] = sc.be ? xhat[(size_t)v * D + c] : 0.0;
  }
  return vertex_energy_vals<D>(sc, m.mass[v], sc.kfr != 0.0 ? cv[v] : 0.0, xv, x0v, xhv);
}

}  // namespace isb
