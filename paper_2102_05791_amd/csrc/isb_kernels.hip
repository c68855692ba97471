// Grid-wide kernels of the plain (host-driven) solver and the one-off precompute.
//
// Element kernels run one simplex per thread over an element range and scatter their
// per-vertex results either with FP64 global atomics or, when the range is one colour of a
// graph colouring (no two elements share a vertex), with plain read-modify-writes, which is
// race free and bitwise reproducible. Reductions write one partial per block (wavefront
// shuffles, then LDS across the block's waves) and are finished by one block in a fixed
// order, so every sum is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "isb_device.hpp"
#include "isb_elem.hpp"
#include "isb_internal.hpp"
#include "isb_patch.hpp"

namespace isb {

// ---------------------------------------------------------------------------------------------
// host-side grid helpers
// ---------------------------------------------------------------------------------------------
int red_blocks(int n) {
  int b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return b > kMaxRedBlocks ? kMaxRedBlocks : b;
}

static int grid_for(int n) {
  int b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return b > 65535 ? 65535 : b;
}

// ---------------------------------------------------------------------------------------------
// precompute
// ---------------------------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(kBlock) k_precompute_geom(int n_e, const double* __restrict__ X,
                                                            const int32_t* __restrict__ conn, double* Dinv, double* W) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_e; e += gridDim.x * blockDim.x) {
    int v[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) v[k] = conn[(size_t)k * n_e + e];
    double Dm[D][D];
    gather_edges<D, double>(X, v, Dm);
    double C[D][D];
    cofactor<D, double>(Dm, C);
    double det = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) det += Dm[r][0] * C[r][0];
    // Dm^-1 = cof(Dm)^T / det
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int c = 0; c < D; ++c) Dinv[(size_t)(j * D + c) * n_e + e] = C[c][j] / det;
    W[e] = det / (D == 2 ? 2.0 : 6.0);
  }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_precompute_material(int n_e, const double* __restrict__ Dinv,
                                                                const double* __restrict__ W,
                                                                const double* __restrict__ fdir,
                                                                const double* __restrict__ mu,
                                                                const double* __restrict__ lam,
                                                                const double* __restrict__ kf, double* gf, double* wmu,
                                                                double* wlam, double* wkf, float* Dinv32, float* gf32,
                                                                float* wmu32, float* wlam32, float* wkf32) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_e; e += gridDim.x * blockDim.x) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double di = Dinv[(size_t)(j * D + c) * n_e + e];
        acc += di * fdir[(size_t)e * D + c];
        if (Dinv32) Dinv32[(size_t)(j * D + c) * n_e + e] = float(di);
      }
      gf[(size_t)j * n_e + e] = acc;
      if (gf32) gf32[(size_t)j * n_e + e] = float(acc);
    }
    const double w = W[e];
    const double a = w * mu[e], b = w * lam[e], c = w * kf[e];
    wmu[e] = a;
    wlam[e] = b;
    wkf[e] = c;
    if (wmu32) {
      wmu32[e] = float(a);
      wlam32[e] = float(b);
      wkf32[e] = float(c);
    }
  }
}

// one colour of elements: every element adds rho W / (D+1) to each of its vertices
template <int D>
__global__ void __launch_bounds__(kBlock) k_mass_colour(ERange r, const int32_t* __restrict__ conn, int n_e,
                                                        const double* __restrict__ W, const double* __restrict__ rho,
                                                        double* mass) {
  for (int k = r.begin + blockIdx.x * blockDim.x + threadIdx.x; k < r.end; k += gridDim.x * blockDim.x) {
    const int e = elem_id(r, k);
    const double q = rho[e] * W[e] / double(D + 1);
#pragma unroll
    for (int i = 0; i <= D; ++i) mass[conn[(size_t)i * n_e + e]] += q;
  }
}

void launch_precompute_geom(int D, int n_e, const double* X, const int32_t* conn, double* Dinv, double* W,
                            hipStream_t s) {
  if (n_e <= 0) return;
  if (D == 2)
    k_precompute_geom<2><<<grid_for(n_e), kBlock, 0, s>>>(n_e, X, conn, Dinv, W);
  else
    k_precompute_geom<3><<<grid_for(n_e), kBlock, 0, s>>>(n_e, X, conn, Dinv, W);
}

void launch_precompute_material(int D, int n_e, const double* Dinv, const double* W, const double* fdir,
                                const double* mu, const double* lam, const double* kf, double* gf, double* wmu,
                                double* wlam, double* wkf, float* Dinv32, float* gf32, float* wmu32, float* wlam32,
                                float* wkf32, hipStream_t s) {
  if (n_e <= 0) return;
  if (D == 2)
    k_precompute_material<2><<<grid_for(n_e), kBlock, 0, s>>>(n_e, Dinv, W, fdir, mu, lam, kf, gf, wmu, wlam, wkf,
                                                              Dinv32, gf32, wmu32, wlam32, wkf32);
  else
    k_precompute_material<3><<<grid_for(n_e), kBlock, 0, s>>>(n_e, Dinv, W, fdir, mu, lam, kf, gf, wmu, wlam, wkf,
                                                              Dinv32, gf32, wmu32, wlam32, wkf32);
}

void launch_mass_colour(int D, ERange r, const int32_t* conn, int n_e, const double* W, const double* rho,
                        double* mass, hipStream_t s) {
  const int n = r.end - r.begin;
  if (n <= 0) return;
  if (D == 2)
    k_mass_colour<2><<<grid_for(n), kBlock, 0, s>>>(r, conn, n_e, W, rho, mass);
  else
    k_mass_colour<3><<<grid_for(n), kBlock, 0, s>>>(r, conn, n_e, W, rho, mass);
}

// ---------------------------------------------------------------------------------------------
// vertex kernels
// ---------------------------------------------------------------------------------------------
// tangential axes: x in 2D, x and z in 3D
template <int D>
__device__ __forceinline__ bool tangential(int c) {
  return c != 1;
}

// x (the initial iterate), xhat (x0 + h v0) and cv (the friction factor of Eq. 17); x and xhat may be
// null when only cv is wanted
template <int D>
__global__ void __launch_bounds__(kBlock) k_setup(DevMesh m, DevScene sc, int v0, int v1,
                                                  const double* __restrict__ x0, const double* __restrict__ vel0,
                                                  double* x, double* xhat, double* cv) {
  for (int v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const size_t i = (size_t)v * D + c;
      const double xh = (sc.be && vel0) ? x0[i] + sc.h * vel0[i] : x0[i];
      if (xhat) xhat[i] = xh;
      if (x) x[i] = m.pinned[i] ? x0[i] : xh;
    }
    cv[v] = fmax(-x0[(size_t)v * D + 1] + sc.eps, 0.0);
  }
}

// gradient of the vertex terms: s_pot (m g e_y - 2 k_c ReLU(-y) e_y + 2 k_fr cv (x_t - x0_t)/h^2) + m (x - xhat)
template <int D>
__global__ void __launch_bounds__(kBlock) k_vertex_grad(DevMesh m, DevScene sc, int v0, int v1,
                                                        const double* __restrict__ x, const double* __restrict__ x0,
                                                        const double* __restrict__ xhat, const double* __restrict__ cv,
                                                        double* G) {
  const double ih2 = sc.ih2;
  for (int v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += gridDim.x * blockDim.x) {
    const double mv = m.mass[v];
    const double cfr = 2.0 * sc.kfr * cv[v] * ih2;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const size_t i = (size_t)v * D + c;
      double g = 0.0;
      if (c == 1)
        g = mv * sc.grav - 2.0 * sc.kc * fmax(-x[i], 0.0);
      else
        g = cfr * (x[i] - x0[i]);
      g *= sc.s_pot;
      if (sc.be) g += mv * (x[i] - xhat[i]);
      G[i] = g;
    }
  }
}

// diagonal Hessian of the vertex terms (inertia, contact indicator [y < 0], friction); 0 on pinned DOFs
template <int D>
__global__ void __launch_bounds__(kBlock) k_vertex_hdiag(DevMesh m, DevScene sc, int v0, int v1,
                                                         const double* __restrict__ x, const double* __restrict__ cv,
                                                         double* vdiag) {
  const double ih2 = sc.ih2;
  for (int v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += gridDim.x * blockDim.x) {
    const double mv = m.mass[v];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const size_t i = (size_t)v * D + c;
      double hd = (c == 1) ? (x[i] < 0.0 ? 2.0 * sc.kc : 0.0) : 2.0 * sc.kfr * cv[v] * ih2;
      hd *= sc.s_pot;
      if (sc.be) hd += mv;
      vdiag[i] = m.pinned[i] ? 0.0 : hd;
    }
  }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_mask(DevMesh m, int v0, int v1, double* vec) {
  for (int i = v0 * D + blockIdx.x * blockDim.x + threadIdx.x; i < v1 * D; i += gridDim.x * blockDim.x)
    if (m.pinned[i]) vec[i] = 0.0;
}

// Jacobi preconditioner 1/|diag H| (1 where the diagonal vanishes), 0 on pinned DOFs
template <int D>
__global__ void __launch_bounds__(kBlock) k_finish_diag(DevMesh m, int v0, int v1, const double* __restrict__ diag,
                                                        double* Dinvp) {
  for (int i = v0 * D + blockIdx.x * blockDim.x + threadIdx.x; i < v1 * D; i += gridDim.x * blockDim.x) {
    const double d = fabs(diag[i]);
    Dinvp[i] = m.pinned[i] ? 0.0 : (d > 0.0 ? 1.0 / d : 1.0);
  }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_vertex_energy(DevMesh m, DevScene sc, int v0, int v1,
                                                          const double* __restrict__ x, const double* __restrict__ dx,
                                                          double alpha, const double* __restrict__ x0,
                                                          const double* __restrict__ xhat,
                                                          const double* __restrict__ cv, double* partials) {
  __shared__ double sh[kBlock / 64];
  double sd = 0.0, sa = 0.0, st = 0.0;
  for (int v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += gridDim.x * blockDim.x) {
    double xa[D], xb[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const size_t i = (size_t)v * D + c;
      xa[c] = x[i];
      xb[c] = dx ? x[i] + alpha * dx[i] : x[i];
    }
    const double ea = vertex_energy<D>(m, sc, v, xa, x0, xhat, cv);
    const double eb = vertex_energy<D>(m, sc, v, xb, x0, xhat, cv);
    sd += eb - ea;
    sa += fabs(ea);
    st += eb;
  }
  sd = block_sum(sd, sh);
  sa = block_sum(sa, sh);
  st = block_sum(st, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 3 + 0] = sd;
    partials[blockIdx.x * 3 + 1] = sa;
    partials[blockIdx.x * 3 + 2] = st;
  }
}

__global__ void __launch_bounds__(kBlock) k_velocity(int n, const double* __restrict__ x1,
                                                     const double* __restrict__ x0, double inv_h, double* v1) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v1[i] = (x1[i] - x0[i]) * inv_h;
}

// b = x1_bar + v1_bar / h (backward Euler), 0 on pinned DOFs
template <int D>
__global__ void __launch_bounds__(kBlock) k_adjoint_rhs(DevMesh m, DevScene sc, int v0, int v1,
                                                        const double* __restrict__ x1_bar,
                                                        const double* __restrict__ v1_bar, double* b) {
  for (int i = v0 * D + blockIdx.x * blockDim.x + threadIdx.x; i < v1 * D; i += gridDim.x * blockDim.x) {
    double r = x1_bar[i];
    if (sc.be && v1_bar) r += v1_bar[i] / sc.h;
    b[i] = m.pinned[i] ? 0.0 : r;
  }
}

// x0_bar = M w - s_pot (d^2 E_fr / dx dx0)^T w - v1_bar / h ; v0_bar = h M w (backward Euler)
template <int D>
__global__ void __launch_bounds__(kBlock) k_vertex_vjp(DevMesh m, DevScene sc, int v0, int v1,
                                                       const double* __restrict__ w, const double* __restrict__ x1,
                                                       const double* __restrict__ x0,
                                                       const double* __restrict__ v1_bar, double* x0_bar,
                                                       double* v0_bar) {
  const double ih2 = sc.ih2;
  for (int v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += gridDim.x * blockDim.x) {
    const double mv = m.mass[v];
    const size_t b = (size_t)v * D;
    const double y0 = x0[b + 1];
    const double cvv = fmax(-y0 + sc.eps, 0.0);
    const double dcv = (-y0 + sc.eps > 0.0) ? -1.0 : 0.0;
    double xb[D], vb[D];
    double ycross = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      xb[c] = sc.be ? mv * w[b + c] : 0.0;
      vb[c] = sc.be ? sc.h * mv * w[b + c] : 0.0;
      if (sc.be && v1_bar) xb[c] -= v1_bar[b + c] / sc.h;
      if (c != 1 && sc.kfr != 0.0) {
        xb[c] -= sc.s_pot * (-2.0 * sc.kfr * cvv * ih2) * w[b + c];
        ycross += 2.0 * sc.kfr * ih2 * (x1[b + c] - x0[b + c]) * w[b + c];
      }
    }
    xb[1] -= sc.s_pot * ycross * dcv;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const bool pin = m.pinned[b + c];
      if (x0_bar) x0_bar[b + c] = pin ? 0.0 : xb[c];
      if (v0_bar) v0_bar[b + c] = pin ? 0.0 : vb[c];
    }
  }
}

#define DISPATCH_D(D_, KERNEL, GRID, ...)                                 \
  do {                                                                    \
    if ((D_) == 2)                                                        \
      KERNEL<2><<<(GRID), kBlock, 0, s>>>(__VA_ARGS__);                   \
    else                                                                  \
      KERNEL<3><<<(GRID), kBlock, 0, s>>>(__VA_ARGS__);                   \
  } while (0)

void launch_setup(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x0, const double* v0p,
                  double* x, double* xhat, double* cv, hipStream_t s) {
  if (v1 <= v0) return;
  DISPATCH_D(m.dim, k_setup, grid_for(v1 - v0), m, sc, v0, v1, x0, v0p, x, xhat, cv);
}
void launch_vertex_grad(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x, const double* x0,
                        const double* xhat, const double* cv, double* G, hipStream_t s) {
  if (v1 <= v0) return;
  DISPATCH_D(m.dim, k_vertex_grad, grid_for(v1 - v0), m, sc, v0, v1, x, x0, xhat, cv, G);
}
void launch_vertex_hdiag(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x, const double* cv,
                         double* vdiag, hipStream_t s) {
  if (v1 <= v0) return;
  DISPATCH_D(m.dim, k_vertex_hdiag, grid_for(v1 - v0), m, sc, v0, v1, x, cv, vdiag);
}
void launch_mask(const DevMesh& m, int v0, int v1, double* vec, hipStream_t s) {
  if (v1 <= v0) return;
  DISPATCH_D(m.dim, k_mask, grid_for((v1 - v0) * m.dim), m, v0, v1, vec);
}
void launch_finish_diag(const DevMesh& m, int v0, int v1, const double* diag, double* Dinvp, hipStream_t s) {
  if (v1 <= v0) return;
  DISPATCH_D(m.dim, k_finish_diag, grid_for((v1 - v0) * m.dim), m, v0, v1, diag, Dinvp);
}
void launch_vertex_energy(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x, const double* dx,
                          double alpha, const double* x0, const double* xhat, const double* cv, double* partials,
                          int part_off, hipStream_t s, int* nblocks_out) {
  const int nb = red_blocks(v1 - v0);
  DISPATCH_D(m.dim, k_vertex_energy, nb, m, sc, v0, v1, x, dx, alpha, x0, xhat, cv, partials + 3 * part_off);
  *nblocks_out = nb;
}
void launch_velocity(int n, const double* x1, const double* x0, double inv_h, double* v1, hipStream_t s) {
  if (n <= 0) return;
  k_velocity<<<grid_for(n), kBlock, 0, s>>>(n, x1, x0, inv_h, v1);
}
void launch_vertex_vjp(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* w, const double* x1,
                       const double* x0, const double* v1_bar, double* x0_bar, double* v0_bar, hipStream_t s) {
  if (v1 <= v0 || (!x0_bar && !v0_bar)) return;
  DISPATCH_D(m.dim, k_vertex_vjp, grid_for(v1 - v0), m, sc, v0, v1, w, x1, x0, v1_bar, x0_bar, v0_bar);
}
void launch_adjoint_rhs(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x1_bar,
                        const double* v1_bar, double* b, hipStream_t s) {
  if (v1 <= v0) return;
  DISPATCH_D(m.dim, k_adjoint_rhs, grid_for((v1 - v0) * m.dim), m, sc, v0, v1, x1_bar, v1_bar, b);
}

// ---------------------------------------------------------------------------------------------
// element kernels
// ---------------------------------------------------------------------------------------------
template <int D, bool ATOMIC, int EM>
__global__ void __launch_bounds__(kBlock) k_elem_grad(DevMesh m, DevScene sc, ERange r, const double* __restrict__ x,
                                                      const double* __restrict__ a, double* G) {
  for (int k = r.begin + blockIdx.x * blockDim.x + threadIdx.x; k < r.end; k += gridDim.x * blockDim.x) {
    const int e = elem_id(r, k);
    int v[D + 1];
    load_conn<D>(m, e, v);
    ElemRest<D, double> R;
    load_rest<D, double>(m, e, R);
    double Ds[D][D];
    gather_edges<D, double>(x, v, Ds);
    ElemState<D, double> S;
    elem_state<D, double>(Ds, R, S);
    double out[D + 1][D];
    elem_grad<D, double, EM>(R, S, a[e], out);
    scatter_vertices<D, ATOMIC, double>(G, v, out, sc.s_pot);
  }
}

template <int D, bool ATOMIC, typename T, int EM>
__global__ void __launch_bounds__(kBlock) k_elem_hv(DevMesh m, DevScene sc, ERange r, const double* __restrict__ x,
                                                    const double* __restrict__ a, const float* __restrict__ a32,
                                                    const double* __restrict__ p, double* Hp, const int* done) {
  if (done && *done) return;
  for (int k = r.begin + blockIdx.x * blockDim.x + threadIdx.x; k < r.end; k += gridDim.x * blockDim.x) {
    const int e = elem_id(r, k);
    int v[D + 1];
    load_conn<D>(m, e, v);
    ElemRest<D, T> R;
    load_rest<D, T>(m, e, R);
    T Ds[D][D], dDs[D][D];
    gather_edges<D, T>(x, v, Ds);
    gather_edges<D, T>(p, v, dDs);
    ElemState<D, T> S;
    elem_state<D, T>(Ds, R, S);
    const T ae = (std::is_same<T, float>::value && a32) ? T(a32[e]) : T(a[e]);
    T out[D + 1][D];
    elem_hessvec<D, T, EM>(R, S, ae, dDs, out);
    scatter_vertices<D, ATOMIC, T>(Hp, v, out, sc.s_pot);
  }
}

// Hessian diagonal, FP64 in both precisions (the Jacobi preconditioner and isb_hessdiag)
template <int D, bool ATOMIC, int EM>
__global__ void __launch_bounds__(kBlock) k_elem_diag(DevMesh m, DevScene sc, ERange r, const double* __restrict__ x,
                                                      const double* __restrict__ a, double* diag) {
  for (int k = r.begin + blockIdx.x * blockDim.x + threadIdx.x; k < r.end; k += gridDim.x * blockDim.x) {
    const int e = elem_id(r, k);
    int v[D + 1];
    load_conn<D>(m, e, v);
    ElemRest<D, double> R;
    load_rest<D, double>(m, e, R);
    double Ds[D][D];
    gather_edges<D, double>(x, v, Ds);
    ElemState<D, double> S;
    elem_state<D, double>(Ds, R, S);
    double out[D + 1][D];
    elem_hessdiag<D, double, EM>(R, S, a[e], out);
    scatter_vertices<D, ATOMIC, double>(diag, v, out, sc.s_pot);
  }
}

// comps per block: (sum s_pot [E_e(x + alpha dx) - E_e(x)], sum s_pot |E_e(x)|, sum s_pot E_e(x + alpha dx))
template <int D, int EM>
__global__ void __launch_bounds__(kBlock) k_elem_energy(DevMesh m, DevScene sc, ERange r,
                                                        const double* __restrict__ x, const double* __restrict__ dx,
                                                        double alpha, const double* __restrict__ a, double* partials) {
  __shared__ double sh[kBlock / 64];
  double sd = 0.0, sa = 0.0, st = 0.0;
  for (int k = r.begin + blockIdx.x * blockDim.x + threadIdx.x; k < r.end; k += gridDim.x * blockDim.x) {
    const int e = elem_id(r, k);
    int v[D + 1];
    load_conn<D>(m, e, v);
    ElemRest<D, double> R;
    load_rest<D, double>(m, e, R);
    double Ds[D][D];
    gather_edges<D, double>(x, v, Ds);
    ElemState<D, double> S;
    elem_state<D, double>(Ds, R, S);
    const double ea = sc.s_pot * elem_energy<D, double, EM>(R, S, a[e]);
    double eb = ea;
    if (dx) {
      gather_edges_step<D>(x, dx, alpha, v, Ds);
      elem_state<D, double>(Ds, R, S);
      eb = sc.s_pot * elem_energy<D, double, EM>(R, S, a[e]);
    }
    sd += eb - ea;
    sa += fabs(ea);
    st += eb;
  }
  sd = block_sum(sd, sh);
  sa = block_sum(sa, sh);
  st = block_sum(st, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 3 + 0] = sd;
    partials[blockIdx.x * 3 + 1] = sa;
    partials[blockIdx.x * 3 + 2] = st;
  }
}

template <int D, int EM>
__global__ void __launch_bounds__(kBlock) k_elem_vjp(DevMesh m, DevScene sc, ERange r, const double* __restrict__ w,
                                                     const double* __restrict__ x1, const double* __restrict__ a,
                                                     double* a_bar, double* mu_bar, double* lam_bar, double* kf_bar) {
  for (int k = r.begin + blockIdx.x * blockDim.x + threadIdx.x; k < r.end; k += gridDim.x * blockDim.x) {
    const int e = elem_id(r, k);
    int v[D + 1];
    load_conn<D>(m, e, v);
    ElemRest<D, double> R;
    load_rest<D, double>(m, e, R);
    double Ds[D][D], dWs[D][D];
    gather_edges<D, double>(x1, v, Ds);
    gather_edges<D, double>(w, v, dWs);
    ElemState<D, double> S;
    elem_state<D, double>(Ds, R, S);
    double out[4];
    elem_vjp<D, double, EM>(R, S, m.W[e], a[e], dWs, out);
    if (a_bar) a_bar[e] = sc.s_pot * out[0];
    if (mu_bar) mu_bar[e] = sc.s_pot * out[1];
    if (lam_bar) lam_bar[e] = sc.s_pot * out[2];
    if (kf_bar) kf_bar[e] = sc.s_pot * out[3];
  }
}

// per block (min J, -max J) so that both finish with a min-reduction
template <int D>
__global__ void __launch_bounds__(kBlock) k_elem_minmax_J(DevMesh m, ERange r, const double* __restrict__ x,
                                                          double* partials) {
  __shared__ double sh[kBlock / 64];
  double lo = 1e300, nhi = 1e300;
  for (int k = r.begin + blockIdx.x * blockDim.x + threadIdx.x; k < r.end; k += gridDim.x * blockDim.x) {
    const int e = elem_id(r, k);
    int v[D + 1];
    load_conn<D>(m, e, v);
    ElemRest<D, double> R;
    load_rest<D, double>(m, e, R);
    double Ds[D][D];
    gather_edges<D, double>(x, v, Ds);
    ElemState<D, double> S;
    elem_state<D, double>(Ds, R, S);
    lo = fmin(lo, S.J);
    nhi = fmin(nhi, -S.J);
  }
  lo = block_min(lo, sh);
  nhi = block_min(nhi, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 2 + 0] = lo;
    partials[blockIdx.x * 2 + 1] = nhi;
  }
}

__global__ void __launch_bounds__(kBlock) k_to_f32(int n, const double* __restrict__ src, float* dst) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = float(src[i]);
}

// calls fn(std::integral_constant<int, EM>) for the energy model of the mesh
template <class Fn>
static void with_model(int model, Fn&& fn) {
  switch (model) {
    case EM_STVK: fn(std::integral_constant<int, EM_STVK>{}); break;
    case EM_COROT: fn(std::integral_constant<int, EM_COROT>{}); break;
    case EM_SNH: fn(std::integral_constant<int, EM_SNH>{}); break;
    default: fn(std::integral_constant<int, EM_NH>{}); break;
  }
}

template <int D>
static void elem_grad_d(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, const double* x, const double* a,
                        double* G, hipStream_t s) {
  const int g = grid_for(r.end - r.begin);
  with_model(m.model, [&](auto em) {
    constexpr int EM = decltype(em)::value;
    if (atomic)
      k_elem_grad<D, true, EM><<<g, kBlock, 0, s>>>(m, sc, r, x, a, G);
    else
      k_elem_grad<D, false, EM><<<g, kBlock, 0, s>>>(m, sc, r, x, a, G);
  });
}

void launch_elem_grad(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, const double* x, const double* a,
                      double* G, hipStream_t s) {
  if (r.end <= r.begin) return;
  if (m.dim == 2)
    elem_grad_d<2>(m, sc, r, atomic, x, a, G, s);
  else
    elem_grad_d<3>(m, sc, r, atomic, x, a, G, s);
}

template <int D, typename T>
static void elem_hv_dt(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, const double* x, const double* a,
                       const float* a32, const double* p, double* Hp, const int* done, hipStream_t s) {
  const int g = grid_for(r.end - r.begin);
  with_model(m.model, [&](auto em) {
    constexpr int EM = decltype(em)::value;
    if (atomic)
      k_elem_hv<D, true, T, EM><<<g, kBlock, 0, s>>>(m, sc, r, x, a, a32, p, Hp, done);
    else
      k_elem_hv<D, false, T, EM><<<g, kBlock, 0, s>>>(m, sc, r, x, a, a32, p, Hp, done);
  });
}

void launch_elem_hv(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, int precision, const double* x,
                    const double* a, const float* a32, const double* p, double* Hp, const int* done, hipStream_t s) {
  if (r.end <= r.begin) return;
  if (m.dim == 2) {
    if (precision)
      elem_hv_dt<2, float>(m, sc, r, atomic, x, a, a32, p, Hp, done, s);
    else
      elem_hv_dt<2, double>(m, sc, r, atomic, x, a, a32, p, Hp, done, s);
  } else {
    if (precision)
      elem_hv_dt<3, float>(m, sc, r, atomic, x, a, a32, p, Hp, done, s);
    else
      elem_hv_dt<3, double>(m, sc, r, atomic, x, a, a32, p, Hp, done, s);
  }
}

template <int D>
static void elem_diag_d(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, const double* x,
                        const double* a, double* diag, hipStream_t s) {
  const int g = grid_for(r.end - r.begin);
  with_model(m.model, [&](auto em) {
    constexpr int EM = decltype(em)::value;
    if (atomic)
      k_elem_diag<D, true, EM><<<g, kBlock, 0, s>>>(m, sc, r, x, a, diag);
    else
      k_elem_diag<D, false, EM><<<g, kBlock, 0, s>>>(m, sc, r, x, a, diag);
  });
}

void launch_elem_diag(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, const double* x, const double* a,
                      double* diag, hipStream_t s) {
  if (r.end <= r.begin) return;
  if (m.dim == 2)
    elem_diag_d<2>(m, sc, r, atomic, x, a, diag, s);
  else
    elem_diag_d<3>(m, sc, r, atomic, x, a, diag, s);
}

void launch_elem_energy(const DevMesh& m, const DevScene& sc, ERange r, const double* x, const double* dx,
                        double alpha, const double* a, double* partials, int part_off, hipStream_t s,
                        int* nblocks_out) {
  const int nb = red_blocks(r.end - r.begin);
  with_model(m.model, [&](auto em) {
    constexpr int EM = decltype(em)::value;
    if (m.dim == 2)
      k_elem_energy<2, EM><<<nb, kBlock, 0, s>>>(m, sc, r, x, dx, alpha, a, partials + 3 * part_off);
    else
      k_elem_energy<3, EM><<<nb, kBlock, 0, s>>>(m, sc, r, x, dx, alpha, a, partials + 3 * part_off);
  });
  *nblocks_out = nb;
}

void launch_elem_vjp(const DevMesh& m, const DevScene& sc, ERange r, const double* w, const double* x1,
                     const double* a, double* a_bar, double* mu_bar, double* lam_bar, double* kf_bar, hipStream_t s) {
  if (r.end <= r.begin) return;
  const int g = grid_for(r.end - r.begin);
  with_model(m.model, [&](auto em) {
    constexpr int EM = decltype(em)::value;
    if (m.dim == 2)
      k_elem_vjp<2, EM><<<g, kBlock, 0, s>>>(m, sc, r, w, x1, a, a_bar, mu_bar, lam_bar, kf_bar);
    else
      k_elem_vjp<3, EM><<<g, kBlock, 0, s>>>(m, sc, r, w, x1, a, a_bar, mu_bar, lam_bar, kf_bar);
  });
}

void launch_elem_minmax_J(const DevMesh& m, ERange r, const double* x, double* partials, hipStream_t s,
                          int* nblocks_out) {
  const int nb = red_blocks(r.end - r.begin);
  DISPATCH_D(m.dim, k_elem_minmax_J, nb, m, r, x, partials);
  *nblocks_out = nb;
}

void launch_to_f32(int n, const double* src, float* dst, hipStream_t s) {
  if (n <= 0) return;
  k_to_f32<<<grid_for(n), kBlock, 0, s>>>(n, src, dst);
}

// ---------------------------------------------------------------------------------------------
// reductions and vector kernels
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                                double* partials) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc += a[i] * b[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// out[c] = sum_b partials[b * ncomp + c], in block order
__global__ void __launch_bounds__(kBlock) k_finalize(const double* __restrict__ partials, int nblocks, int ncomp,
                                                     double* out) {
  __shared__ double sh[kBlock / 64];
  for (int c = 0; c < ncomp; ++c) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += partials[b * ncomp + c];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[c] = acc;
  }
}

__global__ void __launch_bounds__(kBlock) k_finalize_minmax(const double* __restrict__ partials, int nblocks,
                                                            double* out) {
  __shared__ double sh[kBlock / 64];
  double lo = 1e300, nhi = 1e300;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    lo = fmin(lo, partials[2 * b]);
    nhi = fmin(nhi, partials[2 * b + 1]);
  }
  lo = block_min(lo, sh);
  nhi = block_min(nhi, sh);
  if (threadIdx.x == 0) {
    out[0] = lo;
    out[1] = -nhi;
  }
}

__global__ void __launch_bounds__(kBlock) k_axpy(int n, double* x, double alpha, const double* __restrict__ dx) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] += alpha * dx[i];
}

__global__ void __launch_bounds__(kBlock) k_copy(int n, const double* __restrict__ src, double* dst) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// sum of the first nb partials (two components interleaved when ncomp == 2), identical in every block
__device__ __forceinline__ double all_blocks_sum(const double* partials, int nb, int ncomp, int c, double* sh) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partials[b * ncomp + c];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) sh[kBlock / 64] = acc;
  __syncthreads();
  const double r = sh[kBlock / 64];
  __syncthreads();
  return r;
}

// the sums of the first nb pairs of interleaved partials in one pass and one block reduction,
// identical in every block; sh: 2 * (kBlock / 64) + 2 values
__device__ __forceinline__ void all_blocks_sum2(const double* partials, int nb, double* sh, double& a, double& b) {
  double v0 = 0.0, v1 = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    v0 += partials[2 * k];
    v1 += partials[2 * k + 1];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  if (lane == 0) {
    sh[2 * wid] = v0;
    sh[2 * wid + 1] = v1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[2 * w + threadIdx.x];
    sh[2 * (kBlock / 64) + threadIdx.x] = t;
  }
  __syncthreads();
  a = sh[2 * (kBlock / 64)];
  b = sh[2 * (kBlock / 64) + 1];
  __syncthreads();
}

// this block's sums of two values into out[2 * blockIdx.x + k] (one barrier); sh: 2 * (kBlock / 64)
__device__ __forceinline__ void block_partials2(double a, double b, double* sh, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    sh[2 * wid] = a;
    sh[2 * wid + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[2 * w + threadIdx.x];
    out[2 * blockIdx.x + threadIdx.x] = t;
  }
}

// r = b, x = 0, p = D^-1 r, Hp = vdiag p; partials (r.z, r.r); a single block then fills scal
__global__ void __launch_bounds__(kBlock) k_cg_start(int n, const double* __restrict__ b, double sign,
                                                     const double* __restrict__ Dinvp,
                                                     const double* __restrict__ vdiag, double* r, double* p, double* xs,
                                                     double* Hp, double* partials) {
  __shared__ double sh[2 * (kBlock / 64)];
  double rz = 0.0, rr = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double ri = Dinvp[i] != 0.0 ? sign * b[i] : 0.0;
    const double zi = Dinvp[i] * ri;
    r[i] = ri;
    p[i] = zi;
    xs[i] = 0.0;
    Hp[i] = vdiag[i] * zi;
    rz += ri * zi;
    rr += ri * ri;
  }
  block_partials2(rz, rr, sh, partials);
}

__global__ void __launch_bounds__(kBlock) k_cg_start_fin(const double* __restrict__ partials, int nb, CgScal* scal,
                                                         double tol2, int max_it) {
  __shared__ double sh[2 * (kBlock / 64) + 2];
  double rz, rr;
  all_blocks_sum2(partials, nb, sh, rz, rr);
  if (threadIdx.x == 0) {
    scal->rz[0] = rz;
    scal->rr = rr;
    scal->rr0 = rr;
    scal->pHp = 0.0;
    scal->tol2 = tol2;
    scal->max_it = max_it;
    scal->done = (rr <= tol2 || max_it <= 0) ? 1 : 0;
    scal->negcurv = 0;
    scal->iters = 0;
    scal->it_cur = 0;
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_dot(int n, const double* __restrict__ p, const double* __restrict__ Hp,
                                                   double* partials, const CgScal* scal) {
  if (scal->done) return;
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc += p[i] * Hp[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// alpha = rz / pHp; x += alpha p; r -= alpha Hp (masked by D^-1 != 0); partials (r.z, r.r)
__global__ void __launch_bounds__(kBlock) k_cg_update(int n, int nb, const double* __restrict__ p,
                                                      const double* __restrict__ Hp, const double* __restrict__ Dinvp,
                                                      double* r, double* xs, double* partials, CgScal* scal) {
  if (scal->done) return;
  const int it = scal->iters;
  __shared__ double sh[2 * (kBlock / 64) + 2];
  const double pHp = all_blocks_sum(partials, nb, 1, 0, sh);
  __syncthreads();  // every block has read its partials before any overwrites them below
  const double rz = scal->rz[it & 1];
  if (!(pHp > 0.0)) {
    // non-positive curvature: stop; on the first iteration return the preconditioned
    // steepest-descent direction p0 = D^-1 b (Nocedal & Wright, Alg. 7.1)
    if (it == 0)
      for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) xs[i] = p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scal->negcurv = 1;
      scal->done = 1;
      scal->pHp = pHp;
      scal->iters = it;
    }
    return;
  }
  const double alpha = rz / pHp;
  double rz1 = 0.0, rr = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double di = Dinvp[i];
    xs[i] += alpha * p[i];
    const double ri = di != 0.0 ? r[i] - alpha * Hp[i] : 0.0;
    r[i] = ri;
    rz1 += ri * di * ri;
    rr += ri * ri;
  }
  // the partials buffer is reused: this kernel reads nb single partials, then writes 2 per block
  block_partials2(rz1, rr, sh, partials + kMaxRedBlocks);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal->pHp = pHp;
    scal->it_cur = it;
  }
}

// beta = rz_new / rz; p = D^-1 r + beta p; Hp = vdiag p (the start of the next product)
__global__ void __launch_bounds__(kBlock) k_cg_p(int n, int nb, const double* __restrict__ r,
                                                 const double* __restrict__ Dinvp, const double* __restrict__ vdiag,
                                                 double* p, double* Hp, const double* __restrict__ partials,
                                                 CgScal* scal) {
  if (scal->done) return;
  const int it = scal->it_cur;
  const double tol2 = scal->tol2;
  __shared__ double sh[2 * (kBlock / 64) + 2];
  double rz1, rr;
  all_blocks_sum2(partials + kMaxRedBlocks, nb, sh, rz1, rr);
  if (rr <= tol2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scal->done = 1;
      scal->rr = rr;
      scal->iters = it + 1;
    }
    return;
  }
  const double beta = rz1 / scal->rz[it & 1];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double pi = Dinvp[i] * r[i] + beta * p[i];
    p[i] = pi;
    Hp[i] = vdiag[i] * pi;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal->rz[(it + 1) & 1] = rz1;
    scal->rr = rr;
    scal->iters = it + 1;
    if (it + 1 >= scal->max_it) scal->done = 1;  // the cap: rr above tol2 tells the host it did not converge
  }
}

void launch_dot(int n, const double* a, const double* b, double* partials, hipStream_t s, int* nblocks_out) {
  const int nb = red_blocks(n);
  k_dot<<<nb, kBlock, 0, s>>>(n, a, b, partials);
  *nblocks_out = nb;
}
void launch_finalize(const double* partials, int nblocks, int ncomp, double* out, hipStream_t s) {
  k_finalize<<<1, kBlock, 0, s>>>(partials, nblocks, ncomp, out);
}
void launch_finalize_minmax(const double* partials, int nblocks, double* out, hipStream_t s) {
  k_finalize_minmax<<<1, kBlock, 0, s>>>(partials, nblocks, out);
}
void launch_axpy(int n, double* x, double alpha, const double* dx, hipStream_t s) {
  if (n <= 0) return;
  k_axpy<<<grid_for(n), kBlock, 0, s>>>(n, x, alpha, dx);
}
// Streaming copy for the bandwidth probe: one 16-byte element per thread over as many workgroups as
// the data needs (up to 2^30, then each thread takes further elements a grid apart). On gfx950 this
// short-lived-workgroup form streams faster than a persistent grid-stride loop.
__global__ void __launch_bounds__(256) k_stream_copy(int64_t n2, const double2* __restrict__ src,
                                                     double2* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) dst[i] = src[i];
}

__global__ void k_copy_tail(const double* src, double* dst) { dst[0] = src[0]; }

void launch_stream_copy(int64_t n, const double* src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    const int grid = (int)std::min<int64_t>((n2 + 255) / 256, (int64_t)1 << 30);
    k_stream_copy<<<grid, 256, 0, s>>>(n2, reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst));
  }
  if (n & 1) k_copy_tail<<<1, 1, 0, s>>>(src + n - 1, dst + n - 1);
}

void launch_copy(int n, const double* src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  k_copy<<<grid_for(n), kBlock, 0, s>>>(n, src, dst);
}
void launch_cg_start(int n, const double* b, double sign, const double* Dinvp, const double* vdiag, double* r,
                     double* p, double* xs, double* Hp, double* partials, CgScal* scal, double tol2, int max_it,
                     hipStream_t s) {
  const int nb = red_blocks(n);
  k_cg_start<<<nb, kBlock, 0, s>>>(n, b, sign, Dinvp, vdiag, r, p, xs, Hp, partials);
  k_cg_start_fin<<<1, kBlock, 0, s>>>(partials, nb, scal, tol2, max_it);
}
void launch_cg_dot(int n, const double* p, const double* Hp, double* partials, const CgScal* scal, hipStream_t s) {
  k_cg_dot<<<red_blocks(n), kBlock, 0, s>>>(n, p, Hp, partials, scal);
}
void launch_cg_update(int n, const double* p, const double* Hp, const double* Dinvp, double* r, double* xs,
                      double* partials, CgScal* scal, hipStream_t s) {
  const int nb = red_blocks(n);
  k_cg_update<<<nb, kBlock, 0, s>>>(n, nb, p, Hp, Dinvp, r, xs, partials, scal);
}
void launch_cg_p(int n, const double* r, const double* Dinvp, const double* vdiag, double* p, double* Hp,
                 const double* partials, CgScal* scal, hipStream_t s) {
  const int nb = red_blocks(n);
  k_cg_p<<<nb, kBlock, 0, s>>>(n, nb, r, Dinvp, vdiag, p, Hp, partials, scal);
}

__global__ void __launch_bounds__(kBlock) k_mul(int n, const double* __restrict__ a, const double* __restrict__ b,
                                                double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = a[i] * b[i];
}

// out = -Dinv g: the preconditioned steepest-descent direction
__global__ void __launch_bounds__(kBlock) k_neg_precond(int n, const double* __restrict__ Dinvp,
                                                        const double* __restrict__ g, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = -Dinvp[i] * g[i];
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_set_pinned(DevMesh m, int v0, int v1, double value, double* vec) {
  for (int i = v0 * D + blockIdx.x * blockDim.x + threadIdx.x; i < v1 * D; i += gridDim.x * blockDim.x)
    if (m.pinned[i]) vec[i] = value;
}

// per block (min of a, count of non-finite entries)
__global__ void __launch_bounds__(kBlock) k_min_count(int n, const double* __restrict__ a, double* partials) {
  __shared__ double sh[kBlock / 64];
  double lo = 1e300, bad = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double v = a[i];
    if (isfinite(v))
      lo = fmin(lo, v);
    else
      bad += 1.0;
  }
  lo = block_min(lo, sh);
  bad = block_sum(bad, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = lo;
    partials[2 * blockIdx.x + 1] = -bad;
  }
}

__global__ void __launch_bounds__(kBlock) k_fill(int n, double value, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = value;
}
void launch_fill(int n, double value, double* out, hipStream_t s) {
  if (n <= 0) return;
  k_fill<<<grid_for(n), kBlock, 0, s>>>(n, value, out);
}
void launch_mul(int n, const double* a, const double* b, double* out, hipStream_t s) {
  if (n <= 0) return;
  k_mul<<<grid_for(n), kBlock, 0, s>>>(n, a, b, out);
}
void launch_neg_precond(int n, const double* Dinvp, const double* g, double* out, hipStream_t s) {
  if (n <= 0) return;
  k_neg_precond<<<grid_for(n), kBlock, 0, s>>>(n, Dinvp, g, out);
}
void launch_set_pinned(const DevMesh& m, int v0, int v1, double value, double* vec, hipStream_t s) {
  if (v1 <= v0) return;
  DISPATCH_D(m.dim, k_set_pinned, grid_for((v1 - v0) * m.dim), m, v0, v1, value, vec);
}
// out[0] = min a, out[1] = -(number of non-finite entries)
void launch_min_count(int n, const double* a, double* partials, double* out, hipStream_t s) {
  const int nb = red_blocks(n);
  k_min_count<<<nb, kBlock, 0, s>>>(n, a, partials);
  k_finalize_minmax<<<1, kBlock, 0, s>>>(partials, nb, out);
}

// ---------------------------------------------------------------------------------------------
// single-reduction PCG (Chronopoulos and Gear's s = 1 form) for the LDS-staged patch scatter
// ---------------------------------------------------------------------------------------------
// Vectors: r (residual), u = M r (M = D^-1), w = H u, p, s = H p, xs. Per iteration the patch
// Hessian-vector kernel adds the element part of H u into w (which holds the vertex part vdiag u)
// and leaves per-workgroup partials of u^T H_elem u; then k_cgcg_vec forms every scalar from one set
// of partials: gamma = r.u, delta = u.H u, and r.r for the stop test, and updates
//   beta = gamma / gamma_prev, p^T H p = delta - beta gamma / alpha_prev, alpha = gamma / p^T H p,
//   p = u + beta p, s = w + beta s, xs += alpha p, r -= alpha s, u = M r, w = vdiag u,
// writing the partials of the new (gamma, r.r, u^T vdiag u). Two launches per iteration instead of
// four; the partials alternate between two banks of 3 x kMaxRedBlocks values by iteration parity.

// The three interleaved partials (r.u, r.r, u.vdiag u) of nb blocks and nhv curvature partials,
// summed in one pass (all loads in flight together) and one block reduction; every block of the
// launch gets the same (gamma, r.r, delta). sh: 4 * (kBlock / 64) + 4 values.
__device__ __forceinline__ void cgcg_scalars(const double* partials, int nb, const double* hvpart, int nhv,
                                             double* sh, double& gamma, double& rr, double& delta) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    v[0] += partials[3 * b];
    v[1] += partials[3 * b + 1];
    v[2] += partials[3 * b + 2];
  }
  for (int b = threadIdx.x; b < nhv; b += blockDim.x) v[3] += hvpart[b];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = wave_sum(v[k]);
    if (lane == 0) sh[4 * wid + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[4 * w + threadIdx.x];
    sh[4 * (kBlock / 64) + threadIdx.x] = t;
  }
  __syncthreads();
  gamma = sh[4 * (kBlock / 64)];
  rr = sh[4 * (kBlock / 64) + 1];
  delta = sh[4 * (kBlock / 64) + 2] + sh[4 * (kBlock / 64) + 3];
  __syncthreads();  // sh is reused by the block sums below
}

// this block's sums of three values into out[3 * blockIdx.x + k] (one barrier); sh: 3 * (kBlock / 64)
__device__ __forceinline__ void block_partials3(double a, double b, double c, double* sh, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (lane == 0) {
    sh[3 * wid] = a;
    sh[3 * wid + 1] = b;
    sh[3 * wid + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[3 * w + threadIdx.x];
    out[3 * blockIdx.x + threadIdx.x] = t;
  }
}

// r = b (masked), u = M r, w = vdiag u, p = s = xs = 0; bank-0 partials (r.u, r.r, u.vdiag u)
__global__ void __launch_bounds__(kBlock) k_cgcg_start(int n, const double* __restrict__ b, double sign,
                                                       const double* __restrict__ Dinvp,
                                                       const double* __restrict__ vdiag, double* r, double* u,
                                                       double* w, double* p, double* sv, double* xs,
                                                       double* partials) {
  __shared__ double sh[3 * (kBlock / 64)];
  double g = 0.0, rr = 0.0, dv = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double ri = Dinvp[i] != 0.0 ? sign * b[i] : 0.0;
    const double ui = Dinvp[i] * ri;
    const double wi = vdiag[i] * ui;
    r[i] = ri;
    u[i] = ui;
    w[i] = wi;
    p[i] = 0.0;
    sv[i] = 0.0;
    xs[i] = 0.0;
    g += ri * ui;
    rr += ri * ri;
    dv += ui * wi;
  }
  block_partials3(g, rr, dv, sh, partials);
}

__global__ void __launch_bounds__(kBlock) k_cgcg_start_fin(const double* __restrict__ partials, int nb,
                                                           CgScal* scal, double tol2, int max_it) {
  __shared__ double sh[kBlock / 64 + 1];
  const double rr = all_blocks_sum(partials, nb, 3, 1, sh);
  if (threadIdx.x == 0) {
    scal->rr = rr;
    scal->rr0 = rr;
    scal->pHp = 0.0;
    scal->tol2 = tol2;
    scal->max_it = max_it;
    scal->done = (rr <= tol2 || max_it <= 0) ? 1 : 0;
    scal->negcurv = 0;
    scal->iters = 0;
    scal->it_cur = 0;
    scal->alpha_prev = 0.0;
    scal->gamma_prev = 0.0;
  }
}

// iteration it: the partials of r_it, u_it (bank it & 1) and the Hessian-vector kernel's nhv partials
// of u_it^T H_elem u_it give alpha_it and beta_it; then the update to iterate it + 1
__global__ void __launch_bounds__(kBlock) k_cgcg_vec(int n, int nb, const double* __restrict__ hvpart, int nhv,
                                                     double* partials, const double* __restrict__ Dinvp,
                                                     const double* __restrict__ vdiag, double* r, double* u,
                                                     double* w, double* p, double* sv, double* xs, CgScal* scal) {
  if (scal->done) return;
  const int it = scal->iters;
  const double* prev = partials + (it & 1) * 3 * kMaxRedBlocks;
  double* next = partials + ((it + 1) & 1) * 3 * kMaxRedBlocks;
  __shared__ double sh[4 * (kBlock / 64) + 4];
  double gamma, rr, delta;
  cgcg_scalars(prev, nb, hvpart, nhv, sh, gamma, rr, delta);
  if (rr <= scal->tol2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scal->done = 1;
      scal->rr = rr;
    }
    return;
  }
  const double beta = it == 0 ? 0.0 : gamma / scal->gamma_prev;
  const double pHp = it == 0 ? delta : delta - beta * gamma / scal->alpha_prev;
  if (!(pHp > 0.0)) {
    // non-positive curvature: stop; on the first iteration return the preconditioned
    // steepest-descent direction p0 = u0 = D^-1 b (Nocedal & Wright, Alg. 7.1)
    if (it == 0)
      for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) xs[i] = u[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scal->negcurv = 1;
      scal->done = 1;
      scal->pHp = pHp;
      scal->rr = rr;
    }
    return;
  }
  const double alpha = gamma / pHp;
  double g = 0.0, rn = 0.0, dv = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double di = Dinvp[i], vi = vdiag[i];
    const double pi = u[i] + beta * p[i];
    const double si = w[i] + beta * sv[i];
    xs[i] += alpha * pi;
    const double ri = di != 0.0 ? r[i] - alpha * si : 0.0;
    const double ui = di * ri;
    const double wi = vi * ui;
    p[i] = pi;
    sv[i] = si;
    r[i] = ri;
    u[i] = ui;
    w[i] = wi;
    g += ri * ui;
    rn += ri * ri;
    dv += ui * wi;
  }
  block_partials3(g, rn, dv, sh, next);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal->gamma_prev = gamma;
    scal->alpha_prev = alpha;
    scal->pHp = pHp;
    scal->rr = rr;
    scal->iters = it + 1;
    if (it + 1 >= scal->max_it) scal->done = 1;  // the cap: k_cgcg_final reports the last r.r
  }
}

// r.r of the final iterate (the partials of bank iters & 1, written by the last update or the start)
__global__ void __launch_bounds__(kBlock) k_cgcg_final(const double* __restrict__ partials, int nb, CgScal* scal) {
  __shared__ double sh[kBlock / 64 + 1];
  const int it = scal->iters;
  const double rr = all_blocks_sum(partials + (it & 1) * 3 * kMaxRedBlocks, nb, 3, 1, sh);
  if (threadIdx.x == 0) scal->rr = rr;
}

void launch_cgcg_start(int n, const double* b, double sign, const double* Dinvp, const double* vdiag, double* r,
                       double* u, double* w, double* p, double* sv, double* xs, double* partials, CgScal* scal,
                       double tol2, int max_it, hipStream_t s) {
  const int nb = red_blocks(n);
  k_cgcg_start<<<nb, kBlock, 0, s>>>(n, b, sign, Dinvp, vdiag, r, u, w, p, sv, xs, partials);
  k_cgcg_start_fin<<<1, kBlock, 0, s>>>(partials, nb, scal, tol2, max_it);
}
void launch_cgcg_vec(int n, const double* hvpart, int nhv, double* partials, const double* Dinvp,
                     const double* vdiag, double* r, double* u, double* w, double* p, double* sv, double* xs,
                     CgScal* scal, hipStream_t s) {
  const int nb = red_blocks(n);
  k_cgcg_vec<<<nb, kBlock, 0, s>>>(n, nb, hvpart, nhv, partials, Dinvp, vdiag, r, u, w, p, sv, xs, scal);
}
void launch_cgcg_final(int n, const double* partials, CgScal* scal, hipStream_t s) {
  k_cgcg_final<<<1, kBlock, 0, s>>>(partials, red_blocks(n), scal);
}

// ---------------------------------------------------------------------------------------------
// LDS-staged scatter over element patches
// ---------------------------------------------------------------------------------------------
// One workgroup per patch (grid-stride over patches): stage x (and p) of the patch's distinct
// vertices in LDS, evaluate the elements with LDS gathers and accumulate with LDS atomics, then
// add each distinct vertex DOF to the global output once. Global atomics drop from d(d+1) per
// element to the patch's distinct DOFs, and they no longer collide inside a wavefront.
// CR: compact rest record (uniform material, fibre along an axis; see DevMesh)
template <int D, typename T, int OP, int PB, int EM, bool CR>
__global__ void __launch_bounds__(PB) k_elem_patch(DevMesh m, DevScene sc, PatchPlan P, int p0, int p1,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ a,
                                                            const float* __restrict__ a32,
                                                            const double* __restrict__ pv, double* out,
                                                            const int* done, double* curv) {
  // LDS: x, the accumulator and the Hessian-vector operand p per patch DOF, all FP64 (the element
  // takes differences of x and of p, which must be formed before any rounding to T), then the
  // global id of each patch vertex, so that the flush needs no second load of the vertex list
  extern __shared__ double lds[];
  if (OP == PATCH_HV && done && *done) return;
  // curv (Hessian-vector products only): this workgroup's share of p^T H_elem p, the sum over its
  // elements of p_e . (H_e p_e), for a CG that needs no separate dot-product pass
  double php = 0.0;
  const int nmax = P.max_nv * D;
  double* xs = lds;
  double* acc = lds + nmax;
  double* ps = lds + 2 * nmax;
  int* vid = reinterpret_cast<int*>(lds + (OP == PATCH_HV ? 3 : 2) * nmax);
  for (int pk = p0 + blockIdx.x; pk < p1; pk += gridDim.x) {
    const int vb = P.voff[pk], nv = P.voff[pk + 1] - vb;
    const int eb = P.eoff[pk], ee = P.eoff[pk + 1];
    // one vertex per thread: its id, then its D components of x (and p) in one round trip
    for (int vl = threadIdx.x; vl < nv; vl += blockDim.x) {
      const int gv = P.verts[vb + vl];
      vid[vl] = gv;
      const size_t g = (size_t)gv * D;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        xs[vl * D + c] = x[g + c];
        if (OP == PATCH_HV) ps[vl * D + c] = pv[g + c];
        acc[vl * D + c] = 0.0;
      }
    }
    __syncthreads();
    patch_elements<D, T, OP, EM, CR>(m, sc, P.lconn, P.eperm, eb, ee, xs, ps, acc, a, a32, curv != nullptr, php);
    __syncthreads();
    for (int i = threadIdx.x; i < nv * D; i += blockDim.x) {
      const int vl = i / D, c = i - vl * D;
      unsafeAtomicAdd(out + (size_t)vid[vl] * D + c, acc[i]);
    }
    __syncthreads();
  }
  if (OP == PATCH_HV && curv) {
    double* red = lds;  // free after the last flush (the launch sizes LDS to hold PB / 64 values)
    php = wave_sum(php);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = php;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < PB / 64; ++w) t += red[w];
      curv[blockIdx.x] = sc.s_pot * t;
    }
  }
}

template <int D, typename T, int OP>
static int patch_launch(const DevMesh& m, const DevScene& sc, const PatchPlan& P, int p0, int p1, const double* x,
                        const double* a, const float* a32, const double* p, double* out, const int* done,
                        double* curv, hipStream_t s) {
  const size_t lds = std::max<size_t>((size_t)P.max_nv * (D * sizeof(double) * (OP == PATCH_HV ? 3 : 2) + sizeof(int)),
                                      (1024 / 64) * sizeof(double));
  int grid = p1 - p0;
  if (grid > kMaxPatchGrid) grid = kMaxPatchGrid;
  // workgroup size: P.block when it names a compiled size (the neo-Hookean kernels come in 256, 512
  // and 1024 threads, the alternative models in the default only), else the default: 512 threads
  // for FP32 element math, 256 for FP64. The kernels are bound by LDS traffic (gathers and FP64
  // atomics) at about three patches per CU: larger workgroups only add contention.
  constexpr int kDefault = std::is_same<T, float>::value ? kPatchBlock : kPatchBlock / 2;
  const int pb = (m.model == EM_NH && (P.block == 256 || P.block == 512 || P.block == 1024)) ? P.block : kDefault;
  auto go = [&](auto pbc, auto em) {
    constexpr int PB = decltype(pbc)::value;
    constexpr int EM = decltype(em)::value;
    if (m.axis >= 0)
      k_elem_patch<D, T, OP, PB, EM, true><<<grid, PB, lds, s>>>(m, sc, P, p0, p1, x, a, a32, p, out, done, curv);
    else
      k_elem_patch<D, T, OP, PB, EM, false><<<grid, PB, lds, s>>>(m, sc, P, p0, p1, x, a, a32, p, out, done, curv);
  };
  if (m.model != EM_NH) {
    with_model(m.model, [&](auto em) { go(std::integral_constant<int, kDefault>{}, em); });
  } else if (pb == 256) {
    go(std::integral_constant<int, 256>{}, std::integral_constant<int, EM_NH>{});
  } else if (pb == 1024) {
    go(std::integral_constant<int, 1024>{}, std::integral_constant<int, EM_NH>{});
  } else {
    go(std::integral_constant<int, 512>{}, std::integral_constant<int, EM_NH>{});
  }
  return grid;
}

int launch_elem_patch(const DevMesh& m, const DevScene& sc, const PatchPlan& P, int p0, int p1, int op,
                      int precision, const double* x, const double* a, const float* a32, const double* p,
                      double* out, const int* done, hipStream_t s, double* curv) {
  if (p1 <= p0) return 0;
  if (op != PATCH_HV) curv = nullptr;
#define ISB_PATCH_CASE(D_)                                                                          \
  if (op == PATCH_GRAD)                                                                             \
    return patch_launch<D_, double, PATCH_GRAD>(m, sc, P, p0, p1, x, a, a32, p, out, done, curv, s);  \
  else if (op == PATCH_HV && precision)                                                             \
    return patch_launch<D_, float, PATCH_HV>(m, sc, P, p0, p1, x, a, a32, p, out, done, curv, s);     \
  else if (op == PATCH_HV)                                                                          \
    return patch_launch<D_, double, PATCH_HV>(m, sc, P, p0, p1, x, a, a32, p, out, done, curv, s);    \
  else                                                                                              \
    return patch_launch<D_, double, PATCH_DIAG>(m, sc, P, p0, p1, x, a, a32, p, out, done, curv, s);
  if (m.dim == 2) {
    ISB_PATCH_CASE(2)
  } else {
    ISB_PATCH_CASE(3)
  }
#undef ISB_PATCH_CASE
}

}  // namespace isb
