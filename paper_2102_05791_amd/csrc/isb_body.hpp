// Body-level logic of the batched persistent solver, shared by the gfx950 kernel and by a
// CPU build used in tests (a workgroup emulated with host threads).
//
// One workgroup solves one body at a time, from a list the host deals out ahead of the launch
// (longest processing time first over a per-body cost model). Inside a body: Newton's method on the step
// objective (Eq. 1 / Eq. 14) with a Jacobi-preconditioned CG inner solve, an Armijo line search
// on element-wise energy differences, and v1 = (x1 - x0)/h; or, for the adjoint, one CG solve
// of Eq. 9 at x1. The element scatter (gradient, Hessian diagonal, Hessian-vector product,
// Eq. 10) accumulates into the body's vertex array in LDS with FP64 LDS atomics; each thread
// owns the DOFs i = tid + k * blockDim of the body in every vector operation, so vector passes
// need no synchronisation beyond the workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>

#include "../../include/isb.h"
#include "isb_device.hpp"
#include "isb_elem.hpp"
#include "isb_internal.hpp"
#include "isb_spring.hpp"

namespace isb {

// Same layout as isb_stats.
struct DevStats {
  int32_t newton_iters, cg_iters, adj_cg_iters, ls_backtracks, negcurv_exits, flags;
  double res0, res_final, adj_res_final, energy, min_J, max_J;
};
static_assert(sizeof(DevStats) == sizeof(isb_stats), "stats layout");

struct BatchArgs {
  const int32_t* order;   // bodies of workgroup g: order[wg_off[g] .. wg_off[g+1])
  const int32_t* wg_off;  // [grid+1]
  const int32_t* voff;   // [n_bodies+1]
  const int32_t* eoff;   // [n_bodies+1]
  int n_bodies;
  const double *x0, *v0, *a;
  const float* a32;
  double *x1, *v1;               // step outputs (x1 is also the Newton iterate)
  const double *xbar, *vbar;     // adjoint right-hand side
  double* w;                     // adjoint output
  double *xhat, *G, *Gt, *dx, *r, *cv;  // workspaces
  double* xt;         // [n_v*D] trial point of the line search; swaps with the iterate on acceptance
  float* Dv;          // [n_v*D] Jacobi preconditioner 1/|diag H| (FP32: it only steers convergence)
  void* vdT;          // [n_v*D] vertex-term Hessian diagonal in the element precision
  const uint16_t* lconn;  // [D+1][n_e] body-local vertex ids (a body that fits in LDS has < 65536 vertices)
  DevStats* stats;
  double tol, adj_tol;
  int max_newton, max_cg;
  int want_tail;  // 1: final energy and min/max J into the stats
  int nacc;       // LDS accumulator length: the largest body's DOF count
  void* Fbuf;     // [hv_state_words(D)][n_e] per-element Hessian-vector state at the current Newton
                  // iterate, in the element precision (see BodySolver::store_hv_state)
  double *E0, *E1;  // [n_e + n_s] per-element, then per-spring, energies at the iterate and at the
                    // line-search trial
  // vertex-pair springs (Eq. 2 between two vertices); n_s = 0 without springs
  const int32_t* soff;     // [n_bodies+1] springs of each body
  const uint16_t* slconn;  // [2][n_s] body-local end vertices i, j
  const double *sk, *sil0; // [n_s] stiffness, 1 / rest length
  void* Sbuf;              // [spring_state_words(D)][n_s] spring block K at the iterate, element precision
  int n_s;
  int adj_warm;            // 1: the adjoint starts its CG from the w it is given (ISB_OPT_ADJ_WARM_START)
};

// Reduction slots: two banks of up to 16 waves x 4 values. Consecutive workgroup reductions use
// alternate banks, so one barrier per reduction suffices: a wave writing a bank two reductions
// later has passed the barrier of the reduction in between, which every reader of the bank's
// previous contents reached only after reading them.
constexpr int kRedBank = 16 * 4;
constexpr int kRedSlots = 2 * kRedBank;

// Words of per-element state the Hessian-vector pass reads: triangles keep the symmetric 4x4
// Hessian of W psi with respect to the edge matrix (10 words); tetrahedra keep F and F d (12),
// from which the product is formed matrix-free.
__host__ __device__ constexpr int hv_state_words(int dim) { return dim == 2 ? 10 : dim * dim + dim; }

// Values that steer control flow around barriers (the schedule's entries, reduction results)
// are loaded into vector registers, so the compiler cannot prove them uniform and may structurize
// the loops around them as divergent, letting some lanes loop back past a barrier the others have
// not reached. Broadcasting them from the first active lane makes the branches scalar.
__device__ __forceinline__ int wg_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double wg_uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// A DPP cross-lane move of an FP64 value (both 32-bit halves take the same move); lanes in rows
// outside ROWS receive 0.0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes of a wave (all lanes active), returned to every lane. Within each row of
// 16 lanes: quad_perm [1,0,3,2] and [2,3,0,1] sum the quads, row_ror 4 and 8 the row; then
// row_bcast 15 adds row 0 into row 1 and row 2 into row 3, row_bcast 31 rows 0-1 into rows 2-3,
// and lane 63 holds the total in a fixed order.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x124>(v);
  v += dpp_move<0x128>(v);
  v += dpp_move<0x142, 0xA>(v);
  v += dpp_move<0x143, 0xC>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// sum of N values over the workgroup into one bank of reduction slots; every thread receives the
// same bits
template <int N>
__device__ __forceinline__ void wg_sum(double (&v)[N], double* bank) {
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_total(v[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) bank[wid * N + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += bank[w * N + k];
    v[k] = wg_uniform(s);
  }
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
  return v;
}

// (min, max) over the workgroup into one bank of reduction slots, every thread receives the result
__device__ __forceinline__ void wg_minmax(double& lo, double& hi, double* bank) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  lo = wave_min(lo);
  hi = -wave_min(-hi);
  if (lane == 0) {
    bank[2 * wid] = lo;
    bank[2 * wid + 1] = hi;
  }
  __syncthreads();
  lo = 1e300;
  hi = -1e300;
  for (int w = 0; w < nw; ++w) {
    lo = fmin(lo, bank[2 * w]);
    hi = fmax(hi, bank[2 * w + 1]);
  }
  lo = wg_uniform(lo);
  hi = wg_uniform(hi);
}

// CR: the compact rest record (uniform material, fibre along an axis; see DevMesh::axis)
template <int D, typename T, int EM = EM_NH, bool CR = false>
struct BodySolver {
  const DevMesh& m;
  const DevScene& sc;
  const BatchArgs& A;
  double* acc;  // LDS, one value per body DOF (layout lv below), zero between passes
  double* red;  // LDS reduction slots, two banks (see kRedSlots)
  double* ps;   // LDS, same layout: the CG direction p inside cg() (FP64: the Hv pass takes
                // differences of it), the diagonal accumulator of trial(); zero outside both
  int v0, v1, e0, e1, n, base;

  int rbank = 0;       // bank of the last workgroup reduction
  int s0 = 0, s1 = 0;  // the body's springs

  __device__ __forceinline__ T* Fb() const { return reinterpret_cast<T*>(A.Fbuf); }

  // workgroup reductions, alternating between the two banks of slots
  template <int N>
  __device__ __forceinline__ void sum(double (&v)[N]) {
    rbank ^= 1;
    wg_sum<N>(v, red + rbank * kRedBank);
  }
  __device__ __forceinline__ double sum1(double v) {
    double t[1] = {v};
    sum<1>(t);
    return t[0];
  }

  // LDS arrays hold one component plane after the other (vertex vl, axis c at c * nvs + vl), so
  // that the FP64 atomics of a wave, which touch runs of nearby vertices, spread over the banks;
  // the interleaved layout of the global vectors would put vertices 8 apart on one bank.
  __device__ __forceinline__ int lv(int vl, int c) const { return c * (A.nacc / D) + ISB_CHECKED(vl, v1 - v0, 1); }
  __device__ __forceinline__ int ld(int i) const { return lv(i / D, i % D); }  // body DOF i = vl * D + c

  __device__ __forceinline__ bool pinned(int i) const { return m.pinned[base + i] != 0; }
  __device__ __forceinline__ T* vdp() const { return reinterpret_cast<T*>(A.vdT); }

  // the element's vertices (global ids) from the 16-bit body-local connectivity
  __device__ __forceinline__ void load_lconn(int e, int v[D + 1]) const {
    const size_t ne = (size_t)m.n_e;
#pragma unroll
    for (int k = 0; k <= D; ++k) v[k] = v0 + ISB_CHECKED((int)A.lconn[(size_t)k * ne + e], v1 - v0, 2);
  }

  // preconditioner entry of a free DOF with Hessian diagonal d (1 where d is 0), as stored
  __device__ __forceinline__ static float precond_entry(double d) {
    return d > 0.0 ? (float)fmin(1.0 / d, 3.0e38) : 1.0f;
  }

  // -------- element passes: scatter into acc (local DOF index = (v - v0) * D + c) --------
  __device__ __forceinline__ void lds_scatter(const int v[D + 1], const double out[D + 1][D], double scale) {
#pragma unroll
    for (int k = 0; k <= D; ++k)
#pragma unroll
      for (int c = 0; c < D; ++c) unsafeAtomicAdd(acc + lv(v[k] - v0, c), scale * out[k][c]);
  }

  __device__ __forceinline__ T act(int e) const {
    if constexpr (std::is_same<T, double>::value)
      return A.a[e];
    else
      return A.a32[e];
  }

  // -------- springs: FP64 terms (isb_spring.hpp); the block K is rounded once to T --------
  static constexpr int kSW = spring_state_words(D);
  __device__ __forceinline__ T* Sb() const { return reinterpret_cast<T*>(A.Sbuf); }
  __device__ __forceinline__ void spring_ends(int s, int& i, int& j) const {
    i = ISB_CHECKED((int)A.slconn[s], v1 - v0, 3);
    j = ISB_CHECKED((int)A.slconn[(size_t)A.n_s + s], v1 - v0, 3);
  }
  // +y at vertex j and -y at vertex i (both_plus: +y at both) into the LDS array dst
  __device__ __forceinline__ void spring_lds(double* dst, int i, int j, const double y[D], bool both_plus) const {
#pragma unroll
    for (int r = 0; r < D; ++r) {
      unsafeAtomicAdd(dst + lv(j, r), sc.s_pot * y[r]);
      unsafeAtomicAdd(dst + lv(i, r), both_plus ? sc.s_pot * y[r] : -sc.s_pot * y[r]);
    }
  }
  // stores the block K of a spring and returns its diagonal (each end receives it)
  __device__ __forceinline__ void store_spring_state(int s, const SpringTerms<D>& S, double dg[D]) const {
    double K[kSW];
    spring_block<D>(S, K);
#pragma unroll
    for (int w = 0; w < kSW; ++w) Sb()[(size_t)w * A.n_s + s] = T(K[w]);
    spring_diag<D>(S, dg);
  }

  // Hessian-vector pass: the per-element state streams in coalesced, p comes from LDS. Edge
  // differences of p are formed in FP64 before any rounding to T. Returns this thread's share of
  // p^T H_elem p = sum over elements of dDs(p) . (K_s dDs(p)), so the CG curvature needs no
  // separate pass over the scattered product.
  static constexpr bool kEdgeHessian = (D == 2);
  static constexpr int kQ = D * D;  // entries of the edge matrix, q = j * D + r for Ds[r][j]

  __device__ double pass_hv() {
    const size_t ne = (size_t)m.n_e;
    double php = 0.0;
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      int v[D + 1];
      load_lconn(e, v);
      T out[D + 1][D];
      double d64[kQ];  // edge differences of p, q = j * D + r
      if constexpr (kEdgeHessian) {
        T K[hv_state_words(D)];
#pragma unroll
        for (int w = 0; w < hv_state_words(D); ++w) K[w] = Fb()[(size_t)w * ne + e];
        edge_diffs(v, d64);
        T dd[kQ], y[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) dd[q] = T(d64[q]);
        sym_apply(K, dd, y);
#pragma unroll
        for (int r = 0; r < D; ++r) out[0][r] = T(0);
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
          for (int r = 0; r < D; ++r) {
            out[j + 1][r] = y[j * D + r];
            out[0][r] -= y[j * D + r];
          }
      } else {
        ElemRest<D, T> R;
        load_rest<D, T, CR>(m, e, R);
        T F[D][D], Fd[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
#pragma unroll
          for (int c = 0; c < D; ++c) F[r][c] = Fb()[(size_t)(r * D + c) * ne + e];
          Fd[r] = Fb()[(size_t)(D * D + r) * ne + e];
        }
        const T ae = act(e);
        edge_diffs(v, d64);
        T dDs[D][D];
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
          for (int r = 0; r < D; ++r) dDs[r][j] = T(d64[j * D + r]);
        ElemState<D, T> S;
        elem_state_from_F<D, T>(F, Fd, S);
        elem_hessvec<D, T, EM>(R, S, ae, dDs, out);
      }
      // sum_k out_k . p_k = sum_j out_{j+1} . (p_{j+1} - p_0), since out_0 = -sum_j out_{j+1}
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int r = 0; r < D; ++r) php += double(out[j + 1][r]) * d64[j * D + r];
      double o[D + 1][D];
#pragma unroll
      for (int k = 0; k <= D; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) o[k][c] = double(out[k][c]);
      lds_scatter(v, o, sc.s_pot);
    }
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
      int i, j;
      spring_ends(s, i, j);
      T K[kSW];
#pragma unroll
      for (int w = 0; w < kSW; ++w) K[w] = Sb()[(size_t)w * A.n_s + s];
      double u64[D], y64[D];
      T u[D], y[D];
#pragma unroll
      for (int r = 0; r < D; ++r) {
        u64[r] = ps[lv(j, r)] - ps[lv(i, r)];
        u[r] = T(u64[r]);
      }
      spring_block_apply<D, T>(K, u, y);
#pragma unroll
      for (int r = 0; r < D; ++r) {
        y64[r] = double(y[r]);
        php += y64[r] * u64[r];
      }
      spring_lds(acc, i, j, y64, false);
    }
    return sc.s_pot * php;
  }

  // FP64 edge differences of the LDS direction p over one element, q = j * D + r
  __device__ __forceinline__ void edge_diffs(const int v[D + 1], double d64[kQ]) const {
    double p0[D];
#pragma unroll
    for (int r = 0; r < D; ++r) p0[r] = ps[lv(v[0] - v0, r)];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int r = 0; r < D; ++r) d64[j * D + r] = ps[lv(v[j + 1] - v0, r)] - p0[r];
  }

  // y = K x for the symmetric kQ x kQ matrix whose upper triangle K holds row by row
  __device__ __forceinline__ static void sym_apply(const T* K, const T* x, T* y) {
#pragma unroll
    for (int a = 0; a < kQ; ++a) y[a] = T(0);
    int w = 0;
#pragma unroll
    for (int a = 0; a < kQ; ++a)
#pragma unroll
      for (int b = a; b < kQ; ++b, ++w) {
        y[a] += K[w] * x[b];
        if (b != a) y[b] += K[w] * x[a];
      }
  }

  // Stores what the Hessian-vector passes need at this iterate and returns the element's Hessian
  // diagonal per vertex and axis (FP64, before the s_pot scale). Triangles: the Hessian of W psi
  // with respect to the edge matrix, K_s[q][q'] = d^2 (W psi) / dDs_q dDs_q', in closed form
  // (edge_hessian_2d) and rounded once to T; a unit move of vertex j+1 along r is the unit edge
  // displacement q = j D + r, one of vertex 0 moves every edge by -e_r. Tetrahedra: F and F d,
  // rounded once to T, and the closed-form diagonal.
  __device__ __forceinline__ void store_hv_state(int e, const ElemRest<D, double>& R64,
                                                 const ElemState<D, double>& S64, double ae,
                                                 double diag[D + 1][D]) const {
    const size_t ne = (size_t)m.n_e;
    if constexpr (kEdgeHessian) {
      double K[kQ][kQ];
      edge_hessian_2d<double, EM>(R64, S64, ae, K);
      int w = 0;
#pragma unroll
      for (int a = 0; a < kQ; ++a)
#pragma unroll
        for (int b = a; b < kQ; ++b, ++w) Fb()[(size_t)w * ne + e] = T(K[a][b]);
#pragma unroll
      for (int r = 0; r < D; ++r) {
        double d0 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          diag[j + 1][r] = K[j * D + r][j * D + r];
#pragma unroll
          for (int jj = 0; jj < D; ++jj) d0 += K[j * D + r][jj * D + r];
        }
        diag[0][r] = d0;
      }
    } else {
#pragma unroll
      for (int r = 0; r < D; ++r) {
        Fb()[(size_t)(D * D + r) * ne + e] = T(S64.n[r] * S64.s);
#pragma unroll
        for (int c = 0; c < D; ++c) Fb()[(size_t)(r * D + c) * ne + e] = T(S64.F[r][c]);
      }
      elem_hessdiag<D, double, EM>(R64, S64, ae, diag);
    }
  }

  // diagonal pass (FP64); also stores the Hessian-vector state of every element
  __device__ void pass_diag(const double* x) {
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      int v[D + 1];
      load_lconn(e, v);
      ElemRest<D, double> R64;
      load_rest<D, double, CR>(m, e, R64);
      const double ae = A.a[e];
      double Ds[D][D];
      gather_edges<D, double>(x, v, Ds);
      ElemState<D, double> S64;
      elem_state<D, double>(Ds, R64, S64);
      double od[D + 1][D];
      store_hv_state(e, R64, S64, ae, od);
      lds_scatter(v, od, sc.s_pot);
    }
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
      int i, j;
      spring_ends(s, i, j);
      double d[D];
#pragma unroll
      for (int r = 0; r < D; ++r) d[r] = x[(size_t)(v0 + j) * D + r] - x[(size_t)(v0 + i) * D + r];
      SpringTerms<D> S;
      spring_terms<D>(d, A.sk[s], A.sil0[s], A.a[m.n_e + s], S);
      double dg[D];
      store_spring_state(s, S, dg);
      spring_lds(acc, i, j, dg, true);
    }
  }

  // -------- vertex terms per DOF, from values already in registers --------
  // gradient of the vertex part along axis c: gravity / contact on y, friction on the others
  // (Eq. 15-17), inertia in backward Euler
  __device__ __forceinline__ double vgrad(int c, double xi, double mv, double cvv, double x0i, double xhi) const {
    double g;
    if (c == 1)
      g = mv * sc.grav - 2.0 * sc.kc * fmax(-xi, 0.0);
    else
      g = 2.0 * sc.kfr * cvv * sc.ih2 * (xi - x0i);
    g *= sc.s_pot;
    if (sc.be) g += mv * (xi - xhi);
    return g;
  }

  __device__ __forceinline__ double vhdiag(int c, double xi, double mv, double cvv) const {
    double hd = (c == 1) ? (xi < 0.0 ? 2.0 * sc.kc : 0.0) : 2.0 * sc.kfr * cvv * sc.ih2;
    hd *= sc.s_pot;
    if (sc.be) hd += mv;
    return hd;
  }

  // Jacobi preconditioner 1/|diag H| and the vertex-term diagonal
  __device__ void precond(const double* x) {
    pass_diag(x);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int vg = v0 + i / D, c = i % D;
      const bool pin = pinned(i);
      const double vd = pin ? 0.0 : vhdiag(c, x[base + i], m.mass[vg], A.cv[vg]);
      const double d = fabs(acc[ld(i)] + vd);
      vdp()[base + i] = T(vd);
      A.Dv[base + i] = pin ? 0.0f : precond_entry(d);
      acc[ld(i)] = 0.0;
    }
    __syncthreads();
  }

  // One element pass at the trial point xt = x + alpha dx (x itself when dx is null). It returns
  // out = (sum of g_e(xt) - g_e(x) over elements and vertices, sum |g_e(x)|, g(xt), |grad g(xt)|^2)
  // -- the element differences use the stored energies Ecur of x, the new ones go to Enew -- and
  // leaves behind the gradient at xt in Gout, the Jacobi preconditioner and vertex-term diagonal,
  // the Hessian-vector state per element, and xt itself in xt_out (when given): everything the next
  // Newton iteration needs if the trial is accepted.
  // Each loop issues every global load of an iteration before its first global store: stores
  // count against the same wait counter as loads, and a load placed after a store waits for it.
  static constexpr int kV = 3;  // vertices per thread per chunk of the vertex loop

  __device__ void trial(const double* x, const double* dxp, double alpha, double* Gout, const double* Ecur,
                        double* Enew, double out[4], double* xt_out = nullptr) {
    double* acc2 = ps;  // the CG direction's LDS is free outside CG: it takes the diagonal
    const size_t ne = (size_t)m.n_e;
    double sd = 0.0, sa = 0.0, st = 0.0;
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      int v[D + 1];
      load_lconn(e, v);
      ElemRest<D, double> R64;
      load_rest<D, double, CR>(m, e, R64);
      const double ae = A.a[e];
      const double estored = Ecur ? Ecur[e] : 0.0;
      double Ds[D][D];
      if (dxp)
        gather_edges_step<D>(x, dxp, alpha, v, Ds);
      else
        gather_edges<D, double>(x, v, Ds);
      ElemState<D, double> S64;
      elem_state<D, double>(Ds, R64, S64);
      const double eb = sc.s_pot * elem_energy<D, double, EM>(R64, S64, ae);
      const double ea = Ecur ? estored : eb;
      sd += eb - ea;
      sa += fabs(ea);
      st += eb;
      double o[D + 1][D];
      elem_grad<D, double, EM>(R64, S64, ae, o);
      lds_scatter(v, o, sc.s_pot);
      // global stores once every load of the iteration has been issued: the energy, and the
      // Hessian-vector state, whose computation also yields the Jacobi diagonal (FP64)
      Enew[e] = eb;
      store_hv_state(e, R64, S64, ae, o);
#pragma unroll
      for (int k = 0; k <= D; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) unsafeAtomicAdd(acc2 + lv(v[k] - v0, c), sc.s_pot * o[k][c]);
    }
    // springs: energy difference, gradient, block K and diagonal, as for the elements; the trial
    // point of each end is formed per DOF exactly as the vertex loop below forms it
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
      int i, j;
      spring_ends(s, i, j);
      const double ks = A.sk[s], il0 = A.sil0[s], as = A.a[m.n_e + s];
      const double estored = Ecur ? Ecur[m.n_e + s] : 0.0;
      double d[D];
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const size_t gi = (size_t)(v0 + i) * D + r, gj = (size_t)(v0 + j) * D + r;
        const double xi = dxp ? x[gi] + alpha * dxp[gi] : x[gi];
        const double xj = dxp ? x[gj] + alpha * dxp[gj] : x[gj];
        d[r] = xj - xi;
      }
      SpringTerms<D> S;
      spring_terms<D>(d, ks, il0, as, S);
      const double eb = sc.s_pot * spring_energy<D>(S, ks);
      const double ea = Ecur ? estored : eb;
      sd += eb - ea;
      sa += fabs(ea);
      st += eb;
      double y[D];
#pragma unroll
      for (int r = 0; r < D; ++r) y[r] = S.f * S.n[r];
      spring_lds(acc, i, j, y, false);
      Enew[m.n_e + s] = eb;
      store_spring_state(s, S, y);
      spring_lds(acc2, i, j, y, true);
    }
    __syncthreads();
    // vertex terms, kV vertices per thread at a time: energies at x and xt, then per DOF the
    // gradient, the vertex diagonal and the preconditioner
    double gg = 0.0;
    const int nv = v1 - v0, B = blockDim.x;
    for (int vl0 = threadIdx.x; vl0 < nv; vl0 += kV * B) {
      double xa[kV][D], dd[kV][D], x0v[kV][D], xhv[kV][D], mv[kV], cvv[kV];
      bool pin[kV][D];
      // loads for every lane (indices past the body clamped to its last vertex): loads inside a
      // divergent branch are each waited for before the branch ends
#pragma unroll
      for (int u = 0; u < kV; ++u) {
        const int vg = v0 + (vl0 + u * B < nv ? vl0 + u * B : nv - 1);
        mv[u] = m.mass[vg];
        cvv[u] = A.cv[vg];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const size_t g = (size_t)vg * D + c;
          xa[u][c] = x[g];
          dd[u][c] = dxp ? dxp[g] : 0.0;
          x0v[u][c] = A.x0[g];
          xhv[u][c] = sc.be ? A.xhat[g] : 0.0;
          pin[u][c] = m.pinned[g] != 0;
        }
      }
#pragma unroll
      for (int u = 0; u < kV; ++u) {
        const int vl = vl0 + u * B;
        if (vl < nv) {
          double xb[D];
#pragma unroll
          for (int c = 0; c < D; ++c) xb[c] = xa[u][c] + alpha * dd[u][c];
          const double ea = vertex_energy_vals<D>(sc, mv[u], cvv[u], xa[u], x0v[u], xhv[u]);
          const double eb = vertex_energy_vals<D>(sc, mv[u], cvv[u], xb, x0v[u], xhv[u]);
          sd += eb - ea;
          sa += fabs(ea);
          st += eb;
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const int i = lv(vl, c);
            const size_t g = (size_t)(v0 + vl) * D + c;
            const double gi = pin[u][c] ? 0.0 : acc[i] + vgrad(c, xb[c], mv[u], cvv[u], x0v[u][c], xhv[u][c]);
            gg += gi * gi;
            const double vd = pin[u][c] ? 0.0 : vhdiag(c, xb[c], mv[u], cvv[u]);
            const double d = fabs(acc2[i] + vd);
            Gout[g] = gi;
            if (xt_out) xt_out[g] = xb[c];
            vdp()[g] = T(vd);
            A.Dv[g] = pin[u][c] ? 0.0f : precond_entry(d);
            acc[i] = 0.0;
            acc2[i] = 0.0;
          }
        }
      }
    }
    double t[4] = {sd, sa, st, gg};
    sum<4>(t);
    out[0] = t[0];
    out[1] = t[1];
    out[2] = t[2];
    out[3] = t[3];
  }

  __device__ void minmax_J(const double* x, double& lo, double& hi) {
    lo = 1e300;
    hi = -1e300;
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      int v[D + 1];
      load_lconn(e, v);
      ElemRest<D, double> R;
      load_rest<D, double, CR>(m, e, R);
      double Ds[D][D];
      gather_edges<D, double>(x, v, Ds);
      ElemState<D, double> S;
      elem_state<D, double>(Ds, R, S);
      lo = fmin(lo, S.J);
      hi = fmax(hi, S.J);
    }
    rbank ^= 1;
    wg_minmax(lo, hi, red + rbank * kRedBank);
  }

  // PCG on H(x) xs = sign * rhs (masked to the free DOFs); returns the final r.r. The element
  // state (F, F d) must have been stored by precond(x) or trial(). The direction p lives only in
  // LDS. Per iteration: the Hv pass, which also sums the element part of p^T H p; one vector pass
  // that updates xs and r and leaves z = M r in the accumulator; one LDS-only pass that forms the
  // next p.
  static constexpr int kU = 2;

  // the kU owned DOFs from i0 on of xs, D^-1, r and vdiag. Indices past the body load the DOF
  // `own` instead, one this thread owns and has not yet written in the current pass, so that every
  // lane loads unconditionally without reading a DOF another thread is updating; the caller ignores
  // those values. own < 0: the thread owns no DOF of the body and loads nothing.
  __device__ __forceinline__ void cg_load(int i0, int own, const double* xs, double (&x)[kU], double (&d)[kU],
                                          double (&rv)[kU], double (&v)[kU]) const {
    if (own < 0) {
#pragma unroll
      for (int u = 0; u < kU; ++u) x[u] = d[u] = rv[u] = v[u] = 0.0;
      return;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int iu = i0 + u * (int)blockDim.x;
      const int i = iu < n ? iu : own;
      const int g = base + i;
      x[u] = xs[g];
      d[u] = A.Dv[g];
      rv[u] = A.r[g];
      v[u] = vdp()[g];
    }
  }

  __device__ double cg(const double* rhs, double sign, double tol, int maxit, double* xs, int& iters, bool& neg) {
    double* r = A.r;
    const float* Dv = A.Dv;
    const T* vd = vdp();
    const int B = blockDim.x;
    double rz = 0.0, rr = 0.0, pvp = 0.0;  // pvp: this thread's share of sum vd p^2
    for (int i0 = threadIdx.x; i0 < n; i0 += kC * B) {
      double dv[kC], bv[kC], vv[kC];
#pragma unroll
      for (int u = 0; u < kC; ++u) {
        const int g = base + (i0 + u * B < n ? i0 + u * B : n - 1);
        dv[u] = Dv[g];
        bv[u] = rhs[g];
        vv[u] = vd[g];
      }
#pragma unroll
      for (int u = 0; u < kC; ++u) {
        const int i = i0 + u * B;
        if (i < n) {
          const int g = base + i;
          const double ri = dv[u] != 0.0 ? sign * bv[u] : 0.0;
          const double zi = dv[u] * ri;
          r[g] = ri;
          ps[ld(i)] = zi;
          xs[g] = 0.0;
          rz += ri * zi;
          rr += ri * ri;
          pvp += vv[u] * zi * zi;
        }
      }
    }
    {
      double t[2] = {rz, rr};
      sum<2>(t);
      rz = t[0];
      rr = t[1];
    }
    iters = 0;
    neg = false;
    const double tol2 = tol * tol;
    for (int it = 0; it < maxit && rr > tol2; ++it) {
      // the reduction's barriers also complete the scatter into acc
      const double pHp = sum1(pass_hv() + pvp);
      if (!(pHp > 0.0)) {
        // non-positive curvature: stop; on the first iteration keep the preconditioned
        // steepest-descent direction (Nocedal & Wright, Alg. 7.1)
        neg = true;
        for (int i = threadIdx.x; i < n; i += B) {
          if (it == 0) xs[base + i] = ps[ld(i)];
          acc[ld(i)] = 0.0;
        }
        break;
      }
      const double alpha = rz / pHp;
      // x/r update, kU owned DOFs per thread at a time and software-pipelined: the loads of the
      // next chunk go out before the stores of this one. It also sums this thread's share of
      // vd z^2, vd z p and vd p^2, from which the vertex part of the next direction's curvature
      // follows once beta is known, so the direction pass below touches LDS only.
      double rz1 = 0.0, zz = 0.0, zp = 0.0, pp = 0.0;
      rr = 0.0;
      double cx[kU], cd[kU], cr[kU], cv[kU];
      cg_load(threadIdx.x, (int)threadIdx.x < n ? (int)threadIdx.x : -1, xs, cx, cd, cr, cv);
      for (int i0 = threadIdx.x; i0 < n; i0 += kU * B) {
        double nx[kU], nd[kU], nr[kU], nv[kU];
        cg_load(i0 + kU * B, i0, xs, nx, nd, nr, nv);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int i = i0 + u * B;
          if (i < n) {
            const int g = base + i;
            const int li = ld(i);
            const double pi = ps[li];
            const double hp = acc[li] + cv[u] * pi;
            xs[g] = cx[u] + alpha * pi;
            const double ri = cd[u] != 0.0 ? cr[u] - alpha * hp : 0.0;
            const double zi = cd[u] * ri;
            r[g] = ri;
            acc[li] = zi;
            rz1 += ri * zi;
            rr += ri * ri;
            zz += cv[u] * zi * zi;
            zp += cv[u] * zi * pi;
            pp += cv[u] * pi * pi;
          }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          cx[u] = nx[u];
          cd[u] = nd[u];
          cr[u] = nr[u];
          cv[u] = nv[u];
        }
      }
      {
        double t[2] = {rz1, rr};
        sum<2>(t);
        rz1 = t[0];
        rr = t[1];
      }
      iters = it + 1;
      if (rr <= tol2) {
        for (int i = threadIdx.x; i < n; i += B) acc[ld(i)] = 0.0;
        break;
      }
      const double beta = rz1 / rz;
      rz = rz1;
      pvp = zz + beta * (2.0 * zp + beta * pp);  // sum vd (z + beta p)^2 over this thread's DOFs
      for (int i = threadIdx.x; i < n; i += B) {
        const int li = ld(i);
        ps[li] = acc[li] + beta * ps[li];
        acc[li] = 0.0;
      }
      __syncthreads();
    }
    // every exit leaves p behind in LDS: clear it for the trial pass, which accumulates there
    for (int i = threadIdx.x; i < n; i += B) ps[ld(i)] = 0.0;
    __syncthreads();
    return rr;
  }

  // ISB_FLAG_INVALID_ACTION when an action of the body's elements or springs is <= 0 or not finite
  // (with ISB_FLAG_NONFINITE for the latter), else 0; every thread receives the same value
  __device__ int check_actions() {
    double t[2] = {0.0, 0.0};  // actions <= 0, non-finite actions
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const double ae = A.a[e];
      if (!isfinite(ae))
        t[1] += 1.0;
      else if (!(ae > 0.0))
        t[0] += 1.0;
    }
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
      const double as = A.a[m.n_e + s];
      if (!isfinite(as))
        t[1] += 1.0;
      else if (!(as > 0.0))
        t[0] += 1.0;
    }
    sum<2>(t);
    return (t[0] > 0.0 || t[1] > 0.0 ? ISB_FLAG_INVALID_ACTION : 0) | (t[1] > 0.0 ? ISB_FLAG_NONFINITE : 0);
  }

  // -------- the forward step of one body --------
  // per-DOF loops outside CG take kC owned DOFs per thread at a time, all loads first (indices
  // past the body clamped to its last DOF)
  static constexpr int kC = 4;

  __device__ void step(DevStats& st) {
    double* x = A.x1;
    double* xt = A.xt;
    const int B = blockDim.x;
    for (int i0 = threadIdx.x; i0 < n; i0 += kC * B) {
      double x0v[kC], v0v[kC];
      bool pin[kC];
#pragma unroll
      for (int u = 0; u < kC; ++u) {
        const int g = base + (i0 + u * B < n ? i0 + u * B : n - 1);
        x0v[u] = A.x0[g];
        v0v[u] = (sc.be && A.v0) ? A.v0[g] : 0.0;
        pin[u] = m.pinned[g] != 0;
      }
#pragma unroll
      for (int u = 0; u < kC; ++u)
        if (i0 + u * B < n) {
          const int g = base + i0 + u * B;
          const double xh = (sc.be && A.v0) ? x0v[u] + sc.h * v0v[u] : x0v[u];
          A.xhat[g] = xh;
          x[g] = pin[u] ? x0v[u] : xh;
        }
    }
    for (int vl = threadIdx.x; vl < v1 - v0; vl += blockDim.x)
      A.cv[v0 + vl] = fmax(-A.x0[(size_t)(v0 + vl) * D + 1] + sc.eps, 0.0);
    // invalid actions: no solve; x1 keeps x_init (each thread rereads the DOFs it wrote above)
    if (const int bad = check_actions()) {
      st.flags |= bad;
      if (sc.be && A.v1)
        for (int i = threadIdx.x; i < n; i += B) A.v1[base + i] = (x[base + i] - A.x0[base + i]) / sc.h;
      __syncthreads();
      return;
    }
    double* G = A.G;
    double* Gt = A.Gt;
    double* dx = A.dx;
    double* Ecur = A.E0;
    double* Enew = A.E1;
    double tr[4];
    trial(x, nullptr, 0.0, G, nullptr, Ecur, tr);
    const double res0 = sqrt(tr[3]);
    double res = res0, gcur = tr[2];
    double eta = 0.5, res_prev = res0;  // forcing term and the gradient norm it was set from
    st.res0 = res0;
    if (!isfinite(res0)) st.flags |= ISB_FLAG_NONFINITE;
    while (isfinite(res)) {
      if (res <= A.tol * res0 || res == 0.0) {
        st.flags |= ISB_FLAG_CONVERGED;
        break;
      }
      if (st.newton_iters >= A.max_newton) break;
      // forcing term (Eisenstat and Walker's second choice, with its safeguard): eta follows the
      // square of the last Newton step's reduction of the gradient, tight while Newton converges
      // fast and loose where it stalls (each Newton iteration costs a trial pass of about three CG
      // iterations, so tighter solves that save Newton iterations pay); the CG target stays above
      // half the Newton stopping threshold, which a more accurate last step could not improve on
      if (st.newton_iters > 0) {
        const double q = res / res_prev;
        double e = 0.9 * q * q;
        const double guard = 0.9 * eta * eta;
        if (guard > 0.1) e = fmax(e, guard);
        eta = fmin(0.5, e);
      }
      res_prev = res;
      int it = 0;
      bool neg = false;
      cg(G, -1.0, fmax(eta * res, 0.5 * A.tol * res0), A.max_cg, dx, it, neg);
      st.cg_iters += it;
      st.negcurv_exits += neg ? 1 : 0;
      double gTd = 0.0;
      for (int i0 = threadIdx.x; i0 < n; i0 += kC * B) {
        double gv[kC], dv[kC];
#pragma unroll
        for (int u = 0; u < kC; ++u) {
          const int g = base + (i0 + u * B < n ? i0 + u * B : n - 1);
          gv[u] = G[g];
          dv[u] = dx[g];
        }
#pragma unroll
        for (int u = 0; u < kC; ++u)
          if (i0 + u * B < n) gTd += gv[u] * dv[u];
      }
      gTd = sum1(gTd);
      if (!(gTd < 0.0)) {
        gTd = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
          const double d = -(double)A.Dv[base + i] * G[base + i];
          dx[base + i] = d;
          gTd += G[base + i] * d;
        }
        gTd = sum1(gTd);
        if (!(gTd < 0.0)) {
          st.flags |= ISB_FLAG_STAGNATED;
          break;
        }
      }
      double alpha = 1.0, rt = res;
      bool accepted = false;
      for (int ls = 0; ls <= 30; ++ls) {
        trial(x, dx, alpha, Gt, Ecur, Enew, tr, xt);
        rt = sqrt(tr[3]);
        if (isfinite(tr[0]) && isfinite(rt)) {
          if (fabs(tr[0]) > 1e3 * 2.220446049250313e-16 * tr[1]) {
            accepted = tr[0] <= 1e-4 * alpha * gTd;
          } else if (rt <= 0.5 * res || rt <= A.tol * res0) {
            // below the FP64 resolution of g the Armijo test only sees rounding: a step that at
            // least halves |grad g|, or brings it under the stopping threshold, is accepted instead
            accepted = true;
          } else {
            break;  // shorter steps cannot do better at the rounding floor
          }
        }
        if (accepted) break;
        alpha *= 0.5;
        st.ls_backtracks += 1;
      }
      if (!accepted) {
        // the preconditioner and the stored F now belong to the last rejected trial; the solve ends here
        st.flags |= ISB_FLAG_STAGNATED;
        break;
      }
      // the accepted trial point becomes the iterate (the trial's reduction published it)
      double* tmp = x;
      x = xt;
      xt = tmp;
      tmp = G;
      G = Gt;
      Gt = tmp;
      tmp = Ecur;
      Ecur = Enew;
      Enew = tmp;
      res = rt;
      gcur = tr[2];
      st.newton_iters += 1;
    }
    if (!isfinite(res)) st.flags |= ISB_FLAG_NONFINITE;
    st.res_final = res;
    if (res <= A.tol * res0) st.flags |= ISB_FLAG_CONVERGED;
    // x1 (when the iterate ended in the trial buffer) and v1 = (x1 - x0) / h
    const bool copy_x = x != A.x1, want_v = sc.be && A.v1;
    if (copy_x || want_v)
      for (int i0 = threadIdx.x; i0 < n; i0 += kC * B) {
        double xv[kC], x0v[kC];
#pragma unroll
        for (int u = 0; u < kC; ++u) {
          const int g = base + (i0 + u * B < n ? i0 + u * B : n - 1);
          xv[u] = x[g];
          x0v[u] = want_v ? A.x0[g] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kC; ++u)
          if (i0 + u * B < n) {
            const int g = base + i0 + u * B;
            if (copy_x) A.x1[g] = xv[u];
            if (want_v) A.v1[g] = (xv[u] - x0v[u]) / sc.h;
          }
      }
    st.energy = gcur;
    if (A.want_tail) minmax_J(x, st.min_J, st.max_J);
    __syncthreads();
  }

  // -------- the adjoint solve of one body (Eq. 9) --------
  __device__ void adjoint(DevStats& st) {
    const double* x = A.x1;
    for (int vl = threadIdx.x; vl < v1 - v0; vl += blockDim.x)
      A.cv[v0 + vl] = fmax(-A.x0[(size_t)(v0 + vl) * D + 1] + sc.eps, 0.0);
    double bb = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int g = base + i;
      double rhs = A.xbar[g];
      if (sc.be && A.vbar) rhs += A.vbar[g] / sc.h;
      if (pinned(i)) rhs = 0.0;
      A.G[g] = rhs;
      bb += rhs * rhs;
    }
    bb = sum1(bb);  // its barriers also publish cv
    if (const int bad = check_actions()) {
      st.flags |= bad;
      for (int i = threadIdx.x; i < n; i += blockDim.x) A.w[base + i] = 0.0;
      __syncthreads();
      return;
    }
    const double bnorm = sqrt(bb);
    int it = 0;
    bool neg = false;
    double rr = 0.0;
    if (!isfinite(bnorm)) {
      st.flags |= ISB_FLAG_NONFINITE;
    } else if (bnorm == 0.0) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) A.w[base + i] = 0.0;
    } else {
      precond(x);
      if (A.adj_warm) {
        // start from the given w: CG solves H d = b - H w for the correction d, whose residual is
        // that of H (w + d) = b, so the tolerance stays relative to |b|; w waits in dx meanwhile
        for (int i = threadIdx.x; i < n; i += blockDim.x) ps[ld(i)] = pinned(i) ? 0.0 : A.w[base + i];
        __syncthreads();
        pass_hv();
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
          const int g = base + i, li = ld(i);
          const double wi = ps[li];
          if (!pinned(i)) A.G[g] -= acc[li] + double(vdp()[g]) * wi;
          A.dx[g] = wi;
          acc[li] = 0.0;
          ps[li] = 0.0;
        }
        __syncthreads();
      }
      rr = cg(A.G, 1.0, A.adj_tol * bnorm, A.max_cg, A.w, it, neg);
      if (A.adj_warm)
        for (int i = threadIdx.x; i < n; i += blockDim.x) A.w[base + i] += A.dx[base + i];
    }
    st.adj_cg_iters = it;
    st.adj_res_final = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
    if (!neg && st.adj_res_final <= A.adj_tol) st.flags |= ISB_FLAG_ADJ_CONVERGED;
    __syncthreads();
  }
};

template <int D, typename T, int MODE, int EM = EM_NH, bool CR = false>  // MODE 0: step, 1: adjoint
__device__ void batched_body(const DevMesh& m, const DevScene& sc, const BatchArgs& A, double* smem, int g) {
  double* red = smem;
  double* acc = smem + kRedSlots;
  double* ps = acc + A.nacc;
  // LDS holds whatever the last kernel left: both accumulators start at zero, and every pass
  // clears the entries it used
  for (int i = threadIdx.x; i < 2 * A.nacc; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  // the host's static schedule: every quantity in this loop is scalar, so the loop and its
  // barriers stay uniform
  const int k0 = wg_uniform(A.wg_off[g]), k1 = wg_uniform(A.wg_off[g + 1]);
  for (int k = k0; k < k1; ++k) {
    const int body = wg_uniform(A.order[k]);
    const int bv0 = wg_uniform(A.voff[body]), bv1 = wg_uniform(A.voff[body + 1]);
    const int be0 = wg_uniform(A.eoff[body]), be1 = wg_uniform(A.eoff[body + 1]);
    BodySolver<D, T, EM, CR> S{m, sc, A, acc, red, ps, bv0, bv1, be0, be1, (bv1 - bv0) * D, bv0 * D};
    if (A.n_s > 0) {
      S.s0 = wg_uniform(A.soff[body]);
      S.s1 = wg_uniform(A.soff[body + 1]);
    }
    DevStats st;
    memset(&st, 0, sizeof(st));
    if (MODE == 0)
      S.step(st);
    else
      S.adjoint(st);
    if (threadIdx.x == 0) {
      DevStats& o = A.stats[body];
      if (MODE == 0) {
        const int adj = o.adj_cg_iters;
        const double ares = o.adj_res_final;
        const int aflag = o.flags & ISB_FLAG_ADJ_CONVERGED;
        o = st;
        o.adj_cg_iters = adj;
        o.adj_res_final = ares;
        o.flags |= aflag;
      } else {
        // the step's outcome stays; every other flag is this adjoint's own
        o.adj_cg_iters = st.adj_cg_iters;
        o.adj_res_final = st.adj_res_final;
        o.flags = (o.flags & (ISB_FLAG_CONVERGED | ISB_FLAG_STAGNATED | ISB_FLAG_FP64_FALLBACK)) | st.flags;
      }
    }
  }
}

}  // namespace isb
