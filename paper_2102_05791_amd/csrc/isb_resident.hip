// Resident single-reduction PCG for one body whose element patches can all be resident on the
// GPU at once (one workgroup per patch, every workgroup co-resident): the whole inner solve of a
// Newton step (the linear system of Eq. 1 through Eq. 14) or of the adjoint (Eq. 9) is one
// cooperative launch, with one grid barrier per iteration and the CG vectors of each patch in LDS.
//
// Each workgroup keeps x, u = M r, r, p, s = H p, M (= D^-1), the vertex diagonal, the solution and
// an accumulator for every vertex of its patch, including the vertices it shares with other patches.
// It updates all of them itself, with the same scalars and the same arithmetic as every other
// workgroup that holds them, so the shared copies stay identical. Only the element part of H u
// crosses workgroups, and only at the vertices two or more patches hold (listed first in each
// patch): each patch adds its sums there into a global vector with FP64 atomics, and every
// workgroup reads back the complete sums after the barrier; at its interior vertices the sums stay
// in LDS. Three such vectors rotate (summed into, read, cleared), so one barrier per iteration
// suffices. The curvature u^T H u comes
// from the element pass itself (sum over elements of u_e . H_e u_e, plus the vertex diagonal's
// part), so r.u, u^T H u and r.r of an iteration reach the next one as one set of per-workgroup
// partials, which every workgroup folds in the same order: all of them take the same decisions.
//
// The iteration is the Chronopoulos-Gear form of the patch path's single-reduction CG:
//   beta = gamma / gamma_prev, p^T H p = delta - beta gamma / alpha_prev, alpha = gamma / p^T H p,
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = M r, w = H u,
// stopping when r.r <= tol^2, at the iteration cap, or on non-positive curvature (Nocedal and
// Wright, Alg. 7.1: on the first iteration the preconditioned steepest-descent direction M b).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "isb_body.hpp"
#include "isb_device.hpp"
#include "isb_elem.hpp"
#include "isb_internal.hpp"
#include "isb_patch.hpp"

namespace isb {

__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every value one workgroup passes to another (the sums of H u, the partials, the cleared sums)
// goes through agent-scope loads, stores and atomics, which are coherent across the GPU's L2 slices
// without cache maintenance. A barrier therefore needs no release/acquire fences (each would write
// back and invalidate the whole L2 of the workgroup's XCD, several microseconds at every barrier):
// each wave waits until its own stores and atomics have completed (vmcnt(0)), and the arrival and
// the wait are relaxed atomics. Arrival goes up a two-level tree, so that no counter takes more
// than one XCD's arrivals: the workgroup counts itself on its group's counter, the group's last
// arrival counts the group on the top counter, and the last group's last arrival stores the
// barrier's number into the release word, which every other workgroup polls. All counters are
// monotone (zeroed before the launch): barrier number k is complete at k times the arrivals.
__device__ __forceinline__ void wait_vm_stores() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt not waited for
}

__device__ __forceinline__ unsigned ld_agent_u(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns false on every thread of the workgroup when the launch has been aborted: a workgroup that
// waits more than max_ticks of the constant-rate wall clock marks the launch aborted, and every
// workgroup then leaves the solve.
__device__ __forceinline__ bool grid_barrier(GridBar* g, unsigned& epoch, int* ok_lds, uint64_t max_ticks) {
  wait_vm_stores();
  __syncthreads();
  ++epoch;
  if (threadIdx.x == 0) {
    const unsigned G = gridDim.x, x = blockIdx.x % kBarGroups;
    const unsigned n_groups = G < (unsigned)kBarGroups ? G : (unsigned)kBarGroups;
    const unsigned in_group = (G - x + kBarGroups - 1) / kBarGroups;  // workgroups x, x + 8, ... < G
    bool last = false;
    if (__hip_atomic_fetch_add(&g->group[x][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
        epoch * in_group - 1u)
      last = __hip_atomic_fetch_add(&g->top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch * n_groups - 1u;
    int ok = 1;
    if (last) {
      __hip_atomic_store(&g->flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (ld_agent_u(&g->flag) < epoch) {
        if (ld_agent_u(&g->abort) != 0u || wall_clock64() - t0 > max_ticks) {
          __hip_atomic_store(&g->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    *ok_lds = ok;
  }
  __syncthreads();
  return *ok_lds != 0;
}

// this workgroup's sums of three values, stored to out[0..3) (agent scope, for the other workgroups)
template <int PB>
__device__ __forceinline__ void workgroup_sums3(double a, double b, double c, double* red, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a = wave_total(a);
  b = wave_total(b);
  c = wave_total(c);
  if (lane == 0) {
    red[3 * wid] = a;
    red[3 * wid + 1] = b;
    red[3 * wid + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < PB / 64; ++w) t += red[3 * w + threadIdx.x];
    st_agent(out + threadIdx.x, t);
  }
  __syncthreads();
}

// (gamma, r.r, delta) from the partials of all workgroups (4 values each, the fourth unused), in
// the same order on every workgroup and every thread
template <int PB>
__device__ __forceinline__ void fold_partials(const double* bank, double* red, double& gamma, double& rr,
                                              double& delta) {
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += PB) {
    v0 += ld_agent(bank + 4 * b);
    v1 += ld_agent(bank + 4 * b + 1);
    v2 += ld_agent(bank + 4 * b + 2);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v0 = wave_total(v0);
  v1 = wave_total(v1);
  v2 = wave_total(v2);
  if (lane == 0) {
    red[3 * wid] = v0;
    red[3 * wid + 1] = v1;
    red[3 * wid + 2] = v2;
  }
  __syncthreads();
  gamma = rr = delta = 0.0;
  for (int w = 0; w < PB / 64; ++w) {
    gamma += red[3 * w];
    rr += red[3 * w + 1];
    delta += red[3 * w + 2];
  }
  __syncthreads();
}

// Elements whose rest data and state stay in registers for the whole solve (x does not change
// during it): the first KE * PB elements of the patch, KE per thread. FP32 neo-Hookean only, whose
// state fits a 512-thread workgroup's register budget beside the Hessian-vector product; other
// configurations keep none and evaluate every element's state at every product.
template <typename T, int EM, int PB>
constexpr int resident_cached_per_thread() {
  return (std::is_same<T, float>::value && EM == EM_NH && PB <= 512) ? 3 : 0;
}

// H_elem u of the patch into acc: the cached elements [eb, ec) from registers, the rest [ec, ee)
// from LDS x and the rest data in memory
template <int D, typename T, int EM, bool CR, int PB, int KE, int KS>
__device__ __forceinline__ void resident_hv_pass(const DevMesh& m, const DevScene& sc, const PatchPlan& P, int eb,
                                                 int ec, int ee, const double* xl, const double* ul, double* acc,
                                                 const double* __restrict__ a, const float* __restrict__ a32,
                                                 const ElemRest<D, T> (&cR)[KS], const ElemState<D, T> (&cS)[KS],
                                                 const T (&ca)[KS], const int (&cl)[KS][D + 1], double& php) {
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    if (eb + (int)threadIdx.x + k * PB < ec)
      patch_hv_element<D, T, EM>(cR[k], cS[k], ca[k], cl[k], ul, acc, sc.s_pot, true, php);
  }
  patch_elements<D, T, PATCH_HV, EM, CR>(m, sc, P.lconn, P.eperm, ec, ee, xl, ul, acc, a, a32, true, php);
}

// The workgroup of patch p0 + blockIdx.x. LDS: nine [max_nv][D] FP64 arrays, then the vertex ids
// (v owned, ~v shared and owned elsewhere). W0..W2: [n_v][D] global sums of H_elem u; part: two
// banks of 4 * gridDim.x partials; bar zeroed before the launch.
template <int D, typename T, int EM, bool CR, int PB>
__global__ void __launch_bounds__(PB)
    k_cg_resident(DevMesh m, DevScene sc, PatchPlan P, int p0, const double* __restrict__ x,
                  const double* __restrict__ a, const float* __restrict__ a32, const double* __restrict__ rhs,
                  double sign, const double* __restrict__ Dinvp, const double* __restrict__ vdiag, double* xs_out,
                  double* W0, double* W1, double* W2, double* part, GridBar* bar, CgScal* scal, double tol2,
                  int max_it, uint64_t max_ticks) {
  extern __shared__ double lds[];
  __shared__ double red[3 * (PB / 64)];
  __shared__ int ok_lds;
  const int pk = p0 + blockIdx.x;
  const int vb = P.voff[pk], nv = P.voff[pk + 1] - vb, nd = nv * D;
  // DOFs [0, nds) belong to vertices other patches hold too and go through the global sums; the
  // element part of H u at the rest (vertices only this patch holds) stays in acc
  const int nds = (P.nshared ? P.nshared[pk] : nv) * D;
  const int eb = P.eoff[pk], ee = P.eoff[pk + 1];
  const int nmax = P.max_nv * D;
  double* xl = lds;
  double* ul = xl + nmax;
  double* rl = ul + nmax;
  double* pl = rl + nmax;
  double* sl = pl + nmax;
  double* dl = sl + nmax;
  double* vl = dl + nmax;
  double* acc = vl + nmax;
  double* xsl = acc + nmax;
  int* vid = reinterpret_cast<int*>(xsl + nmax);
  unsigned epoch = 0;

  for (int v = threadIdx.x; v < nv; v += PB) vid[v] = P.verts[vb + v];
  __syncthreads();
  // r = b on the free DOFs, u = M r, p = s = x_s = 0; clear W0 and W1 (owned shared DOFs)
  double g_ = 0.0, r_ = 0.0, d_ = 0.0;
  for (int i = threadIdx.x; i < nd; i += PB) {
    const int v = i / D, c = i - v * D, raw = vid[v];
    const size_t g = (size_t)(raw >= 0 ? raw : ~raw) * D + c;
    const double di = Dinvp[g], vi = vdiag[g];
    const double ri = di != 0.0 ? sign * rhs[g] : 0.0, ui = di * ri;
    xl[i] = x[g];
    dl[i] = di;
    vl[i] = vi;
    rl[i] = ri;
    ul[i] = ui;
    pl[i] = 0.0;
    sl[i] = 0.0;
    xsl[i] = 0.0;
    acc[i] = 0.0;
    if (raw >= 0) {
      if (i < nds) {
        st_agent(W0 + g, 0.0);
        st_agent(W1 + g, 0.0);
      }
      g_ += ri * ui;
      r_ += ri * ri;
      d_ += ui * (vi * ui);
    }
  }
  __syncthreads();  // x of every patch vertex in LDS
  constexpr int KE = resident_cached_per_thread<T, EM, PB>();
  constexpr int KS = KE > 0 ? KE : 1;
  const int ec = min(ee, eb + KE * PB);
  ElemRest<D, T> cR[KS];
  ElemState<D, T> cS[KS];
  T ca[KS];
  int cl[KS][D + 1];
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int slot = eb + threadIdx.x + k * PB;
    if (slot < ec) {
      const int e = P.eperm ? P.eperm[slot] : slot;
#pragma unroll
      for (int q = 0; q <= D; ++q) cl[k][q] = P.lconn[(size_t)q * m.n_e + e];
      load_rest<D, T, CR>(m, e, cR[k]);
      T Ds[D][D];
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int c = 0; c < D; ++c) Ds[c][j] = T(xl[cl[k][j + 1] * D + c] - xl[cl[k][0] * D + c]);
      elem_state<D, T>(Ds, cR[k], cS[k]);
      ca[k] = (std::is_same<T, float>::value && a32) ? T(a32[e]) : T(a[e]);
    }
  }
  bool ok = grid_barrier(bar, epoch, &ok_lds, max_ticks);
  if (ok) {
    // H u_0 into W0
    double php = 0.0;
    resident_hv_pass<D, T, EM, CR, PB, KE, KS>(m, sc, P, eb, ec, ee, xl, ul, acc, a, a32, cR, cS, ca, cl, php);
    __syncthreads();
    for (int i = threadIdx.x; i < nds; i += PB) {
      const int v = i / D, c = i - v * D, raw = vid[v];
      unsafeAtomicAdd(W0 + (size_t)(raw >= 0 ? raw : ~raw) * D + c, acc[i]);
    }
    workgroup_sums3<PB>(g_, r_, d_ + sc.s_pot * php, red, part + 4 * blockIdx.x);
    ok = grid_barrier(bar, epoch, &ok_lds, max_ticks);
  }

  int it = 0, negcurv = 0;
  double rr = 0.0, rr0 = 0.0, pHp = 0.0, alpha_prev = 0.0, gamma_prev = 0.0;
  // DOF slots per thread (DOFs threadIdx.x + k * PB) whose sums are prefetched: three, and none
  // where the element cache holds the registers (the prefetch's registers then spill, which costs
  // more than it saves); later slots load their sums in the update pass
  constexpr int KP = KE > 0 ? 0 : 3;
  while (ok) {
    // W[it % 3] holds H_elem u_it (complete since the barrier). This thread's entries are loaded
    // first, all together and before the partials, so that one round trip covers the global reads
    // of the iteration; a slot past the patch loads its last DOF again and is not used.
    const double* Wc = it % 3 == 0 ? W0 : (it % 3 == 1 ? W1 : W2);
    double wv[KP > 0 ? KP : 1];
#pragma unroll
    for (int k = 0; k < (KP > 0 ? KP : 1); ++k) wv[k] = 0.0;
    if (nds > 0) {
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        int i = min((int)threadIdx.x + k * PB, nds - 1);
        // the slot's index is formed anew each iteration, not hoisted out of the loop and held
        // through the element pass
        asm volatile("" : "+v"(i));
        const int v = i / D, c = i - v * D, raw = vid[v];
        wv[k] = ld_agent(Wc + (size_t)(raw >= 0 ? raw : ~raw) * D + c);
      }
    }
    double gamma, delta;
    fold_partials<PB>(part + (it & 1) * 4 * gridDim.x, red, gamma, rr, delta);
    if (it == 0) rr0 = rr;
    if (rr <= tol2 || it >= max_it) break;
    const double beta = it == 0 ? 0.0 : gamma / gamma_prev;
    pHp = it == 0 ? delta : delta - beta * gamma / alpha_prev;
    if (!(pHp > 0.0)) {
      negcurv = 1;
      if (it == 0)
        for (int i = threadIdx.x; i < nd; i += PB) xsl[i] = ul[i];
      break;
    }
    const double alpha = gamma / pHp;
    // this iteration sums H_elem u_{it+1} into the next W and clears the one after (read last in
    // the previous iteration, before the barrier every workgroup has passed)
    double* Wn = it % 3 == 0 ? W1 : (it % 3 == 1 ? W2 : W0);
    double* Wz = it % 3 == 0 ? W2 : (it % 3 == 1 ? W0 : W1);
    g_ = r_ = d_ = 0.0;
    // the update of DOF i (global index g, encoded vertex raw) given the element part wk of H u
    auto update_dof = [&](int i, size_t g, int raw, double wk) {
      const double vi = vl[i], di = dl[i];
      const double wi = vi * ul[i] + wk;
      const double pi = ul[i] + beta * pl[i];
      const double si = wi + beta * sl[i];
      xsl[i] += alpha * pi;
      const double ri = di != 0.0 ? rl[i] - alpha * si : 0.0;
      const double ui = di * ri;
      pl[i] = pi;
      sl[i] = si;
      rl[i] = ri;
      ul[i] = ui;
      acc[i] = 0.0;
      if (raw >= 0) {
        if (i < nds) st_agent(Wz + g, 0.0);
        g_ += ri * ui;
        r_ += ri * ri;
        d_ += ui * (vi * ui);
      }
    };
    if constexpr (KP == 0) {
      // two DOF slots per trip, both sums requested before either is used: one round trip
      // for both, without holding prefetched values through the fold
      for (int i = threadIdx.x; i < nd; i += 2 * PB) {
        const int j = i + PB;
        const int vi_ = i / D, raw_i = vid[vi_];
        const size_t g_i = (size_t)(raw_i >= 0 ? raw_i : ~raw_i) * D + (i - vi_ * D);
        const double w_i = i < nds ? ld_agent(Wc + g_i) : acc[i];
        int raw_j = 0;
        size_t g_j = 0;
        double w_j = 0.0;
        if (j < nd) {
          const int vj_ = j / D;
          raw_j = vid[vj_];
          g_j = (size_t)(raw_j >= 0 ? raw_j : ~raw_j) * D + (j - vj_ * D);
          w_j = j < nds ? ld_agent(Wc + g_j) : acc[j];
        }
        update_dof(i, g_i, raw_i, w_i);
        if (j < nd) update_dof(j, g_j, raw_j, w_j);
      }
    } else {
      for (int i = threadIdx.x, k = 0; i < nd; i += PB, ++k) {
        const int v = i / D, c = i - v * D, raw = vid[v];
        const size_t g = (size_t)(raw >= 0 ? raw : ~raw) * D + c;
        double wk = i >= nds ? acc[i] : (k < KP ? wv[0] : ld_agent(Wc + g));
#pragma unroll
        for (int q = 1; q < KP; ++q) wk = (k == q && i < nds) ? wv[q] : wk;
        update_dof(i, g, raw, wk);
      }
    }
    __syncthreads();
    double php = 0.0;
    resident_hv_pass<D, T, EM, CR, PB, KE, KS>(m, sc, P, eb, ec, ee, xl, ul, acc, a, a32, cR, cS, ca, cl, php);
    __syncthreads();
    for (int i = threadIdx.x; i < nds; i += PB) {
      const int v = i / D, c = i - v * D, raw = vid[v];
      unsafeAtomicAdd(Wn + (size_t)(raw >= 0 ? raw : ~raw) * D + c, acc[i]);
    }
    workgroup_sums3<PB>(g_, r_, d_ + sc.s_pot * php, red, part + ((it + 1) & 1) * 4 * gridDim.x + 4 * blockIdx.x);
    gamma_prev = gamma;
    alpha_prev = alpha;
    ++it;
    ok = grid_barrier(bar, epoch, &ok_lds, max_ticks);
  }

  for (int i = threadIdx.x; i < nd; i += PB) {
    const int v = i / D, c = i - v * D, raw = vid[v];
    if (raw >= 0) xs_out[(size_t)raw * D + c] = xsl[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal->rr = rr;
    scal->rr0 = rr0;
    scal->pHp = pHp;
    scal->tol2 = tol2;
    scal->done = 1;
    scal->negcurv = negcurv;
    scal->iters = it;
    scal->it_cur = it;
    scal->max_it = max_it;
    scal->fault = ok ? 0 : 1;
    scal->alpha_prev = alpha_prev;
    scal->gamma_prev = gamma_prev;
  }
}

__global__ void k_grid_bar_reset(GridBar* g) {
  unsigned* w = reinterpret_cast<unsigned*>(g);
  for (int i = threadIdx.x; i < (int)(sizeof(GridBar) / sizeof(unsigned)); i += blockDim.x) w[i] = 0u;
}

template <int D, typename T, int EM, bool CR>
static const void* resident_kernel_for() {
  constexpr int PB = std::is_same<T, float>::value ? kResidentBlockF32 : kResidentBlockF64;
  return reinterpret_cast<const void*>(&k_cg_resident<D, T, EM, CR, PB>);
}

template <int D, typename T>
static const void* resident_kernel_dt(int model, bool compact) {
  switch (model) {
    case EM_STVK: return compact ? resident_kernel_for<D, T, EM_STVK, true>() : resident_kernel_for<D, T, EM_STVK, false>();
    case EM_COROT: return compact ? resident_kernel_for<D, T, EM_COROT, true>() : resident_kernel_for<D, T, EM_COROT, false>();
    case EM_SNH: return compact ? resident_kernel_for<D, T, EM_SNH, true>() : resident_kernel_for<D, T, EM_SNH, false>();
    default: return compact ? resident_kernel_for<D, T, EM_NH, true>() : resident_kernel_for<D, T, EM_NH, false>();
  }
}

bool resident_caches_elements(int precision, int model) {
  return precision ? resident_cached_per_thread<float, EM_NH, kResidentBlockF32>() > 0 && model == EM_NH
                   : resident_cached_per_thread<double, EM_NH, kResidentBlockF64>() > 0 && model == EM_NH;
}

hipError_t launch_cg_resident(const DevMesh& m, const DevScene& sc, const PatchPlan& P, int p0, int np, int n_cu,
                              int precision, const double* x, const double* a, const float* a32, const double* rhs,
                              double sign, const double* Dinvp, const double* vdiag, double* xs, double* W0,
                              double* W1, double* W2, double* part, GridBar* bar, CgScal* scal, double tol2,
                              int max_it, int64_t barrier_limit_us, hipStream_t s) {
  if (np < 1) return hipErrorInvalidValue;
  const bool compact = m.axis >= 0;
  const void* k = m.dim == 2 ? (precision ? resident_kernel_dt<2, float>(m.model, compact)
                                          : resident_kernel_dt<2, double>(m.model, compact))
                             : (precision ? resident_kernel_dt<3, float>(m.model, compact)
                                          : resident_kernel_dt<3, double>(m.model, compact));
  const int block = precision ? kResidentBlockF32 : kResidentBlockF64;
  const size_t lds = (size_t)P.max_nv * resident_vertex_bytes(m.dim);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int occ = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, block, lds);
  if (e != hipSuccess) return e;
  if (occ * n_cu < np) return hipErrorCooperativeLaunchTooLarge;
  int rate_khz = 0;  // the wall clock's rate
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  if (rate_khz <= 0) return hipErrorInvalidValue;
  uint64_t max_ticks = (uint64_t)barrier_limit_us * (uint64_t)rate_khz / 1000ull;
  if (max_ticks < 1) max_ticks = 1;
  k_grid_bar_reset<<<1, 256, 0, s>>>(bar);
  DevMesh mm = m;
  DevScene ss = sc;
  PatchPlan pp = P;
  void* args[] = {&mm, &ss, &pp, &p0, &x, &a, &a32, &rhs, &sign, &Dinvp, &vdiag, &xs,
                  &W0, &W1, &W2, &part, &bar, &scal, &tol2, &max_it, &max_ticks};
  return hipLaunchCooperativeKernel(k, dim3(np), dim3(block), args, (unsigned)lds, s);
}

}  // namespace isb
