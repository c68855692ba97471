// The element loop of one LDS-staged patch, shared by the patch scatter kernel and the resident
// CG solver: each thread takes elements eb + threadIdx.x, eb + threadIdx.x + blockDim.x, ... of
// the patch, gathers its corners from the patch's LDS copy of x (and of the Hessian-vector operand
// p), evaluates the element operation (Eq. 3's gradient, Hessian-vector product or Jacobi
// diagonal) and adds s_pot times its per-corner result into the LDS accumulator with LDS atomics.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "isb_device.hpp"
#include "isb_elem.hpp"
#include "isb_internal.hpp"

namespace isb {

// One element's Hessian-vector product on the patch's LDS copy of p (corners l), added s_pot-scaled
// into the LDS accumulator; with want_curv, php gains p_e . (H_e p_e) (unscaled).
template <int D, typename T, int EM>
__device__ __forceinline__ void patch_hv_element(const ElemRest<D, T>& R, const ElemState<D, T>& S, T ae,
                                                 const int l[D + 1], const double* ps, double* acc, double s_pot,
                                                 bool want_curv, double& php) {
  T dDs[D][D];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int c = 0; c < D; ++c) dDs[c][j] = T(ps[l[j + 1] * D + c] - ps[l[0] * D + c]);
  T o[D + 1][D];
  elem_hessvec<D, T, EM>(R, S, ae, dDs, o);
  if (want_curv) {
    // p_e . (H_e p_e) = sum_j o_{j+1} . (p_{j+1} - p_0), since o_0 = -sum_j o_{j+1}
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int c = 0; c < D; ++c) php += double(o[j + 1][c]) * (ps[l[j + 1] * D + c] - ps[l[0] * D + c]);
  }
#pragma unroll
  for (int k = 0; k <= D; ++k)
#pragma unroll
    for (int c = 0; c < D; ++c) unsafeAtomicAdd(acc + l[k] * D + c, s_pot * double(o[k][c]));
}

// lconn: [(D+1)][n_e] patch-local corner ids; xs, ps, acc: [local vertex][D] in LDS, FP64 (edge
// differences of x and p are formed in FP64, then rounded to T). Slots [eb, ee) hold the elements
// eperm[slot] (the slots themselves when eperm is null). php (Hessian-vector products with
// want_curv): this thread's sum over its elements of p_e . (H_e p_e), unscaled by s_pot.
template <int D, typename T, int OP, int EM, bool CR>
__device__ __forceinline__ void patch_elements(const DevMesh& m, const DevScene& sc, const uint16_t* __restrict__ lconn,
                                               const int32_t* __restrict__ eperm, int eb, int ee, const double* xs,
                                               const double* ps, double* acc, const double* __restrict__ a,
                                               const float* __restrict__ a32, bool want_curv, double& php) {
  for (int slot = eb + threadIdx.x; slot < ee; slot += blockDim.x) {
    const int e = eperm ? eperm[slot] : slot;
    int l[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) l[k] = lconn[(size_t)k * m.n_e + e];
    ElemRest<D, T> R;
    load_rest<D, T, CR>(m, e, R);
    T Ds[D][D];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int c = 0; c < D; ++c) Ds[c][j] = T(xs[l[j + 1] * D + c] - xs[l[0] * D + c]);
    ElemState<D, T> S;
    elem_state<D, T>(Ds, R, S);
    // actuation in the element precision: the FP32 copy when the caller made one
    const T ae = (std::is_same<T, float>::value && a32) ? T(a32[e]) : T(a[e]);
    if constexpr (OP == PATCH_HV) {
      patch_hv_element<D, T, EM>(R, S, ae, l, ps, acc, sc.s_pot, want_curv, php);
    } else {
      T o[D + 1][D];
      if constexpr (OP == PATCH_GRAD)
        elem_grad<D, T, EM>(R, S, ae, o);
      else
        elem_hessdiag<D, T, EM>(R, S, ae, o);
#pragma unroll
      for (int k = 0; k <= D; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) unsafeAtomicAdd(acc + l[k] * D + c, sc.s_pot * double(o[k][c]));
    }
  }
}

}  // namespace isb
