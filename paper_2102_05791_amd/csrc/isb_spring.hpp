// Vertex-pair springs: Eq. 2 read literally, with l(x) = |x_j - x_i| the length of the segment
// between two vertices (the energies of d = x_j - x_i in the paper's computation-graph view, Fig. 2):
//
//   E_s = k/2 (l / (a l0) - 1)^2,    l0 = |X_j - X_i|,  a the spring's own action.
//
// With c = 1/(a l0), n = d/l and f = dE/dl = k c (c l - 1):
//   gradient         +f n at j, -f n at i
//   Hessian blocks   [[K, -K], [-K, K]],  K = k c^2 n n^T + (f/l)(I - n n^T)
//   action cotangent dG_j/da = -(k c (2 c l - 1) / a) n
// All spring arithmetic is FP64 (a spring costs a few dozen flops; no FP32 variant).
#pragma once

#include <hip/hip_runtime.h>

namespace isb {

// words of the symmetric D x D spring block K kept per spring between Hessian-vector passes
__host__ __device__ constexpr int spring_state_words(int dim) { return dim * (dim + 1) / 2; }

template <int D>
struct SpringTerms {
  double n[D];  // unit direction i -> j
  double l;     // current length
  double c;     // 1 / (a l0)
  double f;     // dE/dl
  double kn;    // k c^2: stiffness along n
  double kt;    // f / l: stiffness across n
};

// d = x_j - x_i; il0 = 1 / l0
template <int D>
__device__ __forceinline__ void spring_terms(const double d[D], double k, double il0, double a, SpringTerms<D>& S) {
  double l2 = 0.0;
#pragma unroll
  for (int r = 0; r < D; ++r) l2 += d[r] * d[r];
  S.l = sqrt(l2);
  const double il = 1.0 / S.l;
#pragma unroll
  for (int r = 0; r < D; ++r) S.n[r] = d[r] * il;
  S.c = il0 / a;
  S.f = k * S.c * (S.c * S.l - 1.0);
  S.kn = k * S.c * S.c;
  S.kt = S.f * il;
}

template <int D>
__device__ __forceinline__ double spring_energy(const SpringTerms<D>& S, double k) {
  const double t = S.c * S.l - 1.0;
  return 0.5 * k * t * t;
}

// y = K u
template <int D>
__device__ __forceinline__ void spring_apply(const SpringTerms<D>& S, const double u[D], double y[D]) {
  double nu = 0.0;
#pragma unroll
  for (int r = 0; r < D; ++r) nu += S.n[r] * u[r];
#pragma unroll
  for (int r = 0; r < D; ++r) y[r] = S.kt * u[r] + (S.kn - S.kt) * nu * S.n[r];
}

// K_rr, the Hessian diagonal each end receives
template <int D>
__device__ __forceinline__ void spring_diag(const SpringTerms<D>& S, double dg[D]) {
#pragma unroll
  for (int r = 0; r < D; ++r) dg[r] = S.kt + (S.kn - S.kt) * S.n[r] * S.n[r];
}

// upper triangle of K row by row (spring_state_words(D) values)
template <int D>
__device__ __forceinline__ void spring_block(const SpringTerms<D>& S, double* K) {
  int w = 0;
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int q = r; q < D; ++q, ++w) K[w] = (r == q ? S.kt : 0.0) + (S.kn - S.kt) * S.n[r] * S.n[q];
}

// y = K u from the stored upper triangle
template <int D, typename T>
__device__ __forceinline__ void spring_block_apply(const T* K, const T u[D], T y[D]) {
#pragma unroll
  for (int r = 0; r < D; ++r) y[r] = T(0);
  int w = 0;
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int q = r; q < D; ++q, ++w) {
      y[r] += K[w] * u[q];
      if (q != r) y[q] += K[w] * u[r];
    }
}

// -w^T dG/da and -w^T dG/dk for dw = w_j - w_i (before the s_pot scale)
template <int D>
__device__ __forceinline__ void spring_vjp(const SpringTerms<D>& S, double k, double a, const double dw[D],
                                           double& a_bar, double& k_bar) {
  double ndw = 0.0;
#pragma unroll
  for (int r = 0; r < D; ++r) ndw += S.n[r] * dw[r];
  a_bar = k * S.c * (2.0 * S.c * S.l - 1.0) / a * ndw;
  k_bar = -S.c * (S.c * S.l - 1.0) * ndw;
}

}  // namespace isb
