// Per-element energy, gradient, Hessian-vector product, Hessian diagonal and parameter
// cotangents of the neo-Hookean + contractile-fibre element (Sec. 3, Eq. 2-3).
//
// Every routine works on one simplex with D = 2 (triangle) or 3 (tetrahedron) in the
// element precision T (double, or float in mixed mode). The element sees the vertex
// positions only through the edge matrix Ds = [x_1 - x_0, ..., x_D - x_0], so that
// F = Ds Dm^-1 is linear in x (Sec. 3). Rest data per element: Dm^-1, the fibre vector
// gf = Dm^-1 d (so F d = Ds gf), and W mu, W lam, W k_f with W the rest volume.
//
// Energy density (W times):
//   psi = mu/2 (I1 - D) - mu l(J) + lam/2 l(J)^2 + k_f/2 (s/a - 1)^2,   s = |F d|
// with l(J) = (J-1) - (J-1)^2/2, the quadratic expansion of log J about J = 1 that stays
// finite for inverted elements. First Piola stress:
//   P = mu F + (lam l - mu) l' cof F + (k_f/a)(s/a - 1) n d^T,          n = F d / s
// and its differential along dF (q = dF d):
//   dP = mu dF + (lam l - mu) l' dcof(dF) + [lam l'^2 + (lam l - mu) l''] (cof F : dF) cof F
//        + (k_f/a^2)(n.q) n d^T + (k_f/a)(s/a - 1)/s (q - n (n.q)) d^T.
// The gradient w.r.t. Ds is W P Dm^-T: its column j is the gradient at vertex j+1 and
// vertex 0 takes minus the column sum. Where s = 0 the fibre direction is undefined and
// the fibre contributes nothing to the gradient and Hessian.
#pragma once

#include <hip/hip_runtime.h>

namespace isb {

template <int D, typename T>
struct ElemRest {
  T Dinv[D][D];
  T gf[D];
  T wmu, wlam, wkf;
};

template <int D, typename T>
struct ElemState {
  T F[D][D];
  T C[D][D];   // cof F = dJ/dF
  T J, l, dl;  // det F, l(J), l'(J)
  T s, sinv;   // fibre stretch |F d| and its inverse (0 when s == 0)
  T n[D];      // F d / s
};

template <int D, typename T>
__device__ __forceinline__ void cofactor(const T F[D][D], T C[D][D]) {
  if constexpr (D == 2) {
    C[0][0] = F[1][1];
    C[0][1] = -F[1][0];
    C[1][0] = -F[0][1];
    C[1][1] = F[0][0];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = (k + 1) % 3, j = (k + 2) % 3;
      // column k of cof F is (column i) x (column j)
      C[0][k] = F[1][i] * F[2][j] - F[2][i] * F[1][j];
      C[1][k] = F[2][i] * F[0][j] - F[0][i] * F[2][j];
      C[2][k] = F[0][i] * F[1][j] - F[1][i] * F[0][j];
    }
  }
}

// directional derivative of cof F along dF
template <int D, typename T>
__device__ __forceinline__ void cofactor_diff(const T F[D][D], const T dF[D][D], T dC[D][D]) {
  if constexpr (D == 2) {
    cofactor<2, T>(dF, dC);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = (k + 1) % 3, j = (k + 2) % 3;
      dC[0][k] = dF[1][i] * F[2][j] - dF[2][i] * F[1][j] + F[1][i] * dF[2][j] - F[2][i] * dF[1][j];
      dC[1][k] = dF[2][i] * F[0][j] - dF[0][i] * F[2][j] + F[2][i] * dF[0][j] - F[0][i] * dF[2][j];
      dC[2][k] = dF[0][i] * F[1][j] - dF[1][i] * F[0][j] + F[0][i] * dF[1][j] - F[1][i] * dF[0][j];
    }
  }
}

// M = Ds Dm^-1
template <int D, typename T>
__device__ __forceinline__ void mul_dinv(const T Ds[D][D], const T Dinv[D][D], T M[D][D]) {
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) acc += Ds[r][j] * Dinv[j][c];
      M[r][c] = acc;
    }
}

template <int D, typename T>
__device__ __forceinline__ void elem_state(const T Ds[D][D], const ElemRest<D, T>& R, ElemState<D, T>& S) {
  mul_dinv<D, T>(Ds, R.Dinv, S.F);
  cofactor<D, T>(S.F, S.C);
  T J = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) J += S.F[r][0] * S.C[r][0];
  S.J = J;
  const T jm1 = J - T(1);
  S.l = jm1 - T(0.5) * jm1 * jm1;
  S.dl = T(2) - J;
  T ss = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) {
    T fd = T(0);
#pragma unroll
    for (int j = 0; j < D; ++j) fd += Ds[r][j] * R.gf[j];
    S.n[r] = fd;
    ss += fd * fd;
  }
  S.s = sqrt(ss);
  S.sinv = S.s > T(0) ? T(1) / S.s : T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) S.n[r] *= S.sinv;
}

// the same state from a stored F and F d (no vertex gather)
template <int D, typename T>
__device__ __forceinline__ void elem_state_from_F(const T F[D][D], const T Fd[D], ElemState<D, T>& S) {
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) S.F[r][c] = F[r][c];
  cofactor<D, T>(S.F, S.C);
  T J = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) J += S.F[r][0] * S.C[r][0];
  S.J = J;
  const T jm1 = J - T(1);
  S.l = jm1 - T(0.5) * jm1 * jm1;
  S.dl = T(2) - J;
  T ss = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) ss += Fd[r] * Fd[r];
  S.s = sqrt(ss);
  S.sinv = S.s > T(0) ? T(1) / S.s : T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) S.n[r] = Fd[r] * S.sinv;
}

// W psi(F)
template <int D, typename T>
__device__ __forceinline__ T elem_energy(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a) {
  T I1 = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) I1 += S.F[r][c] * S.F[r][c];
  const T e = S.s / a - T(1);
  return T(0.5) * R.wmu * (I1 - T(D)) - R.wmu * S.l + T(0.5) * R.wlam * S.l * S.l + T(0.5) * R.wkf * e * e;
}

// Map a W-scaled stress-like matrix Q (NH part, times Dm^-T) plus a fibre vector f (times gf^T)
// to the D+1 vertex gradients: out[j+1] = Q Dm^-T column j + f gf[j]; out[0] = -sum.
template <int D, typename T>
__device__ __forceinline__ void to_vertices(const T Q[D][D], const T f[D], const ElemRest<D, T>& R, T out[D + 1][D]) {
#pragma unroll
  for (int r = 0; r < D; ++r) out[0][r] = T(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
#pragma unroll
    for (int r = 0; r < D; ++r) {
      T acc = f[r] * R.gf[j];
#pragma unroll
      for (int c = 0; c < D; ++c) acc += Q[r][c] * R.Dinv[j][c];
      out[j + 1][r] = acc;
      out[0][r] -= acc;
    }
  }
}

// gradient of W psi w.r.t. the D+1 vertex positions
template <int D, typename T>
__device__ __forceinline__ void elem_grad(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a, T out[D + 1][D]) {
  const T cnh = (R.wlam * S.l - R.wmu) * S.dl;
  T Q[D][D], f[D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) Q[r][c] = R.wmu * S.F[r][c] + cnh * S.C[r][c];
  const T cf = (R.wkf / a) * (S.s / a - T(1));
#pragma unroll
  for (int r = 0; r < D; ++r) f[r] = cf * S.n[r];
  to_vertices<D, T>(Q, f, R, out);
}

// Hessian of W psi applied to the vertex displacement whose edge matrix is dDs
template <int D, typename T>
__device__ __forceinline__ void elem_hessvec(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a,
                                             const T dDs[D][D], T out[D + 1][D]) {
  T dF[D][D], dC[D][D], Q[D][D], f[D], q[D];
  mul_dinv<D, T>(dDs, R.Dinv, dF);
  cofactor_diff<D, T>(S.F, dF, dC);
  T CdF = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) CdF += S.C[r][c] * dF[r][c];
  const T c1 = (R.wlam * S.l - R.wmu) * S.dl;
  const T c2 = (R.wlam * S.dl * S.dl - (R.wlam * S.l - R.wmu)) * CdF;  // l'' = -1
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) Q[r][c] = R.wmu * dF[r][c] + c1 * dC[r][c] + c2 * S.C[r][c];
  T nq = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < D; ++j) acc += dDs[r][j] * R.gf[j];
    q[r] = acc;
    nq += S.n[r] * acc;
  }
  const T ia = T(1) / a;
  const T k1 = R.wkf * ia * ia * nq;
  const T k2 = R.wkf * ia * (S.s * ia - T(1)) * S.sinv;
#pragma unroll
  for (int r = 0; r < D; ++r) f[r] = k1 * S.n[r] + k2 * (q[r] - S.n[r] * nq);
  to_vertices<D, T>(Q, f, R, out);
}

// diagonal of the element Hessian of W psi, per vertex and axis
template <int D, typename T>
__device__ __forceinline__ void elem_hessdiag(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a, T out[D + 1][D]) {
  // a unit displacement of vertex i along axis c gives the rank-one dF = e_c b_i^T, for which
  // dcof(dF) : dF vanishes; b_i is row i-1 of Dm^-1 (minus their sum for vertex 0).
  const T c2 = R.wlam * S.dl * S.dl - (R.wlam * S.l - R.wmu);
  const T ia = T(1) / a;
  const T k1 = R.wkf * ia * ia;
  const T k2 = R.wkf * ia * (S.s * ia - T(1)) * S.sinv;
#pragma unroll
  for (int i = 0; i <= D; ++i) {
    T b[D], gi = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) b[c] = T(0);
    if (i == 0) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
#pragma unroll
        for (int c = 0; c < D; ++c) b[c] -= R.Dinv[j][c];
        gi -= R.gf[j];
      }
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) b[c] = R.Dinv[i - 1][c];
      gi = R.gf[i - 1];
    }
    T bb = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) bb += b[c] * b[c];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T cb = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) cb += S.C[c][k] * b[k];
      const T nc2 = S.n[c] * S.n[c];
      out[i][c] = R.wmu * bb + c2 * cb * cb + gi * gi * (k1 * nc2 + k2 * (T(1) - nc2));
    }
  }
}

// Hessian of W psi of a triangle with respect to its edge matrix Ds, K[q][q'] with q = j*2 + r for
// Ds[r][j], in closed form (the second derivative of Eq. 3 and Eq. 2 through F = Ds Dm^-1):
//   K[(r,j),(r',j')] = [r == r'] (W mu M[j][j'] + k2 gf[j] gf[j'])
//                    + [r != r'] c1 det(Dm^-1) s_r e(j,j')          (the cofactor term)
//                    + c2 g[r][j] g[r'][j']                          (the log term, rank one)
//                    + (k1 - k2) gf[j] gf[j'] n[r] n[r']             (the fibre's stretch direction)
// with M = Dm^-1 Dm^-T, g = cof F Dm^-T, s_0 = 1, s_1 = -1, e(0,1) = 1, e(1,0) = -1, e(j,j) = 0,
// c1 = (W lam l - W mu) l', c2 = W lam l'^2 - (W lam l - W mu) (l'' = -1), k1 = W k_f / a^2 and
// k2 = (W k_f / a)(s/a - 1)/s: the same terms elem_hessvec applies to a direction.
template <typename T>
__device__ __forceinline__ void edge_hessian_2d(const ElemRest<2, T>& R, const ElemState<2, T>& S, T a,
                                                T K[4][4]) {
  const T c1 = (R.wlam * S.l - R.wmu) * S.dl;
  const T c2 = R.wlam * S.dl * S.dl - (R.wlam * S.l - R.wmu);
  const T ia = T(1) / a;
  const T k1 = R.wkf * ia * ia;
  const T k2 = R.wkf * ia * (S.s * ia - T(1)) * S.sinv;
  const T detDinv = R.Dinv[0][0] * R.Dinv[1][1] - R.Dinv[0][1] * R.Dinv[1][0];
  T M[2][2], g[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      M[j][k] = R.Dinv[j][0] * R.Dinv[k][0] + R.Dinv[j][1] * R.Dinv[k][1];
      g[j][k] = S.C[j][0] * R.Dinv[k][0] + S.C[j][1] * R.Dinv[k][1];  // g[r][j]
    }
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
          const T ff = R.gf[j] * R.gf[jj];
          T v = c2 * g[r][j] * g[rr][jj] + (k1 - k2) * ff * S.n[r] * S.n[rr];
          if (r == rr)
            v += R.wmu * M[j][jj] + k2 * ff;
          else if (j != jj)
            v += c1 * detDinv * T(r == 0 ? 1 : -1) * T(j == 0 ? 1 : -1);
          K[j * 2 + r][jj * 2 + rr] = v;
        }
}

// Cotangents -w^T dG/dtheta of one element (G = d(W psi)/dx), before the s_pot scale:
// returns {a_bar, mu_bar, lam_bar, kf_bar} for the edge matrix dWs of the adjoint vector w.
template <int D, typename T>
__device__ __forceinline__ void elem_vjp(const ElemRest<D, T>& R, const ElemState<D, T>& S, T W, T a,
                                         const T dWs[D][D], T out[4]) {
  T dF[D][D];
  mul_dinv<D, T>(dWs, R.Dinv, dF);
  T FmC = T(0), CdF = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      FmC += (S.F[r][c] - S.dl * S.C[r][c]) * dF[r][c];
      CdF += S.C[r][c] * dF[r][c];
    }
  T nq = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < D; ++j) acc += dWs[r][j] * R.gf[j];
    nq += S.n[r] * acc;
  }
  const T ia = T(1) / a;
  out[0] = -R.wkf * (ia * ia - T(2) * S.s * ia * ia * ia) * nq;
  out[1] = -W * FmC;
  out[2] = -W * S.l * S.dl * CdF;
  out[3] = -W * ia * (S.s * ia - T(1)) * nq;
}

}  // namespace isb
