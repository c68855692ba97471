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
//
// The isotropic part may instead be one of the other models Sec. 3 names (template parameter EM;
// the fibre term is the same in all), each linear in the Lame pair:
//   EM_STVK   St. Venant-Kirchhoff, E = (F^T F - I)/2: mu E:E + lam/2 tr(E)^2
//   EM_COROT  corotated, F = R S with R the closest rotation to F: mu |F - R|^2 + lam/2 tr(S - I)^2
//   EM_SNH    stable neo-Hookean without its log barrier, Lame pair reparametrised and shifted to
//             zero rest energy: mu/2 (I1 - D) - mu (J - 1) + (lam + mu)/2 (J - 1)^2
#pragma once

#include <hip/hip_runtime.h>

namespace isb {

// isotropic energy models (ISB_ENERGY_* of the C ABI)
constexpr int EM_NH = 0, EM_STVK = 1, EM_COROT = 2, EM_SNH = 3;

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

// ---------------------------------------------------------------------------------------------
// the alternative isotropic models (EM != EM_NH)
// ---------------------------------------------------------------------------------------------
// Per-element values the alternative models derive from F once: for the corotated model the
// closest rotation R, S = R^T F (symmetrised), tr S and, in 3D, (tr S I - S)^-1, from which dR
// along dF follows (F = R S, dR = R Omega with Omega S + S Omega = R^T dF - dF^T R).
template <int D, typename T>
struct IsoPre {
  T R[D][D], Sm[D][D], Minv[D][D];
  T trS;
};

// largest-eigenvalue eigenvector of a symmetric 4x4 matrix by cyclic Jacobi rotations
template <typename T>
__device__ __forceinline__ void top_eigvec4(T A[4][4], T q[4]) {
  T V[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) V[i][j] = T(i == j ? 1 : 0);
  for (int sweep = 0; sweep < 6; ++sweep) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int r = p + 1; r < 4; ++r) {
        const T apq = A[p][r];
        if (fabs(apq) <= T(1e-30) * (fabs(A[p][p]) + fabs(A[r][r])) || apq == T(0)) continue;
        const T th = (A[r][r] - A[p][p]) / (T(2) * apq);
        const T t = fabs(th) > T(1e15) ? T(0.5) / th : (th >= T(0) ? T(1) : T(-1)) / (fabs(th) + sqrt(th * th + T(1)));
        const T c = T(1) / sqrt(t * t + T(1)), sn = t * c;
        // A <- J^T A J with J the rotation in the (p, r) plane
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const T akp = A[k][p], akr = A[k][r];
          A[k][p] = c * akp - sn * akr;
          A[k][r] = sn * akp + c * akr;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const T apk = A[p][k], ark = A[r][k];
          A[p][k] = c * apk - sn * ark;
          A[r][k] = sn * apk + c * ark;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const T vkp = V[k][p], vkr = V[k][r];
          V[k][p] = c * vkp - sn * vkr;
          V[k][r] = sn * vkp + c * vkr;
        }
      }
  }
  int best = 0;
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (A[k][k] > A[best][best]) best = k;
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = V[k][best];
}

// R = argmax over rotations of tr(R^T F): in 2D the rotation by the angle of (F00 + F11, F10 - F01);
// in 3D the rotation of the unit quaternion that maximises q^T N(F) q (Horn's quadratic form of
// tr(R(q)^T F)), the top eigenvector of N
template <int D, typename T>
__device__ __forceinline__ void closest_rotation(const T F[D][D], T R[D][D]) {
  if constexpr (D == 2) {
    const T c0 = F[0][0] + F[1][1], s0 = F[1][0] - F[0][1];
    const T r = sqrt(c0 * c0 + s0 * s0);
    const T c = r > T(0) ? c0 / r : T(1), sn = r > T(0) ? s0 / r : T(0);
    R[0][0] = c;
    R[0][1] = -sn;
    R[1][0] = sn;
    R[1][1] = c;
  } else {
    T N[4][4] = {{F[0][0] + F[1][1] + F[2][2], F[2][1] - F[1][2], F[0][2] - F[2][0], F[1][0] - F[0][1]},
                 {F[2][1] - F[1][2], F[0][0] - F[1][1] - F[2][2], F[0][1] + F[1][0], F[0][2] + F[2][0]},
                 {F[0][2] - F[2][0], F[0][1] + F[1][0], -F[0][0] + F[1][1] - F[2][2], F[1][2] + F[2][1]},
                 {F[1][0] - F[0][1], F[0][2] + F[2][0], F[1][2] + F[2][1], -F[0][0] - F[1][1] + F[2][2]}};
    T q[4];
    top_eigvec4<T>(N, q);
    const T qn = T(1) / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const T w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
    R[0][0] = w * w + x * x - y * y - z * z;
    R[0][1] = T(2) * (x * y - w * z);
    R[0][2] = T(2) * (x * z + w * y);
    R[1][0] = T(2) * (x * y + w * z);
    R[1][1] = w * w - x * x + y * y - z * z;
    R[1][2] = T(2) * (y * z - w * x);
    R[2][0] = T(2) * (x * z - w * y);
    R[2][1] = T(2) * (y * z + w * x);
    R[2][2] = w * w - x * x - y * y + z * z;
  }
}

// The corotated values are formed in FP64 from the element's F in every precision and rounded
// once: an FP32 eigen-solve and inverse would add their own errors to the rotation, which the
// products then amplify through the cancellation in F - R near rest.
template <int D, typename T, int EM>
__device__ __forceinline__ void iso_pre(const ElemState<D, T>& S, IsoPre<D, T>& P) {
  if constexpr (EM == EM_COROT) {
    double F[D][D], R[D][D], Sm[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) F[i][j] = double(S.F[i][j]);
    closest_rotation<D, double>(F, R);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) acc += R[k][i] * F[k][j];
        Sm[i][j] = acc;
      }
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) tr += Sm[i][i];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        P.R[i][j] = T(R[i][j]);
        P.Sm[i][j] = T(0.5 * (Sm[i][j] + Sm[j][i]));
      }
    P.trS = T(tr);
    if constexpr (D == 3) {
      double M[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[i][j] = (i == j ? tr : 0.0) - 0.5 * (Sm[i][j] + Sm[j][i]);
      double C[3][3];
      cofactor<3, double>(M, C);
      const double idet = 1.0 / (M[0][0] * C[0][0] + M[1][0] * C[1][0] + M[2][0] * C[2][0]);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P.Minv[i][j] = T(C[j][i] * idet);  // M^-1 = cof(M)^T / det M
    }
  }
}

// W psi_iso
template <int D, typename T, int EM>
__device__ __forceinline__ T iso_energy(const ElemRest<D, T>& R, const ElemState<D, T>& S, const IsoPre<D, T>& P) {
  if constexpr (EM == EM_STVK) {
    T E[D][D], ee = T(0), tr = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) acc += S.F[k][i] * S.F[k][j];
        E[i][j] = T(0.5) * (acc - (i == j ? T(1) : T(0)));
        ee += E[i][j] * E[i][j];
      }
#pragma unroll
    for (int i = 0; i < D; ++i) tr += E[i][i];
    return R.wmu * ee + T(0.5) * R.wlam * tr * tr;
  } else if constexpr (EM == EM_COROT) {
    T dd = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const T v = S.F[i][j] - P.R[i][j];
        dd += v * v;
      }
    const T t = P.trS - T(D);
    return R.wmu * dd + T(0.5) * R.wlam * t * t;
  } else {
    T I1 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) I1 += S.F[i][j] * S.F[i][j];
    const T j1 = S.J - T(1);
    return T(0.5) * R.wmu * (I1 - T(D)) - R.wmu * j1 + T(0.5) * (R.wlam + R.wmu) * j1 * j1;
  }
}

// Q = W P_iso(F)
template <int D, typename T, int EM>
__device__ __forceinline__ void iso_stress(const ElemRest<D, T>& R, const ElemState<D, T>& S, const IsoPre<D, T>& P,
                                           T Q[D][D]) {
  if constexpr (EM == EM_STVK) {
    T A[D][D], tr = T(0);  // A = 2 mu E + lam tr(E) I (W-scaled)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) acc += S.F[k][i] * S.F[k][j];
        A[i][j] = T(0.5) * (acc - (i == j ? T(1) : T(0)));
      }
#pragma unroll
    for (int i = 0; i < D; ++i) tr += A[i][i];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) A[i][j] = T(2) * R.wmu * A[i][j] + (i == j ? R.wlam * tr : T(0));
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) acc += S.F[i][k] * A[k][j];
        Q[i][j] = acc;
      }
  } else if constexpr (EM == EM_COROT) {
    const T lt = R.wlam * (P.trS - T(D));
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) Q[i][j] = T(2) * R.wmu * (S.F[i][j] - P.R[i][j]) + lt * P.R[i][j];
  } else {
    const T cj = (R.wlam + R.wmu) * (S.J - T(1)) - R.wmu;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) Q[i][j] = R.wmu * S.F[i][j] + cj * S.C[i][j];
  }
}

// dQ = W dP_iso(F; dF)
template <int D, typename T, int EM>
__device__ __forceinline__ void iso_dstress(const ElemRest<D, T>& R, const ElemState<D, T>& S, const IsoPre<D, T>& P,
                                            const T dF[D][D], T dQ[D][D]) {
  if constexpr (EM == EM_STVK) {
    T A[D][D], B[D][D], trE = T(0), trdE = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T ftf = T(0), d = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
          ftf += S.F[k][i] * S.F[k][j];
          d += dF[k][i] * S.F[k][j] + S.F[k][i] * dF[k][j];
        }
        A[i][j] = T(0.5) * (ftf - (i == j ? T(1) : T(0)));  // E
        B[i][j] = T(0.5) * d;                                // dE
      }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      trE += A[i][i];
      trdE += B[i][i];
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        A[i][j] = T(2) * R.wmu * A[i][j] + (i == j ? R.wlam * trE : T(0));
        B[i][j] = T(2) * R.wmu * B[i][j] + (i == j ? R.wlam * trdE : T(0));
      }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) acc += dF[i][k] * A[k][j] + S.F[i][k] * B[k][j];
        dQ[i][j] = acc;
      }
  } else if constexpr (EM == EM_COROT) {
    // K = R^T dF - dF^T R (skew); Omega from K; dR = R Omega; tr(dS) = R : dF
    T RtdF[D][D], trRdF = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) acc += P.R[k][i] * dF[k][j];
        RtdF[i][j] = acc;
      }
#pragma unroll
    for (int i = 0; i < D; ++i) trRdF += RtdF[i][i];
    T Om[D][D];
    if constexpr (D == 2) {
      const T om = (RtdF[1][0] - RtdF[0][1]) / P.trS;
      Om[0][0] = T(0);
      Om[1][1] = T(0);
      Om[1][0] = om;
      Om[0][1] = -om;
    } else {
      const T k[3] = {RtdF[2][1] - RtdF[1][2], RtdF[0][2] - RtdF[2][0], RtdF[1][0] - RtdF[0][1]};
      T w[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) w[i] = P.Minv[i][0] * k[0] + P.Minv[i][1] * k[1] + P.Minv[i][2] * k[2];
      Om[0][0] = Om[1][1] = Om[2][2] = T(0);
      Om[2][1] = w[0];
      Om[1][2] = -w[0];
      Om[0][2] = w[1];
      Om[2][0] = -w[1];
      Om[1][0] = w[2];
      Om[0][1] = -w[2];
    }
    const T lt = R.wlam * (P.trS - T(D)), lr = R.wlam * trRdF;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T dR = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) dR += P.R[i][k] * Om[k][j];
        dQ[i][j] = T(2) * R.wmu * (dF[i][j] - dR) + lr * P.R[i][j] + lt * dR;
      }
  } else {
    T dC[D][D], CdF = T(0);
    cofactor_diff<D, T>(S.F, dF, dC);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) CdF += S.C[i][j] * dF[i][j];
    const T lp = R.wlam + R.wmu;
    const T cj = lp * (S.J - T(1)) - R.wmu;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) dQ[i][j] = R.wmu * dF[i][j] + lp * CdF * S.C[i][j] + cj * dC[i][j];
  }
}

// (P_mu : dF, P_lam : dF) with P_iso = mu P_mu + lam P_lam (unscaled by W)
template <int D, typename T, int EM>
__device__ __forceinline__ void iso_param(const ElemState<D, T>& S, const IsoPre<D, T>& P, const T dF[D][D], T& pmu,
                                          T& plam) {
  pmu = T(0);
  plam = T(0);
  if constexpr (EM == EM_STVK) {
    T E[D][D], tr = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) acc += S.F[k][i] * S.F[k][j];
        E[i][j] = T(0.5) * (acc - (i == j ? T(1) : T(0)));
      }
#pragma unroll
    for (int i = 0; i < D; ++i) tr += E[i][i];
    // P_mu = 2 F E, P_lam = tr(E) F
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T fe = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) fe += S.F[i][k] * E[k][j];
        pmu += T(2) * fe * dF[i][j];
        plam += tr * S.F[i][j] * dF[i][j];
      }
  } else if constexpr (EM == EM_COROT) {
    // P_mu = 2 (F - R), P_lam = (tr S - D) R
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        pmu += T(2) * (S.F[i][j] - P.R[i][j]) * dF[i][j];
        plam += (P.trS - T(D)) * P.R[i][j] * dF[i][j];
      }
  } else {
    // P_mu = F + (J - 2) cof F, P_lam = (J - 1) cof F
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        pmu += (S.F[i][j] + (S.J - T(2)) * S.C[i][j]) * dF[i][j];
        plam += (S.J - T(1)) * S.C[i][j] * dF[i][j];
      }
  }
}

// W psi(F)
template <int D, typename T, int EM = EM_NH>
__device__ __forceinline__ T elem_energy(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a) {
  if constexpr (EM != EM_NH) {
    IsoPre<D, T> P;
    iso_pre<D, T, EM>(S, P);
    const T e = S.s / a - T(1);
    return iso_energy<D, T, EM>(R, S, P) + T(0.5) * R.wkf * e * e;
  }
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
template <int D, typename T, int EM = EM_NH>
__device__ __forceinline__ void elem_grad(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a, T out[D + 1][D]) {
  T Q[D][D], f[D];
  if constexpr (EM == EM_NH) {
    const T cnh = (R.wlam * S.l - R.wmu) * S.dl;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int c = 0; c < D; ++c) Q[r][c] = R.wmu * S.F[r][c] + cnh * S.C[r][c];
  } else {
    IsoPre<D, T> P;
    iso_pre<D, T, EM>(S, P);
    iso_stress<D, T, EM>(R, S, P, Q);
  }
  const T cf = (R.wkf / a) * (S.s / a - T(1));
#pragma unroll
  for (int r = 0; r < D; ++r) f[r] = cf * S.n[r];
  to_vertices<D, T>(Q, f, R, out);
}

// Hessian of W psi applied to the vertex displacement whose edge matrix is dDs
// the fibre part of the Hessian applied to dDs, as the vector f that to_vertices spreads by gf
template <int D, typename T>
__device__ __forceinline__ void fibre_hessvec(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a,
                                              const T dDs[D][D], T f[D]) {
  T q[D], nq = T(0);
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
}

// the Hessian of an alternative model applied to dDs, with the per-element values P precomputed
template <int D, typename T, int EM>
__device__ __forceinline__ void elem_hessvec_pre(const ElemRest<D, T>& R, const ElemState<D, T>& S,
                                                 const IsoPre<D, T>& P, T a, const T dDs[D][D], T out[D + 1][D]) {
  T dF[D][D], Q[D][D], f[D];
  mul_dinv<D, T>(dDs, R.Dinv, dF);
  iso_dstress<D, T, EM>(R, S, P, dF, Q);
  fibre_hessvec<D, T>(R, S, a, dDs, f);
  to_vertices<D, T>(Q, f, R, out);
}

template <int D, typename T, int EM = EM_NH>
__device__ __forceinline__ void elem_hessvec(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a,
                                             const T dDs[D][D], T out[D + 1][D]) {
  if constexpr (EM != EM_NH) {
    IsoPre<D, T> P;
    iso_pre<D, T, EM>(S, P);
    elem_hessvec_pre<D, T, EM>(R, S, P, a, dDs, out);
    return;
  }
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
template <int D, typename T, int EM = EM_NH>
__device__ __forceinline__ void elem_hessdiag(const ElemRest<D, T>& R, const ElemState<D, T>& S, T a, T out[D + 1][D]) {
  if constexpr (EM != EM_NH) {
    // one product per vertex and axis: the displacement e_c at vertex i has the edge matrix
    // e_c e_{i-1}^T (i >= 1) or -e_c 1^T (i = 0); the diagonal entry is the product's (i, c) entry
    IsoPre<D, T> P;
    iso_pre<D, T, EM>(S, P);
#pragma unroll
    for (int i = 0; i <= D; ++i)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        T dDs[D][D], o[D + 1][D];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
          for (int j = 0; j < D; ++j) dDs[r][j] = (r == c && (i == 0 || j == i - 1)) ? T(i == 0 ? -1 : 1) : T(0);
        elem_hessvec_pre<D, T, EM>(R, S, P, a, dDs, o);
        out[i][c] = o[i][c];
      }
    return;
  }
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
template <typename T, int EM = EM_NH>
__device__ __forceinline__ void edge_hessian_2d(const ElemRest<2, T>& R, const ElemState<2, T>& S, T a,
                                                T K[4][4]) {
  if constexpr (EM != EM_NH) {
    // column q = j*2 + r is the product with the unit edge displacement Ds[r][j] = 1; its entries
    // for vertices 1 and 2 are the edge-matrix gradient
    IsoPre<2, T> P;
    iso_pre<2, T, EM>(S, P);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        T dDs[2][2] = {{T(0), T(0)}, {T(0), T(0)}}, o[3][2];
        dDs[r][j] = T(1);
        elem_hessvec_pre<2, T, EM>(R, S, P, a, dDs, o);
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int rr = 0; rr < 2; ++rr) K[jj * 2 + rr][j * 2 + r] = o[jj + 1][rr];
      }
    return;
  }
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
template <int D, typename T, int EM = EM_NH>
__device__ __forceinline__ void elem_vjp(const ElemRest<D, T>& R, const ElemState<D, T>& S, T W, T a,
                                         const T dWs[D][D], T out[4]) {
  T dF[D][D];
  mul_dinv<D, T>(dWs, R.Dinv, dF);
  T FmC = T(0), CdF = T(0);  // P_mu : dF and P_lam : dF
  if constexpr (EM == EM_NH) {
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        FmC += (S.F[r][c] - S.dl * S.C[r][c]) * dF[r][c];
        CdF += S.C[r][c] * dF[r][c];
      }
    CdF *= S.l * S.dl;
  } else {
    IsoPre<D, T> P;
    iso_pre<D, T, EM>(S, P);
    iso_param<D, T, EM>(S, P, dF, FmC, CdF);
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
  out[2] = -W * CdF;
  out[3] = -W * ia * (S.s * ia - T(1)) * nq;
}

}  // namespace isb
