"""FP64 reference energies and derivatives (test infrastructure only).

Everything is written out from the definitions in the paper, vectorised over
elements with NumPy. The Hessian is assembled explicitly (no matrix-free
products), so this module shares no algorithm with the GPU path.

  * Element energy: neo-Hookean density (Sec. 3, Eq. 3) with the quadratic
    stand-in for log J that the paper uses for inverted elements, plus the
    contractile fibre term (Eq. 2) written per element along a material
    direction; F is linear in x (Sec. 3).
  * Spring energy: Eq. 2 as a literal spring between two vertices i, j with
    l(x) = |x_j - x_i|, rest length l0 = |X_j - X_i| and its own action (Fig. 2's
    reading of energies of d = x_j - x_i).
  * Vertex energies: ground contact (Sec. 5.2, Eq. 15), friction through the
    velocity v(x) = (x - x0)/h (Eq. 16-17), gravity.
  * Objectives: quasistatic E (Eq. 1) and backward Euler
    1/2 |x - (x0 + h v0)|_M^2 + h^2 E (Eq. 14).

Readings where the paper is silent:
  log J is replaced by l(J) = (J-1) - (J-1)^2/2 for every J; I1 - d in 3D;
  one fibre per element with l/l0 = |F d|; lumped mass rho W / (d+1) per corner;
  contact has no 1/2 and an indicator [y < 0]; friction factor
  ReLU(-y0 + eps) on the tangential components; gravity lives inside E;
  a spring's energy is k/2 (l/(a l0) - 1)^2 with no volume weight, and the action
  vector lists the elements' actions first and then the springs'.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------------------------
# geometry (Sec. 3: F is a linear function of x)
# --------------------------------------------------------------------------------------------
def edge_matrix(x: np.ndarray, T: np.ndarray) -> np.ndarray:
    """D[e] = [x_{T[e,1]} - x_{T[e,0]}, ..., x_{T[e,d]} - x_{T[e,0]}] as columns, [n_e, d, d]."""
    e = x[T[:, 1:]] - x[T[:, :1]]          # [n_e, d (edge), d (coord)]
    return np.swapaxes(e, 1, 2)


def det(F: np.ndarray) -> np.ndarray:
    d = F.shape[-1]
    if d == 2:
        return F[..., 0, 0] * F[..., 1, 1] - F[..., 0, 1] * F[..., 1, 0]
    return np.linalg.det(F)


def cofactor(F: np.ndarray) -> np.ndarray:
    """cof F = dJ/dF (= J F^-T when F is invertible)."""
    d = F.shape[-1]
    C = np.empty_like(F)
    if d == 2:
        C[..., 0, 0] = F[..., 1, 1]
        C[..., 0, 1] = -F[..., 1, 0]
        C[..., 1, 0] = -F[..., 0, 1]
        C[..., 1, 1] = F[..., 0, 0]
        return C
    c0, c1, c2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    C[..., :, 0] = np.cross(c1, c2)
    C[..., :, 1] = np.cross(c2, c0)
    C[..., :, 2] = np.cross(c0, c1)
    return C


def cofactor_diff(F: np.ndarray, dF: np.ndarray) -> np.ndarray:
    """Directional derivative of cof F along dF."""
    d = F.shape[-1]
    if d == 2:
        return cofactor(dF)
    C = np.empty_like(F)
    f = [F[..., :, k] for k in range(3)]
    g = [dF[..., :, k] for k in range(3)]
    for k in range(3):
        i, j = (k + 1) % 3, (k + 2) % 3
        C[..., :, k] = np.cross(g[i], f[j]) + np.cross(f[i], g[j])
    return C


class Mesh:
    """Rest-shape quantities of a simplicial mesh (Sec. 3; lumped M of Eq. 14)."""

    def __init__(self, X, T, rho):
        self.X = np.asarray(X, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        self.n_v, self.d = self.X.shape
        self.n_e = self.T.shape[0]
        Dm = edge_matrix(self.X, self.T)
        self.W = det(Dm) / math.factorial(self.d)
        if np.any(self.W <= 0):
            raise ValueError("non-positive rest volume")
        self.DmInv = np.linalg.inv(Dm)
        self.mass = np.zeros(self.n_v)
        np.add.at(self.mass, self.T, (np.asarray(rho, dtype=np.float64) * self.W / (self.d + 1))[:, None])

    def F(self, x):
        return edge_matrix(x, self.T) @ self.DmInv


# --------------------------------------------------------------------------------------------
# element energy density and its first and second derivatives (Eq. 2, Eq. 3)
# --------------------------------------------------------------------------------------------
def logq(J):
    """Quadratic replacement of log J about J = 1 (finite for J <= 0)."""
    return (J - 1.0) - 0.5 * (J - 1.0) ** 2


def logq_d(J):
    return 2.0 - J


LOGQ_DD = -1.0


# Isotropic element energies (the neo-Hookean density of Eq. 3 and the alternatives Sec. 3 names;
# all are functions of F alone) and the fibre term of Eq. 2 along a material direction.
MODELS = ("nh", "stvk", "corot", "snh")


def closest_rotation(F):
    """R = argmax over rotations of tr(R^T F): U V^T from the SVD F = U S V^T, with the sign of the
    last singular vector flipped when det(U V^T) < 0, so that det R = 1 also for inverted F."""
    U, _, Vt = np.linalg.svd(F)
    flip = np.where(det(U @ Vt) < 0.0, -1.0, 1.0)
    U = U.copy()
    U[..., :, -1] *= flip[..., None]
    return U @ Vt


def _corot_dR(R, S, dF):
    """dR = R Omega for the polar pair F = R S (S symmetric): Omega is skew with
    Omega S + S Omega = R^T dF - dF^T R."""
    d = R.shape[-1]
    K = np.swapaxes(R, -1, -2) @ dF
    K = K - np.swapaxes(K, -1, -2)
    trS = np.trace(S, axis1=-2, axis2=-1)
    if d == 2:
        om = K[:, 1, 0] / trS
        Om = np.zeros_like(R)
        Om[:, 1, 0] = om
        Om[:, 0, 1] = -om
    else:
        # Omega = skew(w), Omega S + S Omega = skew((tr S I - S) w)
        k = np.stack([K[:, 2, 1], K[:, 0, 2], K[:, 1, 0]], axis=-1)
        w = np.linalg.solve(trS[:, None, None] * np.eye(3)[None] - S, k[..., None])[..., 0]
        Om = np.zeros_like(R)
        Om[:, 2, 1], Om[:, 1, 2] = w[:, 0], -w[:, 0]
        Om[:, 0, 2], Om[:, 2, 0] = w[:, 1], -w[:, 1]
        Om[:, 1, 0], Om[:, 0, 1] = w[:, 2], -w[:, 2]
    return R @ Om


def _polar(F):
    R = closest_rotation(F)
    S = np.swapaxes(R, -1, -2) @ F
    return R, 0.5 * (S + np.swapaxes(S, -1, -2))


def iso_param_parts(F, model="nh"):
    """(psi_mu, psi_lam, P_mu, P_lam): the isotropic density and its first Piola stress are
    mu psi_mu + lam psi_lam and mu P_mu + lam P_lam in every model (both linear in the Lame pair).

      nh    Eq. 3 with log J replaced by l(J) = (J-1) - (J-1)^2/2:
            mu/2 (I1 - d) - mu l(J) + lam/2 l(J)^2
      stvk  St. Venant-Kirchhoff, E = (F^T F - I)/2:  mu E:E + lam/2 tr(E)^2
      corot corotated, F = R S with R the closest rotation:  mu |F - R|^2 + lam/2 tr(S - I)^2
      snh   stable neo-Hookean without its log barrier, Lame pair reparametrised (lam -> lam + mu,
            rest stress zero) and shifted to zero rest energy:
            mu/2 (I1 - d) - mu (J - 1) + (lam + mu)/2 (J - 1)^2
    """
    d = F.shape[-1]
    eye = np.eye(d)[None]
    if model == "nh":
        J = det(F)
        lJ, dl = logq(J), logq_d(J)
        C = cofactor(F)
        I1 = np.sum(F * F, axis=(-2, -1))
        return (0.5 * (I1 - d) - lJ, 0.5 * lJ ** 2, F - dl[:, None, None] * C, (lJ * dl)[:, None, None] * C)
    if model == "stvk":
        E = 0.5 * (np.swapaxes(F, -1, -2) @ F - eye)
        trE = np.trace(E, axis1=-2, axis2=-1)
        return np.sum(E * E, axis=(-2, -1)), 0.5 * trE ** 2, 2.0 * F @ E, trE[:, None, None] * F
    if model == "corot":
        R, S = _polar(F)
        t = np.trace(S, axis1=-2, axis2=-1) - d
        return np.sum((F - R) ** 2, axis=(-2, -1)), 0.5 * t ** 2, 2.0 * (F - R), t[:, None, None] * R
    if model == "snh":
        J = det(F)
        C = cofactor(F)
        I1 = np.sum(F * F, axis=(-2, -1))
        j1 = J - 1.0
        return (0.5 * (I1 - d) - j1 + 0.5 * j1 ** 2, 0.5 * j1 ** 2, F + (j1 - 1.0)[:, None, None] * C,
                j1[:, None, None] * C)
    raise ValueError(f"unknown energy model {model!r}")


def iso_stress_diff(F, dF, mu, lam, model="nh"):
    """d(P_iso) along dF."""
    mu3, lam3 = mu[:, None, None], lam[:, None, None]
    if model == "nh":
        J = det(F)
        lJ, dl = logq(J), logq_d(J)
        C = cofactor(F)
        dJ = np.sum(C * dF, axis=(-2, -1))
        dP = mu3 * dF
        dP += ((lam * lJ - mu) * dl)[:, None, None] * cofactor_diff(F, dF)
        dP += ((lam * dl * dl + (lam * lJ - mu) * LOGQ_DD) * dJ)[:, None, None] * C
        return dP
    if model == "stvk":
        d = F.shape[-1]
        E = 0.5 * (np.swapaxes(F, -1, -2) @ F - np.eye(d)[None])
        dE = 0.5 * (np.swapaxes(dF, -1, -2) @ F + np.swapaxes(F, -1, -2) @ dF)
        trE = np.trace(E, axis1=-2, axis2=-1)[:, None, None]
        trdE = np.trace(dE, axis1=-2, axis2=-1)[:, None, None]
        return dF @ (2.0 * mu3 * E) + lam3 * trE * dF + F @ (2.0 * mu3 * dE) + lam3 * trdE * F
    if model == "corot":
        d = F.shape[-1]
        R, S = _polar(F)
        dR = _corot_dR(R, S, dF)
        t = (np.trace(S, axis1=-2, axis2=-1) - d)[:, None, None]
        trRdF = np.sum(R * dF, axis=(-2, -1))[:, None, None]     # tr(dS) = tr(R^T dF)
        return 2.0 * mu3 * (dF - dR) + lam3 * trRdF * R + lam3 * t * dR
    if model == "snh":
        J = det(F)
        C = cofactor(F)
        dJ = np.sum(C * dF, axis=(-2, -1))
        lp = lam + mu
        dP = mu3 * dF + (lp * dJ)[:, None, None] * C
        dP += (lp * (J - 1.0) - mu)[:, None, None] * cofactor_diff(F, dF)
        return dP
    raise ValueError(f"unknown energy model {model!r}")


def fibre_terms(F, fd):
    """(s, n): fibre stretch |F d| and unit direction F d / s."""
    Ffd = np.einsum("eij,ej->ei", F, fd)
    s = np.linalg.norm(Ffd, axis=-1)
    return s, Ffd / s[:, None]


def psi(F, mu, lam, kf, a, fd, model="nh"):
    """Energy density: the isotropic model's density plus kf/2 (|F fd| / a - 1)^2 (Eq. 2)."""
    pm, pl, _, _ = iso_param_parts(F, model)
    s, _ = fibre_terms(F, fd)
    return mu * pm + lam * pl + 0.5 * kf * (s / a - 1.0) ** 2


def stress(F, mu, lam, kf, a, fd, model="nh"):
    """First Piola stress P = d psi / dF."""
    _, _, Pm, Pl = iso_param_parts(F, model)
    P = mu[:, None, None] * Pm + lam[:, None, None] * Pl
    s, n = fibre_terms(F, fd)
    P += ((kf / a) * (s / a - 1.0))[:, None, None] * np.einsum("ei,ej->eij", n, fd)
    return P


def stress_diff(F, dF, mu, lam, kf, a, fd, model="nh"):
    """dP = (d^2 psi / dF^2) : dF."""
    dP = iso_stress_diff(F, dF, mu, lam, model)
    s, n = fibre_terms(F, fd)
    q = np.einsum("eij,ej->ei", dF, fd)                   # dF fd
    nq = np.sum(n * q, axis=-1)
    dn = (q - n * nq[:, None]) / s[:, None]               # d(n) = (I - n n^T) dF fd / s
    dP += ((kf / (a * a)) * nq)[:, None, None] * np.einsum("ei,ej->eij", n, fd)
    dP += ((kf / a) * (s / a - 1.0))[:, None, None] * np.einsum("ei,ej->eij", dn, fd)
    return dP


# --------------------------------------------------------------------------------------------
# per-element vertex gradients and Hessian blocks
# --------------------------------------------------------------------------------------------
def corner_grads(mesh: Mesh, G):
    """Map a per-element dE/dF-shaped quantity G [n_e, d, d] to per-corner gradients.

    E_e depends on x through F = D_s(x) Dm^-1, so dE_e/dD_s = W G Dm^-T; column j of it is the
    gradient at corner j+1 and corner 0 takes minus their sum. Returns [n_e, d+1, d].
    """
    H = mesh.W[:, None, None] * (G @ np.swapaxes(mesh.DmInv, 1, 2))
    out = np.empty((mesh.n_e, mesh.d + 1, mesh.d))
    out[:, 1:, :] = np.swapaxes(H, 1, 2)
    out[:, 0, :] = -out[:, 1:, :].sum(axis=1)
    return out


def corner_dF(mesh: Mesh, j: int, c: int):
    """dF of every element for a unit displacement of its corner j along axis c."""
    dDs = np.zeros((mesh.n_e, mesh.d, mesh.d))
    if j == 0:
        dDs[:, c, :] = -1.0
    else:
        dDs[:, c, j - 1] = 1.0
    return dDs @ mesh.DmInv


def element_hessians(mesh: Mesh, x, mu, lam, kf, a, fd, model="nh"):
    """Dense element Hessians [n_e, (d+1)d, (d+1)d] of E_e = W psi(F), row/col index = corner*d + axis."""
    F = mesh.F(x)
    nd = (mesh.d + 1) * mesh.d
    K = np.empty((mesh.n_e, nd, nd))
    for j in range(mesh.d + 1):
        for c in range(mesh.d):
            dP = stress_diff(F, corner_dF(mesh, j, c), mu, lam, kf, a, fd, model)
            K[:, :, j * mesh.d + c] = corner_grads(mesh, dP).reshape(mesh.n_e, nd)
    return K


# --------------------------------------------------------------------------------------------
# vertex-pair springs (Eq. 2 with d = x_j - x_i; Fig. 2)
# --------------------------------------------------------------------------------------------
def spring_energy(x, S, k, l0, a):
    """k/2 (l/(a l0) - 1)^2 per spring, l = |x_j - x_i| for the pair (i, j) = S[s]."""
    l = np.linalg.norm(x[S[:, 1]] - x[S[:, 0]], axis=-1)
    return 0.5 * k * (l / (a * l0) - 1.0) ** 2


def spring_force_terms(x, S, k, l0, a):
    """(n, l, c, f) with n = d/l the spring's unit direction, c = 1/(a l0) and f = dE/dl = k c (c l - 1)."""
    dvec = x[S[:, 1]] - x[S[:, 0]]
    l = np.linalg.norm(dvec, axis=-1)
    n = dvec / l[:, None]
    c = 1.0 / (a * l0)
    return n, l, c, k * c * (c * l - 1.0)


def spring_grad(x, S, k, l0, a):
    """Assembled gradient of the springs' energy [n_v, d]: +f n at j, -f n at i."""
    n, _, _, f = spring_force_terms(x, S, k, l0, a)
    G = np.zeros_like(x)
    np.add.at(G, S[:, 1], f[:, None] * n)
    np.add.at(G, S[:, 0], -f[:, None] * n)
    return G


def spring_hessians(x, S, k, l0, a):
    """Dense spring Hessians [n_s, 2d, 2d], row/col index = end*d + axis with end 0 = i, 1 = j.

    With K = d^2E/dd^2 = k c^2 n n^T + (f / l)(I - n n^T), the blocks are [[K, -K], [-K, K]]."""
    n, l, c, f = spring_force_terms(x, S, k, l0, a)
    d = x.shape[1]
    nn = np.einsum("si,sj->sij", n, n)
    K = (k * c * c)[:, None, None] * nn + (f / l)[:, None, None] * (np.eye(d)[None] - nn)
    out = np.empty((S.shape[0], 2 * d, 2 * d))
    out[:, :d, :d] = K
    out[:, d:, d:] = K
    out[:, :d, d:] = -K
    out[:, d:, :d] = -K
    return out


# --------------------------------------------------------------------------------------------
# the step objective g(x) (Eq. 1 quasistatic, Eq. 14 backward Euler) and its derivatives
# --------------------------------------------------------------------------------------------
class Problem:
    """One body: mesh, material, scene constants. All arrays FP64; x is [n_v, d]."""

    def __init__(self, X, T, pinned, mu, lam, kf, fdir, rho, scene, springs=None, k_spring=None, model="nh"):
        self.mesh = Mesh(X, T, rho)
        if model not in MODELS:
            raise ValueError(f"unknown energy model {model!r}")
        self.model = model
        # vertex-pair springs (i, j) with stiffness k and rest length |X_j - X_i|
        self.S = np.zeros((0, 2), np.int64) if springs is None else np.asarray(springs, dtype=np.int64)
        self.ks = np.zeros(0) if k_spring is None else np.asarray(k_spring, dtype=np.float64)
        self.n_s = self.S.shape[0]
        if self.ks.shape != (self.n_s,):
            raise ValueError("one stiffness per spring")
        self.l0 = np.linalg.norm(self.mesh.X[self.S[:, 1]] - self.mesh.X[self.S[:, 0]], axis=-1)
        if np.any(self.l0 <= 0):
            raise ValueError("a spring with zero rest length")
        self.pinned = np.asarray(pinned, dtype=bool)
        self.free = ~self.pinned.ravel()
        self.mu = np.asarray(mu, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.kf = np.asarray(kf, dtype=np.float64)
        self.fd = np.asarray(fdir, dtype=np.float64)
        self.sc = dict(scene)
        self.be = self.sc["integrator"] == "be"
        self.h = float(self.sc["h"])
        # the potential energy is scaled by h^2 in the backward-Euler objective (Eq. 14)
        self.s_pot = self.h ** 2 if self.be else 1.0

    @classmethod
    def from_workload(cls, w):
        return cls(w.X, w.T, w.pinned, w.mu, w.lam, w.kf, w.fdir, w.rho, w.scene,
                   getattr(w, "S", None), getattr(w, "ks", None), getattr(w, "model", "nh"))

    def split(self, a):
        """(element actions [n_e], spring actions [n_s]) of an action vector [n_e + n_s]."""
        a = np.asarray(a, dtype=np.float64)
        if a.shape != (self.mesh.n_e + self.n_s,):
            raise ValueError("the action vector has one entry per element and then one per spring")
        return a[:self.mesh.n_e], a[self.mesh.n_e:]

    # ---- vertex terms (Eq. 15-17 and gravity) ----
    def friction_factor(self, x0):
        return np.maximum(-x0[:, 1] + self.sc["eps_friction"], 0.0)

    def tangential(self):
        return [0] if self.mesh.d == 2 else [0, 2]

    def vertex_energy(self, x, x0):
        """Per-vertex potential energy [n_v] (gravity + contact + friction)."""
        m, g = self.mesh.mass, self.sc["gravity"]
        y = x[:, 1]
        e = m * g * y + self.sc["k_contact"] * np.maximum(-y, 0.0) ** 2
        if self.sc["k_friction"] != 0.0:
            cv = self.friction_factor(x0)
            vt = (x[:, self.tangential()] - x0[:, self.tangential()]) / self.h
            e = e + self.sc["k_friction"] * cv * np.sum(vt * vt, axis=1)
        return e

    def vertex_grad(self, x, x0):
        m, g = self.mesh.mass, self.sc["gravity"]
        G = np.zeros_like(x)
        G[:, 1] = m * g - 2.0 * self.sc["k_contact"] * np.maximum(-x[:, 1], 0.0)
        if self.sc["k_friction"] != 0.0:
            cv = self.friction_factor(x0)
            t = self.tangential()
            G[:, t] += (2.0 * self.sc["k_friction"] * cv / self.h ** 2)[:, None] * (x[:, t] - x0[:, t])
        return G

    def vertex_hess_diag(self, x, x0):
        Hd = np.zeros_like(x)
        Hd[:, 1] = 2.0 * self.sc["k_contact"] * (x[:, 1] < 0.0)
        if self.sc["k_friction"] != 0.0:
            cv = self.friction_factor(x0)
            Hd[:, self.tangential()] += (2.0 * self.sc["k_friction"] * cv / self.h ** 2)[:, None]
        return Hd

    # ---- element terms ----
    def element_energy(self, x, a):
        F = self.mesh.F(x)
        return self.mesh.W * psi(F, self.mu, self.lam, self.kf, a, self.fd, self.model)

    def element_grad(self, x, a):
        """Assembled gradient of sum_e E_e, [n_v, d]."""
        F = self.mesh.F(x)
        cg = corner_grads(self.mesh, stress(F, self.mu, self.lam, self.kf, a, self.fd, self.model))
        G = np.zeros_like(x)
        np.add.at(G, self.mesh.T, cg)
        return G

    # ---- objective ----
    def x_hat(self, x0, v0):
        return x0 + self.h * v0 if self.be else x0

    def energy_terms(self, x, x0, v0, a):
        """(per-element terms then per-spring terms, per-vertex terms) of g; their total sum is g(x)."""
        ae, as_ = self.split(a)
        ee = self.s_pot * np.concatenate([self.element_energy(x, ae),
                                          spring_energy(x, self.S, self.ks, self.l0, as_)])
        ev = self.s_pot * self.vertex_energy(x, x0)
        if self.be:
            dx = x - self.x_hat(x0, v0)
            ev = ev + 0.5 * self.mesh.mass * np.sum(dx * dx, axis=1)
        return ee, ev

    def energy(self, x, x0, v0, a):
        ee, ev = self.energy_terms(x, x0, v0, a)
        return float(np.sum(ee) + np.sum(ev))

    def grad(self, x, x0, v0, a):
        """dg/dx [n_v, d]; pinned DOFs are not masked here."""
        ae, as_ = self.split(a)
        G = self.s_pot * (self.element_grad(x, ae) + spring_grad(x, self.S, self.ks, self.l0, as_)
                          + self.vertex_grad(x, x0))
        if self.be:
            G += self.mesh.mass[:, None] * (x - self.x_hat(x0, v0))
        return G

    def hessian(self, x, x0, a) -> sp.csr_matrix:
        """Assembled d^2 g / dx^2 over all n_v*d DOFs (row-major DOF = v*d + axis)."""
        d = self.mesh.d
        ae, as_ = self.split(a)
        n = self.mesh.n_v * d
        H = sp.csr_matrix((n, n))
        for K, conn in ((element_hessians(self.mesh, x, self.mu, self.lam, self.kf, ae, self.fd, self.model),
                         self.mesh.T),
                        (spring_hessians(x, self.S, self.ks, self.l0, as_), self.S)):
            dofs = (conn[:, :, None] * d + np.arange(d)[None, None, :]).reshape(conn.shape[0], conn.shape[1] * d)
            rows = np.repeat(dofs, dofs.shape[1], axis=1).ravel()
            cols = np.tile(dofs, (1, dofs.shape[1])).ravel()
            H = H + sp.coo_matrix(((self.s_pot * K).ravel(), (rows, cols)), shape=(n, n)).tocsr()
        diag = self.s_pot * self.vertex_hess_diag(x, x0)
        if self.be:
            diag = diag + self.mesh.mass[:, None]
        H = H + sp.diags(diag.ravel())
        return H.tocsr()
