"""FP64 reference step, adjoint and parameter VJP (test infrastructure only).

The step is the minimiser of the objective (Eq. 1 quasistatic, Eq. 13-14 backward
Euler). The paper leaves the forward solver free (Sec. 3 end, Sec. 6), so the
oracle takes the most plain route to it: Newton on the assembled sparse Hessian
with a direct (SuperLU) solve, shifted by a multiple of the identity when the
Hessian is not positive definite (Nocedal & Wright, Numerical Optimization,
Alg. 3.3), and an Armijo backtracking line search on element-wise energy
differences. It uses no CG and no matrix-free product.

The adjoint follows Eq. 9: with G = dg/dx and w = H(x1)^-1 xbar (H symmetric,
positive definite at a minimum, Sec. 4), dL/dtheta = -w^T dG/dtheta, solved with
the same direct factorisation. The velocity update v1 = (x1 - x0)/h of Eq. 14 is
differentiated by the chain rule (Fig. dynamics-cell), which adds vbar1/h to the
right-hand side and -vbar1/h to xbar0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Problem, edge_matrix, iso_param_parts, spring_force_terms

ARMIJO_C1 = 1e-4
LS_MAX = 30
EPS = np.finfo(np.float64).eps
# Above this many free DOFs the sparse direct factorisation of a 3D mesh fills in too much; the
# linear solves then use SciPy's conjugate gradient on the assembled matrix (a library routine,
# Jacobi-preconditioned, relative tolerance 1e-14) instead.
DIRECT_MAX_DOFS = 60000
ITER_RTOL = 1e-14


def _factor_pd(H: sp.csr_matrix):
    """LU of H with a symmetric permutation; returns (lu, is_pd) by Sylvester's inertia."""
    lu = spla.splu(H.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    symmetric_perm = np.array_equal(lu.perm_r, lu.perm_c)
    is_pd = symmetric_perm and bool(np.all(lu.U.diagonal() > 0))
    return lu, is_pd


def _cg_solve(A: sp.csr_matrix, rhs: np.ndarray):
    """SciPy CG on the assembled matrix with a Jacobi preconditioner; (x, ok) where ok means
    converged with positive curvature along the solution."""
    d = np.abs(A.diagonal())
    d[d == 0] = 1.0
    M = spla.LinearOperator(A.shape, matvec=lambda v: v / d, dtype=np.float64)
    x, info = spla.cg(A, rhs, rtol=ITER_RTOL, atol=0.0, maxiter=50000, M=M)
    ok = info == 0 and float(x @ (A @ x)) > 0.0
    return x, ok


def newton_direction(H: sp.csr_matrix, rhs: np.ndarray, direct_max: int | None = None):
    """Solve (H + tau I) dx = rhs with the smallest tau >= 0 of the doubling sequence that is PD."""
    direct_max = DIRECT_MAX_DOFS if direct_max is None else direct_max
    diag = H.diagonal()
    scale = np.mean(np.abs(diag))
    beta = 1e-3 * scale if scale > 0 else 1e-3
    tau = 0.0 if diag.min() > 0 else -diag.min() + beta
    n = H.shape[0]
    for _ in range(80):
        A = H if tau == 0.0 else (H + tau * sp.identity(n, format="csr"))
        if n <= direct_max:
            try:
                lu, ok = _factor_pd(A)
            except RuntimeError:
                ok = False
            if ok:
                return lu.solve(rhs), tau
        else:
            x, ok = _cg_solve(A.tocsr(), rhs)
            if ok:
                return x, tau
        tau = max(2.0 * tau, beta)
    raise RuntimeError("no positive-definite shift found")


def step(prob: Problem, x0, v0, a, tol=1e-13, max_iter=50, direct_max=None):
    """One implicit step: x1 = argmin g(x; x0, v0, a); v1 = (x1 - x0)/h in backward Euler.

    Stops at |G_free| <= tol |G_free(x_init)|, or when the line search can no longer make
    progress (rounding floor), or after max_iter Newton iterations. Returns (x1, v1, stats).
    """
    x0 = np.asarray(x0, dtype=np.float64)
    v0 = np.zeros_like(x0) if v0 is None else np.asarray(v0, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    free = prob.free
    x = prob.x_hat(x0, v0).copy()
    x[prob.pinned] = x0[prob.pinned]

    def grad_free(xx):
        return prob.grad(xx, x0, v0, a).ravel()[free]

    G = grad_free(x)
    res0 = float(np.linalg.norm(G))
    stats = dict(newton_iters=0, res0=res0, res_final=res0, ls_backtracks=0, shifts=0,
                 stagnated=False, converged=res0 == 0.0, res_hist=[res0])
    if res0 == 0.0:
        return x, _velocity(prob, x, x0), stats
    for _ in range(max_iter):
        res = float(np.linalg.norm(G))
        if res <= tol * res0:
            stats["converged"] = True
            break
        H = prob.hessian(x, x0, a)[free][:, free]
        dx, tau = newton_direction(H, -G, direct_max)
        stats["shifts"] += int(tau > 0)
        gTd = float(G @ dx)
        ee0, ev0 = prob.energy_terms(x, x0, v0, a)
        scale = float(np.sum(np.abs(ee0)) + np.sum(np.abs(ev0)))
        alpha, accepted, G_new = 1.0, False, None
        for _ls in range(LS_MAX):
            xt = x.copy()
            xt.reshape(-1)[free] += alpha * dx
            ee1, ev1 = prob.energy_terms(xt, x0, v0, a)
            dg = float(np.sum(ee1 - ee0) + np.sum(ev1 - ev0))
            if abs(dg) <= 1e3 * EPS * scale:
                # energy change below FP64 resolution, where the Armijo test only sees rounding:
                # accept only if |G| at least halves (a smaller decrease is noise; stagnation)
                Gt = grad_free(xt)
                if np.linalg.norm(Gt) <= 0.5 * res:
                    accepted, G_new = True, Gt
                else:
                    break                       # shorter steps cannot do better at the floor
            elif dg <= ARMIJO_C1 * alpha * gTd:
                accepted = True
            if accepted:
                break
            alpha *= 0.5
            stats["ls_backtracks"] += 1
        if not accepted:
            stats["stagnated"] = True
            break
        x = xt
        G = G_new if G_new is not None else grad_free(x)
        stats["newton_iters"] += 1
        stats["res_hist"].append(float(np.linalg.norm(G)))
    res_final = float(np.linalg.norm(G))
    stats["res_final"] = res_final
    stats["converged"] = stats["converged"] or res_final <= tol * res0
    return x, _velocity(prob, x, x0), stats


def _velocity(prob: Problem, x1, x0):
    return (x1 - x0) / prob.h if prob.be else None


def adjoint(prob: Problem, x1, x0, a, x1_bar, v1_bar=None, direct_max=None):
    """w = H(x1)^-1 (x1_bar + v1_bar/h) over the free DOFs; w = 0 on pinned DOFs (Eq. 9)."""
    direct_max = DIRECT_MAX_DOFS if direct_max is None else direct_max
    rhs = np.asarray(x1_bar, dtype=np.float64).copy()
    if prob.be and v1_bar is not None:
        rhs = rhs + np.asarray(v1_bar, dtype=np.float64) / prob.h
    free = prob.free
    H = prob.hessian(x1, x0, a)[free][:, free]
    w = np.zeros(prob.mesh.n_v * prob.mesh.d)
    if H.shape[0] <= direct_max:
        w[free] = spla.spsolve(H.tocsc(), rhs.ravel()[free])
    else:
        sol, ok = _cg_solve(H.tocsr(), rhs.ravel()[free])
        if not ok:
            raise RuntimeError("adjoint CG did not converge (Hessian not positive definite?)")
        w[free] = sol
    return w.reshape(x1.shape)


def vjp_params(prob: Problem, w, x1, x0, a, v1_bar=None):
    """Cotangents of (a, mu, lam, kf, k_spring, x0, v0) given the adjoint vector w (Eq. 9, Eq. 14).

    Each is -w^T dG/dtheta evaluated at x1, where G = dg/dx, plus the explicit v1 path. a_bar
    lists the elements' entries and then the springs'.
    """
    m = prob.mesh
    s_pot = prob.s_pot
    a, a_s = prob.split(a)
    F = m.F(x1)
    _, _, P_mu, P_lam = iso_param_parts(F, prob.model)
    Ffd = np.einsum("eij,ej->ei", F, prob.fd)
    s = np.linalg.norm(Ffd, axis=-1)
    n = Ffd / s[:, None]
    dFw = edge_matrix(w, m.T) @ m.DmInv           # F evaluated on w (F is linear in x)
    n_dFw_d = np.einsum("ei,eij,ej->e", n, dFw, prob.fd)
    W = m.W
    out = {}
    out["a_bar"] = -s_pot * W * prob.kf * (1.0 / a ** 2 - 2.0 * s / a ** 3) * n_dFw_d
    out["mu_bar"] = -s_pot * W * np.sum(P_mu * dFw, axis=(-2, -1))
    out["lam_bar"] = -s_pot * W * np.sum(P_lam * dFw, axis=(-2, -1))
    out["kf_bar"] = -s_pot * W * (1.0 / a) * (s / a - 1.0) * n_dFw_d
    # springs: G = f n at j and -f n at i with f = k c (c l - 1), c = 1/(a l0); only f depends on
    # a (dc/da = -c/a) and on k, so -w^T dG/dtheta = -(df/dtheta) n.(w_j - w_i)
    n_s, l_s, c_s, _ = spring_force_terms(x1, prob.S, prob.ks, prob.l0, a_s)
    n_dw = np.sum(n_s * (w[prob.S[:, 1]] - w[prob.S[:, 0]]), axis=-1)
    df_da = -prob.ks * c_s * (2.0 * c_s * l_s - 1.0) / a_s
    out["a_bar"] = np.concatenate([out["a_bar"], -s_pot * df_da * n_dw])
    out["ks_bar"] = -s_pot * c_s * (c_s * l_s - 1.0) * n_dw
    # state cotangents: G depends on x0 through the inertia term and through friction
    x0_bar = np.zeros_like(x1)
    v0_bar = np.zeros_like(x1)
    if prob.be:
        x0_bar += m.mass[:, None] * w
        v0_bar += prob.h * m.mass[:, None] * w
        if v1_bar is not None:
            x0_bar -= np.asarray(v1_bar) / prob.h
    kfr = prob.sc["k_friction"]
    if kfr != 0.0:
        t = prob.tangential()
        cv = prob.friction_factor(x0)
        dcv = np.where(-x0[:, 1] + prob.sc["eps_friction"] > 0.0, -1.0, 0.0)
        h2 = prob.h ** 2
        # d^2 E_fr / dx_t dx0_t = -2 kfr cv / h^2 ; d^2 E_fr / dx_t dy0 = 2 kfr (x_t - x0_t) cv'(y0) / h^2
        x0_bar[:, t] -= s_pot * (-2.0 * kfr * cv / h2)[:, None] * w[:, t]
        x0_bar[:, 1] -= s_pot * np.sum((2.0 * kfr / h2) * (x1[:, t] - x0[:, t]) * w[:, t], axis=1) * dcv
    x0_bar[prob.pinned] = 0.0
    v0_bar[prob.pinned] = 0.0
    out["x0_bar"] = x0_bar
    out["v0_bar"] = v0_bar
    return out


def com_x_loss(prob: Problem, x):
    """L = -(mass-weighted centre of mass, x component)."""
    m = prob.mesh.mass
    return -float(np.sum(m * x[:, 0]) / np.sum(m))


def com_x_loss_grad(prob: Problem, x):
    m = prob.mesh.mass
    g = np.zeros_like(x)
    g[:, 0] = -m / np.sum(m)
    return g


def rollout(prob: Problem, x0, v0, actions, tol=1e-13, max_iter=50):
    """Run len(actions) steps; returns the list of states [(x_0, v_0), ..., (x_T, v_T)] and stats."""
    states = [(np.asarray(x0, dtype=np.float64).copy(), np.asarray(v0, dtype=np.float64).copy())]
    all_stats = []
    x, v = states[0]
    for a in actions:
        x, v, st = step(prob, x, v, a, tol=tol, max_iter=max_iter)
        states.append((x, v))
        all_stats.append(st)
    return states, all_stats


def rollout_grad(prob: Problem, states, actions, x_bar_T, v_bar_T=None):
    """Backprop through time over a stored rollout: returns dL/da [T, n_e + n_s], dL/dx0, dL/dv0."""
    T = len(actions)
    x_bar = np.asarray(x_bar_T, dtype=np.float64)
    v_bar = np.zeros_like(x_bar) if v_bar_T is None else np.asarray(v_bar_T, dtype=np.float64)
    a_bar = np.zeros((T, prob.mesh.n_e + prob.n_s))
    for t in range(T - 1, -1, -1):
        x0, _ = states[t]
        x1, _ = states[t + 1]
        w = adjoint(prob, x1, x0, actions[t], x_bar, v_bar)
        out = vjp_params(prob, w, x1, x0, actions[t], v_bar)
        a_bar[t] = out["a_bar"]
        x_bar, v_bar = out["x0_bar"], out["v0_bar"]
    return a_bar, x_bar, v_bar
