"""Pins of the oracle's vertex-pair springs (Eq. 2 with l = |x_j - x_i|, Fig. 2), all CPU.

Energy and derivatives against hand-derived values, finite differences and an independent torch
autograd of the spring energy; frame invariance; the stationary state of a spring pair holding a
mass under gravity (a scalar equation solved by root finding); and the implicit gradient of whole
solves with respect to spring actions and stiffnesses against finite differences.
"""
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import fem, solve
from oracle.fem import Problem
from synth import meshes, scenes


def _spring_problem(X, T, S, ks, pinned=None, sc=None, mu=0.0, lam=0.0, kf=0.0):
    X = np.asarray(X, float)
    T = np.asarray(T, np.int32)
    n_e, d = T.shape[0], X.shape[1]
    if pinned is None:
        pinned = np.zeros(X.shape, np.uint8)
    if sc is None:
        sc = scenes.scene("qs", k_contact=0.0, k_friction=0.0, gravity=0.0)
    return Problem(X, T, pinned, np.full(n_e, mu), np.full(n_e, lam), np.full(n_e, kf),
                   meshes.x_fibres(n_e, d), np.ones(n_e), sc, springs=np.asarray(S), k_spring=np.asarray(ks, float))


def _random_spring_strip(sc, seed=0, dim=2):
    """A small strip with springs on the horizontal edges plus random extra pairs (diagonals and
    longer reaches), elastic triangles with fibres, random actions, and a perturbed state."""
    rng = np.random.default_rng(seed)
    if dim == 2:
        X, T = meshes.tri_grid(4, 2)
        S = meshes.grid_springs(4, 2)
    else:
        X, T = meshes.tet_grid(2, 2, 1)
        S = np.zeros((0, 2), np.int32)
    extra = []
    while len(extra) < 6:
        i, j = rng.integers(0, X.shape[0], size=2)
        if i != j:
            extra.append((i, j))
    S = np.concatenate([S, np.asarray(extra, np.int32)])
    p = _spring_problem(X, T, S, rng.uniform(50.0, 500.0, size=S.shape[0]), sc=sc,
                        mu=1000.0, lam=2000.0, kf=1500.0)
    a = rng.uniform(0.7, 1.0, size=p.mesh.n_e + p.n_s)
    x = X + 0.1 * rng.normal(size=X.shape)
    return p, a, x, rng


# ---------------------------------------------------------------------------------------------
# hand-derived values of Eq. 2 for one spring
# ---------------------------------------------------------------------------------------------
def test_single_spring_hand_values():
    # rest (0,0)-(2,0): l0 = 2; a = 0.5 gives a rest length a l0 = 1
    S = np.array([[0, 1]])
    k, l0, a = np.array([3.0]), np.array([2.0]), np.array([0.5])
    x = np.array([[0.0, 0.0], [3.0, 0.0]])           # l = 3: E = 3/2 (3/1 - 1)^2 = 6
    assert fem.spring_energy(x, S, k, l0, a)[0] == pytest.approx(6.0, abs=1e-14)
    # dE/dl = k/(a l0) (l/(a l0) - 1) = 6, along +x at j and -x at i
    assert np.allclose(fem.spring_grad(x, S, k, l0, a), [[-6.0, 0.0], [6.0, 0.0]], atol=1e-14)
    # d^2E/dd^2 = k/(a l0)^2 n n^T + (dE/dl / l)(I - n n^T) = diag(3, 2)
    H = fem.spring_hessians(x, S, k, l0, a)[0]
    K = np.diag([3.0, 2.0])
    assert np.allclose(H, np.block([[K, -K], [-K, K]]), atol=1e-14)
    # at l = a l0 in any direction the spring is at rest: zero energy and force, K = k/(a l0)^2 n n^T
    x = np.array([[0.0, 0.0], [0.6, 0.8]])
    assert abs(fem.spring_energy(x, S, k, l0, a)[0]) <= 1e-30
    assert np.allclose(fem.spring_grad(x, S, k, l0, a), 0.0, atol=1e-14)
    n = np.array([0.6, 0.8])
    assert np.allclose(fem.spring_hessians(x, S, k, l0, a)[0][2:, 2:], 3.0 * np.outer(n, n), atol=1e-14)
    # compressed to half the rest length: E = k/2 (1/2 - 1)^2, force pushes the ends apart
    x = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.5]])
    assert fem.spring_energy(x, S, k, l0, a)[0] == pytest.approx(0.375, abs=1e-14)
    assert np.allclose(fem.spring_grad(x, S, k, l0, a)[1], [0.0, 0.0, -1.5], atol=1e-14)


def test_problem_energy_sums_elements_springs_and_vertices():
    sc = scenes.scene("be", k_contact=1e3, k_friction=10.0)
    p, a, x, rng = _random_spring_strip(sc, seed=1)
    x0 = p.mesh.X - np.array([0.0, 0.05])
    v0 = rng.normal(size=x.shape)
    ee, ev = p.energy_terms(x, x0, v0, a)
    assert ee.shape == (p.mesh.n_e + p.n_s,)
    ae, as_ = p.split(a)
    assert np.allclose(ee[p.mesh.n_e:], p.s_pot * fem.spring_energy(x, p.S, p.ks, p.l0, as_), rtol=1e-15)
    assert np.allclose(ee[:p.mesh.n_e], p.s_pot * p.element_energy(x, ae), rtol=1e-15)
    with pytest.raises(ValueError):
        p.split(a[:-1])


# ---------------------------------------------------------------------------------------------
# finite differences, symmetry and frame invariance
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("integrator", ["qs", "be"])
def test_spring_gradient_and_hessian_vs_finite_differences(integrator):
    sc = scenes.scene(integrator, k_contact=1e3, k_friction=10.0)
    p, a, x, rng = _random_spring_strip(sc, seed=2)
    x0 = p.mesh.X - np.array([0.0, 0.05])
    v0 = rng.normal(size=x.shape)
    G = p.grad(x, x0, v0, a).ravel()
    H = p.hessian(x, x0, a).toarray()
    assert np.allclose(H, H.T, rtol=0, atol=1e-9 * np.abs(H).max())
    eps = 1e-6
    for dof in rng.choice(x.size, size=8, replace=False):
        e = np.zeros(x.size)
        e[dof] = eps
        xp, xm = x + e.reshape(x.shape), x - e.reshape(x.shape)
        fd = (p.energy(xp, x0, v0, a) - p.energy(xm, x0, v0, a)) / (2 * eps)
        assert fd == pytest.approx(G[dof], rel=1e-6, abs=1e-6 * np.abs(G).max())
        fdg = (p.grad(xp, x0, v0, a).ravel() - p.grad(xm, x0, v0, a).ravel()) / (2 * eps)
        assert np.allclose(fdg, H[:, dof], rtol=1e-5, atol=1e-6 * np.abs(H).max())


def test_spring_rotation_translation_invariance_and_balance():
    sc = scenes.scene("qs", k_contact=0.0, k_friction=0.0, gravity=0.0)
    p, a, x, rng = _random_spring_strip(sc, seed=3)
    ae, as_ = p.split(a)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    y = x @ R.T + np.array([3.0, -2.0])
    E = fem.spring_energy(x, p.S, p.ks, p.l0, as_)
    assert np.allclose(fem.spring_energy(y, p.S, p.ks, p.l0, as_), E, rtol=1e-12, atol=1e-14)
    G = fem.spring_grad(x, p.S, p.ks, p.l0, as_)
    scale = np.abs(G).max()
    assert np.allclose(G.sum(axis=0), 0.0, atol=1e-12 * scale)            # no net force
    torque = np.sum(x[:, 0] * G[:, 1] - x[:, 1] * G[:, 0])
    assert abs(torque) <= 1e-12 * scale * np.abs(x).max() * x.shape[0]    # no net torque
    # the gradient rotates with the frame
    assert np.allclose(fem.spring_grad(y, p.S, p.ks, p.l0, as_), G @ R.T, atol=1e-12 * scale)


# ---------------------------------------------------------------------------------------------
# the closed forms against reverse-mode AD of the spring energy (Sec. 4.1, Eq. 10)
# ---------------------------------------------------------------------------------------------
def test_spring_derivatives_match_torch_autograd():
    torch = pytest.importorskip("torch")
    sc = scenes.scene("qs", k_contact=0.0, k_friction=0.0, gravity=0.0)
    p, a, x, rng = _random_spring_strip(sc, seed=4)
    ae, as_ = p.split(a)
    S = torch.from_numpy(p.S)

    def energy(xt, at, kt):
        dvec = xt[S[:, 1]] - xt[S[:, 0]]
        l = torch.sqrt((dvec * dvec).sum(-1))
        l0 = torch.from_numpy(p.l0)
        return (0.5 * kt * (l / (at * l0) - 1.0) ** 2).sum()

    xt = torch.tensor(x, requires_grad=True)
    at = torch.tensor(as_, requires_grad=True)
    kt = torch.tensor(p.ks, requires_grad=True)
    (g,) = torch.autograd.grad(energy(xt, at, kt), xt, create_graph=True)
    G = fem.spring_grad(x, p.S, p.ks, p.l0, as_)
    assert np.allclose(g.detach().numpy(), G, rtol=1e-12, atol=1e-12 * np.abs(G).max())
    # Hessian-vector product as the gradient of <f, v> (Eq. 10)
    v = torch.from_numpy(rng.normal(size=x.shape))
    hv, a_mixed, k_mixed = torch.autograd.grad((g * v).sum(), (xt, at, kt), retain_graph=True)
    Hs = fem.spring_hessians(x, p.S, p.ks, p.l0, as_)
    Hv = np.zeros_like(x)
    vv = v.numpy()
    for s, (i, j) in enumerate(p.S):
        loc = Hs[s] @ np.concatenate([vv[i], vv[j]])
        Hv[i] += loc[:2]
        Hv[j] += loc[2:]
    assert np.allclose(hv.numpy(), Hv, rtol=1e-11, atol=1e-11 * np.abs(Hv).max())
    # mixed partials d<G, w>/da and d<G, w>/dk are minus the oracle's spring cotangents (Eq. 9)
    p_qs = p  # quasistatic: s_pot = 1
    out = solve.vjp_params(p_qs, vv, x, p.mesh.X, a)
    assert np.allclose(out["a_bar"][p.mesh.n_e:], -a_mixed.numpy(), rtol=1e-11, atol=1e-12)
    assert np.allclose(out["ks_bar"], -k_mixed.numpy(), rtol=1e-11, atol=1e-14)


# ---------------------------------------------------------------------------------------------
# a stationary state fixed by a scalar equation; the fibre-only check of Eq. 2 (l = a l0)
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("act", [1.0, 0.85])
def test_spring_pair_holds_mass_under_gravity(act):
    # vertices 0 (-1, 0) and 1 (1, 0) pinned; vertex 2 at (0, -1) hangs from two springs of rest
    # length sqrt(2). Its mass is one third of the (massive, stress-free) triangle's area 1. At
    # (0, -y): l = sqrt(1 + y^2) and stationarity is m g = 2 f(l) y / l, f = k c (c l - 1), c = 1/(a l0)
    g, k = 9.8, 2.0
    X = np.array([[-1.0, 0.0], [1.0, 0.0], [0.0, -1.0]])
    pinned = np.zeros((3, 2), np.uint8)
    pinned[:2] = 1
    sc = scenes.scene("qs", k_contact=0.0, k_friction=0.0, gravity=g)
    p = _spring_problem(X, [[0, 2, 1]], [[0, 2], [1, 2]], [k, k], pinned=pinned, sc=sc)
    m = 1.0 / 3.0
    assert p.mesh.mass[2] == pytest.approx(m, rel=1e-15)
    c = 1.0 / (act * math.sqrt(2.0))
    resid = lambda y: m * g - 2.0 * k * c * (c * math.sqrt(1 + y * y) - 1.0) * y / math.sqrt(1 + y * y)
    y_star = scipy.optimize.brentq(resid, 1e-6, 50.0, xtol=1e-15, rtol=1e-15)
    x1, _, st = solve.step(p, X, None, np.array([1.0, act, act]), tol=1e-14)
    assert st["converged"]
    assert x1[2, 0] == pytest.approx(0.0, abs=1e-12)
    assert x1[2, 1] == pytest.approx(-y_star, rel=1e-11)


def test_single_free_spring_settles_at_action_times_rest_length():
    # one pinned end, no gravity: the minimiser has l = a l0 along the initial direction (Eq. 2)
    X = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 1.0]])
    pinned = np.zeros((3, 2), np.uint8)
    pinned[[0, 2]] = 1
    p = _spring_problem(X, [[0, 1, 2]], [[0, 1]], [5.0], pinned=pinned)
    x1, _, st = solve.step(p, X, None, np.array([1.0, 0.7]), tol=1e-14)
    assert st["converged"]
    assert np.allclose(x1[1], [1.4, 0.0], atol=1e-12)


# ---------------------------------------------------------------------------------------------
# the implicit gradient through whole solves against finite differences
# ---------------------------------------------------------------------------------------------
def test_spring_action_and_stiffness_gradients_match_fd_of_rollout():
    w = scenes.be_spring_strip(4, 2, steps=2)
    w.x0 = w.X + np.array([0.0, 0.02])
    p = Problem.from_workload(w)
    acts = w.actions.copy()

    def loss(A, ks=None):
        if ks is not None:
            p.ks = ks
        states, _ = solve.rollout(p, w.x0, w.v0, A, tol=1e-14)
        p.ks = w.ks.copy()
        return solve.com_x_loss(p, states[-1][0])

    states, _ = solve.rollout(p, w.x0, w.v0, acts, tol=1e-14)
    a_bar, _, _ = solve.rollout_grad(p, states, acts, solve.com_x_loss_grad(p, states[-1][0]))
    assert a_bar.shape == (2, w.n_e + w.n_s)
    eps = 1e-6
    rng = np.random.default_rng(0)
    for t, s in [(0, 0), (1, 3), (0, w.n_s - 1), (1, 5)]:
        col = w.n_e + s
        Ap, Am = acts.copy(), acts.copy()
        Ap[t, col] += eps
        Am[t, col] -= eps
        fd = (loss(Ap) - loss(Am)) / (2 * eps)
        assert a_bar[t, col] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    assert np.abs(a_bar[:, w.n_e:]).max() > 1e-6
    # stiffness cotangent of the last step (single-step VJP) against a finite difference of that step
    x1, _ = states[-1]
    x_prev, v_prev = states[-2]
    xb = solve.com_x_loss_grad(p, x1)
    wv = solve.adjoint(p, x1, x_prev, acts[-1], xb)
    ks_bar = solve.vjp_params(p, wv, x1, x_prev, acts[-1])["ks_bar"]
    for s in rng.choice(w.n_s, size=3, replace=False):
        vals = []
        for sgn in (1, -1):
            ks = w.ks.copy()
            ks[s] += sgn * 1e-2
            p.ks = ks
            x1s, _, _ = solve.step(p, x_prev, v_prev, acts[-1], tol=1e-14)
            vals.append(solve.com_x_loss(p, x1s))
        p.ks = w.ks.copy()
        assert ks_bar[s] == pytest.approx((vals[0] - vals[1]) / 2e-2, rel=1e-5, abs=1e-12)
