"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself: a closed
form, a textbook stiffness, an invariant, finite differences, an independent
automatic differentiation (the paper's own recipe of Sec. 4.1, Eq. 10: forces by
autograd of E, Hessian-vector products by autograd of <f, v>), or brute force on a
tiny input. All CPU.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import fem, solve
from oracle.fem import Problem
from synth import meshes, scenes

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _tri(X, T, mu=1000.0, lam=2000.0, kf=1500.0, pinned=None, sc=None, fd=None):
    X = np.asarray(X, float)
    T = np.asarray(T, np.int32)
    n_e, d = T.shape[0], X.shape[1]
    if pinned is None:
        pinned = np.zeros(X.shape, np.uint8)
    if fd is None:
        fd = meshes.x_fibres(n_e, d)
    if sc is None:
        sc = scenes.scene("qs", k_contact=0.0, k_friction=0.0, gravity=0.0)
    return Problem(X, T, pinned, np.full(n_e, mu), np.full(n_e, lam), np.full(n_e, kf), fd,
                   np.ones(n_e), sc)


def _random_fd(rng, n_e, d):
    f = rng.normal(size=(n_e, d))
    return f / np.linalg.norm(f, axis=1, keepdims=True)


def _small_strip(dim=2, sc=None, seed=0):
    if dim == 2:
        X, T = meshes.tri_grid(4, 2)
    else:
        X, T = meshes.tet_grid(2, 2, 1)
    rng = np.random.default_rng(seed)
    p = _tri(X, T, sc=sc, fd=_random_fd(rng, T.shape[0], dim))
    return p, rng


# ---------------------------------------------------------------------------------------------
# V1: the rest state is stress free (Eq. 3 at F = I; Eq. 2 at a = 1, l = l0)
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_rest_state_zero_energy_and_stress(dim):
    p, rng = _small_strip(dim)
    a = np.ones(p.mesh.n_e)
    F = np.broadcast_to(np.eye(dim), (p.mesh.n_e, dim, dim)).copy()
    assert np.allclose(fem.psi(F, p.mu, p.lam, p.kf, a, p.fd), 0.0, atol=1e-12)
    assert np.allclose(fem.stress(F, p.mu, p.lam, p.kf, a, p.fd), 0.0, atol=1e-12)
    assert np.allclose(p.element_grad(p.mesh.X, a), 0.0, atol=1e-10)


def test_quasistatic_rest_returns_rest_in_zero_iterations():
    w = scenes.qs_cantilever()
    w.scene["gravity"] = 0.0
    p = Problem.from_workload(w)
    x1, _, st = solve.step(p, w.X, None, np.ones(w.n_e))
    assert st["newton_iters"] == 0 and st["res0"] == 0.0
    assert np.array_equal(x1, w.X)


def test_log_replacement_matches_log_to_second_order():
    # the quadratic stand-in agrees with log J in value, slope and curvature at J = 1 (Sec. 3)
    J = 1.0 + np.array([-1e-2, -1e-3, 1e-3, 1e-2])
    err = np.abs(fem.logq(J) - np.log(J))
    assert np.all(err <= 0.5 * np.abs(J - 1.0) ** 3)
    assert fem.logq(1.0) == 0.0 and fem.logq_d(1.0) == 1.0 and fem.LOGQ_DD == -1.0
    assert np.isfinite(fem.logq(np.array([-1.0, 0.0]))).all()


# ---------------------------------------------------------------------------------------------
# V2: at rest the Hessian is the textbook linear-elastic stiffness (+ the fibre term)
# ---------------------------------------------------------------------------------------------
def test_unit_triangle_stiffness_golden():
    g = GOLDEN["unit_triangle_cst_plane_strain"]
    mu, lam = scenes.lame(1e4, 0.3)
    p = _tri([[0, 0], [1, 0], [0, 1]], [[0, 1, 2]], mu=mu, lam=lam, kf=0.0)
    K = fem.element_hessians(p.mesh, p.mesh.X, p.mu, p.lam, p.kf, np.ones(1), p.fd)[0]
    assert K[0, 0] == pytest.approx(g["K_00"], rel=1e-13)
    assert K[0, 1] == pytest.approx(g["K_01"], rel=1e-13)
    assert K[0, 2] == pytest.approx(g["K_02"], rel=1e-13)
    assert K[1, 1] == pytest.approx(g["K_11"], rel=1e-13)


def _cst_stiffness(X3, E, nu):
    """Constant-strain triangle, plane strain: K = A B^T D B (textbook)."""
    (x1, y1), (x2, y2), (x3, y3) = X3
    A2 = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1)
    b = np.array([y2 - y3, y3 - y1, y1 - y2]) / A2
    c = np.array([x3 - x2, x1 - x3, x2 - x1]) / A2
    B = np.zeros((3, 6))
    B[0, 0::2] = b
    B[1, 1::2] = c
    B[2, 0::2] = c
    B[2, 1::2] = b
    k = E / ((1 + nu) * (1 - 2 * nu))
    D = k * np.array([[1 - nu, nu, 0], [nu, 1 - nu, 0], [0, 0, (1 - 2 * nu) / 2]])
    return 0.5 * A2 * B.T @ D @ B


def _tet_stiffness(X4, E, nu):
    """Linear tetrahedron: K = V B^T D B with the isotropic 6x6 D (textbook)."""
    M = np.hstack([np.ones((4, 1)), X4])
    V = np.linalg.det(M) / 6.0
    grads = np.linalg.inv(M)[1:, :].T        # row i = grad N_i
    B = np.zeros((6, 12))
    for i in range(4):
        gx, gy, gz = grads[i]
        B[0, 3 * i] = gx
        B[1, 3 * i + 1] = gy
        B[2, 3 * i + 2] = gz
        B[3, 3 * i] = gy
        B[3, 3 * i + 1] = gx
        B[4, 3 * i + 1] = gz
        B[4, 3 * i + 2] = gy
        B[5, 3 * i] = gz
        B[5, 3 * i + 2] = gx
    k = E / ((1 + nu) * (1 - 2 * nu))
    D = np.zeros((6, 6))
    D[:3, :3] = k * nu
    D[np.arange(3), np.arange(3)] = k * (1 - nu)
    D[np.arange(3, 6), np.arange(3, 6)] = k * (1 - 2 * nu) / 2
    return V * B.T @ D @ B


@pytest.mark.parametrize("dim", [2, 3])
def test_rest_hessian_is_linear_elastic_stiffness(dim):
    rng = np.random.default_rng(7)
    E, nu = 1e4, 0.3
    mu, lam = scenes.lame(E, nu)
    for _ in range(5):
        X = rng.normal(size=(dim + 1, dim))
        T = np.arange(dim + 1)[None, :]
        if fem.det(fem.edge_matrix(X, T))[0] < 0:
            X[[1, 2]] = X[[2, 1]]
        fd = _random_fd(rng, 1, dim)
        kf = 321.0
        p = _tri(X, T, mu=mu, lam=lam, kf=kf, fd=fd)
        K = fem.element_hessians(p.mesh, X, p.mu, p.lam, p.kf, np.ones(1), p.fd)[0]
        Kref = _cst_stiffness(X, E, nu) if dim == 2 else _tet_stiffness(X, E, nu)
        # fibre at a = 1 and F = I adds W kf (d^T dF d)^2 with dF = D_s(u) Dm^-1
        W = p.mesh.W[0]
        Bf = np.zeros(((dim + 1) * dim,))
        gvec = p.mesh.DmInv[0] @ fd[0]        # d^T dF d = sum_j (u_j - u_0) . d * g_j
        for j in range(dim):
            Bf[(j + 1) * dim:(j + 2) * dim] += gvec[j] * fd[0]
            Bf[0:dim] -= gvec[j] * fd[0]
        Kref = Kref + W * kf * np.outer(Bf, Bf)
        assert np.allclose(K, Kref, rtol=1e-11, atol=1e-9 * np.abs(Kref).max())


# ---------------------------------------------------------------------------------------------
# V3: frame invariance; internal forces have zero net force and zero net torque
# ---------------------------------------------------------------------------------------------
def _rotation(rng, dim):
    Q, _ = np.linalg.qr(rng.normal(size=(dim, dim)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


@pytest.mark.parametrize("dim", [2, 3])
def test_rotation_translation_invariance_and_balance(dim):
    p, rng = _small_strip(dim)
    a = rng.uniform(0.7, 1.0, p.mesh.n_e)
    x = p.mesh.X + 0.1 * rng.normal(size=p.mesh.X.shape)
    R, t = _rotation(rng, dim), rng.normal(size=dim)
    e1 = p.element_energy(x, a)
    e2 = p.element_energy(x @ R.T + t, a)
    assert np.allclose(e1, e2, rtol=1e-12, atol=1e-12)
    G = p.element_grad(x, a)
    assert np.allclose(G.sum(axis=0), 0.0, atol=1e-9 * np.abs(G).max())
    if dim == 2:
        torque = np.sum(x[:, 0] * G[:, 1] - x[:, 1] * G[:, 0])
    else:
        torque = np.cross(x, G).sum(axis=0)
    assert np.allclose(torque, 0.0, atol=1e-9 * np.abs(G).max() * np.abs(x).max())


# ---------------------------------------------------------------------------------------------
# V4: homogeneous patch test: the FEM minimiser is an exact affine map diag(s*, t*)
# ---------------------------------------------------------------------------------------------
def test_homogeneous_patch():
    from scipy.optimize import minimize
    mu, lam = scenes.lame(1e4, 0.3)
    kf, a = 1e4, 0.7
    X, T = meshes.tri_grid(10, 4)
    pinned = np.zeros(X.shape, np.uint8)
    pinned[0] = 1                        # vertex (0,0): both DOFs
    pinned[10, 1] = 1                    # vertex (10,0): y only (roller)
    p = _tri(X, T, mu=mu, lam=lam, kf=kf, pinned=pinned)
    x1, _, st = solve.step(p, X, None, np.full(p.mesh.n_e, a), tol=1e-13)

    def dens(v):                          # the 1-element problem for F = diag(s, t)
        s, t = v
        J = s * t
        lJ = (J - 1) - 0.5 * (J - 1) ** 2
        return 0.5 * mu * (s * s + t * t - 2) - mu * lJ + 0.5 * lam * lJ ** 2 + 0.5 * kf * (s / a - 1) ** 2
    r = minimize(dens, [0.8, 1.1], method="BFGS", options=dict(gtol=1e-12))
    s_star, t_star = r.x
    assert s_star == pytest.approx(0.81625, abs=2e-5) and t_star == pytest.approx(1.08156, abs=2e-5)
    assert np.allclose(x1, X * np.array([s_star, t_star]), atol=1e-7)


# ---------------------------------------------------------------------------------------------
# V5: gradient and Hessian against central finite differences; Hessian symmetry
# ---------------------------------------------------------------------------------------------
def _contact_scene(integrator):
    return scenes.scene(integrator, h=0.05, k_contact=3e3, k_friction=50.0, eps_friction=0.3, gravity=9.8)


@pytest.mark.parametrize("dim,integrator", [(2, "qs"), (2, "be"), (3, "be")])
def test_gradient_and_hessian_vs_finite_differences(dim, integrator):
    p, rng = _small_strip(dim, sc=_contact_scene(integrator), seed=3)
    n_e = p.mesh.n_e
    a = rng.uniform(0.7, 1.0, n_e)
    x0 = p.mesh.X + 0.05 * rng.normal(size=p.mesh.X.shape)
    x0[:, 1] -= 0.1                        # some vertices below the ground: contact + friction active
    v0 = rng.normal(size=x0.shape)
    x = x0 + 0.1 * rng.normal(size=x0.shape)
    g = lambda xx: p.energy(xx, x0, v0, a)
    G = p.grad(x, x0, v0, a)
    u = rng.normal(size=x.shape)
    eps = 1e-6
    fd = (g(x + eps * u) - g(x - eps * u)) / (2 * eps)
    assert fd == pytest.approx(np.sum(G * u), rel=1e-7, abs=1e-9)
    H = p.hessian(x, x0, a)
    Hu = (H @ u.ravel()).reshape(x.shape)
    fdH = (p.grad(x + eps * u, x0, v0, a) - p.grad(x - eps * u, x0, v0, a)) / (2 * eps)
    assert np.allclose(Hu, fdH, rtol=1e-6, atol=1e-6 * np.abs(fdH).max())
    assert abs(H - H.T).max() <= 1e-12 * abs(H).max()


# ---------------------------------------------------------------------------------------------
# V6: the closed forms equal reverse-mode AD of the energy (the paper's Sec. 4.1 recipe)
# ---------------------------------------------------------------------------------------------
def _torch_energy(torch, p, x, x0, v0, a):
    """The objective written once more as torch FP64 ops (test-only cross-check)."""
    m = p.mesh
    T = torch.as_tensor(m.T)
    Dinv = torch.as_tensor(m.DmInv)
    e = x[T[:, 1:]] - x[T[:, :1]]
    F = e.transpose(1, 2) @ Dinv
    J = torch.linalg.det(F)
    lJ = (J - 1) - 0.5 * (J - 1) ** 2
    I1 = (F * F).sum(dim=(1, 2))
    mu, lam, kf = (torch.as_tensor(v) for v in (p.mu, p.lam, p.kf))
    fd = torch.as_tensor(p.fd)
    s = torch.linalg.norm(torch.einsum("eij,ej->ei", F, fd), dim=1)
    psi = 0.5 * mu * (I1 - m.d) - mu * lJ + 0.5 * lam * lJ ** 2 + 0.5 * kf * (s / a - 1) ** 2
    E = (torch.as_tensor(m.W) * psi).sum()
    mass = torch.as_tensor(m.mass)
    y = x[:, 1]
    E = E + (mass * p.sc["gravity"] * y).sum() + p.sc["k_contact"] * (torch.relu(-y) ** 2).sum()
    cv = torch.relu(-x0[:, 1] + p.sc["eps_friction"])
    t = p.tangential()
    vt = (x[:, t] - x0[:, t]) / p.h
    E = E + (p.sc["k_friction"] * cv * (vt * vt).sum(dim=1)).sum()
    if p.be:
        dx = x - (x0 + p.h * v0)
        return 0.5 * (mass * (dx * dx).sum(dim=1)).sum() + p.h ** 2 * E
    return E


@pytest.mark.parametrize("dim", [2, 3])
def test_closed_forms_match_torch_double_backward(dim):
    torch = pytest.importorskip("torch")
    p, rng = _small_strip(dim, sc=_contact_scene("be"), seed=11)
    a_np = rng.uniform(0.7, 1.0, p.mesh.n_e)
    x0_np = p.mesh.X + 0.05 * rng.normal(size=p.mesh.X.shape)
    x0_np[:, 1] -= 0.1
    v0_np = rng.normal(size=x0_np.shape)
    x_np = x0_np + 0.1 * rng.normal(size=x0_np.shape)
    u_np = rng.normal(size=x_np.shape)
    x = torch.tensor(x_np, requires_grad=True)
    x0, v0, a = torch.tensor(x0_np), torch.tensor(v0_np), torch.tensor(a_np)
    E = _torch_energy(torch, p, x, x0, v0, a)
    assert E.item() == pytest.approx(p.energy(x_np, x0_np, v0_np, a_np), rel=1e-13)
    (gx,) = torch.autograd.grad(E, x, create_graph=True)
    assert np.allclose(gx.detach().numpy(), p.grad(x_np, x0_np, v0_np, a_np), rtol=1e-11, atol=1e-11)
    (hv,) = torch.autograd.grad((gx * torch.tensor(u_np)).sum(), x)
    Hu = (p.hessian(x_np, x0_np, a_np) @ u_np.ravel()).reshape(x_np.shape)
    assert np.allclose(hv.numpy(), Hu, rtol=1e-10, atol=1e-10 * np.abs(Hu).max())


def test_vjp_closed_forms_match_torch_mixed_partials():
    """-w^T dG/dtheta for theta in (a, mu, lam, kf, x0, v0) by autograd of <G, w> (Sec. 4.1)."""
    torch = pytest.importorskip("torch")
    p, rng = _small_strip(2, sc=_contact_scene("be"), seed=5)
    n_e = p.mesh.n_e
    a_np = rng.uniform(0.7, 1.0, n_e)
    x0_np = p.mesh.X + 0.05 * rng.normal(size=p.mesh.X.shape)
    x0_np[:, 1] -= 0.1
    v0_np = rng.normal(size=x0_np.shape)
    x1_np = x0_np + 0.1 * rng.normal(size=x0_np.shape)
    w_np = rng.normal(size=x0_np.shape)
    theta = {k: torch.tensor(v, requires_grad=True) for k, v in
             dict(a=a_np, mu=p.mu, lam=p.lam, kf=p.kf, x0=x0_np, v0=v0_np).items()}
    q = Problem(p.mesh.X, p.mesh.T, p.pinned, p.mu, p.lam, p.kf, p.fd, np.ones(n_e), p.sc)
    x = torch.tensor(x1_np, requires_grad=True)

    class _P:  # torch view of the same problem with trainable parameters
        pass
    tp = _P()
    tp.mesh, tp.sc, tp.h, tp.be, tp.fd = q.mesh, q.sc, q.h, q.be, q.fd
    tp.mu, tp.lam, tp.kf = theta["mu"], theta["lam"], theta["kf"]
    tp.tangential = q.tangential
    E = _torch_energy(torch, tp, x, theta["x0"], theta["v0"], theta["a"])
    (G,) = torch.autograd.grad(E, x, create_graph=True)
    inner = -(G * torch.tensor(w_np)).sum()
    grads = torch.autograd.grad(inner, [theta[k] for k in ("a", "mu", "lam", "kf", "x0", "v0")])
    out = solve.vjp_params(q, w_np, x1_np, x0_np, a_np, v1_bar=None)
    for name, gref in zip(("a_bar", "mu_bar", "lam_bar", "kf_bar", "x0_bar", "v0_bar"), grads):
        gref = gref.numpy()
        assert np.allclose(out[name], gref, rtol=1e-10, atol=1e-10 * max(np.abs(gref).max(), 1e-30)), name


# ---------------------------------------------------------------------------------------------
# V7 / V8: closed-form solutions of the step (golden values)
# ---------------------------------------------------------------------------------------------
def test_free_fall_closed_form():
    g = GOLDEN["free_fall"]
    X, T = meshes.tri_grid(3, 2)
    sc = scenes.scene("be", h=0.1, k_contact=0.0, k_friction=0.0, gravity=9.8)
    p = _tri(X, T, mu=0.0, lam=0.0, kf=0.0, sc=sc)
    v0 = np.tile([0.5, 1.0], (X.shape[0], 1))
    x1, v1, st = solve.step(p, X, v0, np.ones(T.shape[0]))
    assert st["newton_iters"] == 1
    assert np.allclose(x1 - X, g["dx"], atol=1e-14)
    assert np.allclose(v1, g["v1"], atol=1e-12)


def test_single_triangle_contact_depth():
    g = GOLDEN["contact_rest_depth"]
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    pinned = np.zeros((3, 2), np.uint8)
    pinned[:, 0] = 1
    sc = scenes.scene("qs", k_contact=1e5, k_friction=0.0, gravity=9.8)
    p = _tri(X, [[0, 1, 2]], mu=0.0, lam=0.0, kf=0.0, pinned=pinned, sc=sc)
    assert np.allclose(p.mesh.mass, g["mass"], rtol=1e-15)
    x0 = X.copy()
    x0[:, 1] = -1e-3                        # start in contact so the indicator [y < 0] is on
    x1, _, st = solve.step(p, x0, None, np.ones(1), tol=1e-14)
    assert np.allclose(x1[:, 1], g["y_star"], rtol=1e-9)
    assert np.array_equal(x1[:, 0], x0[:, 0])


def test_lumped_mass_total_is_area():
    X, T = meshes.tri_grid(7, 3)
    p = _tri(X, T)
    assert p.mesh.mass.sum() == pytest.approx(21.0, rel=1e-14)
    X, T = meshes.tet_grid(3, 2, 2)
    p = _tri(X, T)
    assert p.mesh.mass.sum() == pytest.approx(12.0, rel=1e-14)
    assert np.all(p.mesh.W > 0)


# ---------------------------------------------------------------------------------------------
# V9 / V10 / V11 / V15: invariants of the solve
# ---------------------------------------------------------------------------------------------
def test_newton_converges_quadratically():
    w = scenes.qs_cantilever()
    p = Problem.from_workload(w)
    _, _, st = solve.step(p, w.x0, None, w.actions[0], tol=1e-13)
    r = np.array(st["res_hist"]) / st["res0"]
    assert st["converged"]
    tail = [(r[k], r[k + 1]) for k in range(len(r) - 1) if 1e-12 < r[k + 1] and r[k] < 1e-2]
    assert tail, r
    for rk, rk1 in tail:
        assert rk1 <= 1e3 * rk * rk, r


def test_momentum_conserved_without_external_forces():
    X, T = meshes.tri_grid(6, 3)
    sc = scenes.scene("be", h=1 / 60, k_contact=0.0, k_friction=0.0, gravity=0.0)
    rng = np.random.default_rng(2)
    p = _tri(X, T, sc=sc, fd=_random_fd(rng, T.shape[0], 2))
    x, v = X.copy(), rng.normal(size=X.shape)
    P0 = (p.mesh.mass[:, None] * v).sum(axis=0)
    for k in range(3):
        x, v, st = solve.step(p, x, v, rng.uniform(0.7, 1.0, T.shape[0]), tol=1e-13)
    P1 = (p.mesh.mass[:, None] * v).sum(axis=0)
    assert np.allclose(P0, P1, atol=1e-9 * np.abs(v).max())


def test_com_gradient_vanishes_without_friction():
    w = scenes.be_strip(nx=8, ny=2, steps=4)
    w.scene["k_friction"] = 0.0
    p = Problem.from_workload(w)
    states, _ = solve.rollout(p, w.x0, w.v0, w.actions)
    a_bar, _, _ = solve.rollout_grad(p, states, w.actions, solve.com_x_loss_grad(p, states[-1][0]))
    assert np.abs(a_bar).max() <= 1e-10


def test_fibre_only_element_reaches_rest_length_times_action():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    pinned = np.zeros((3, 2), np.uint8)
    pinned[0] = 1
    pinned[2] = 1
    pinned[1, 1] = 1
    p = _tri(X, [[0, 1, 2]], mu=0.0, lam=0.0, kf=10.0, pinned=pinned)
    for a in (0.6, 0.85, 1.3):
        x1, _, _ = solve.step(p, X, None, np.array([a]), tol=1e-14)
        assert np.linalg.norm(x1[1] - x1[0]) == pytest.approx(a, rel=1e-12)


# ---------------------------------------------------------------------------------------------
# V12 / V13 / V14: the implicit gradient against finite differences of whole solves and brute force
# ---------------------------------------------------------------------------------------------
def test_brute_force_dense_hessian_and_newton_on_cantilever():
    w = scenes.qs_cantilever()
    p = Problem.from_workload(w)
    a = w.actions[0]
    rng = np.random.default_rng(1)
    x = w.X + 0.05 * rng.normal(size=w.X.shape)
    H = p.hessian(x, w.x0, a).toarray()
    n = H.shape[0]
    eps = 1e-5
    Hfd = np.zeros_like(H)
    for k in range(n):
        e = np.zeros(n)
        e[k] = eps
        Hfd[:, k] = ((p.grad(x + e.reshape(x.shape), w.x0, None, a)
                      - p.grad(x - e.reshape(x.shape), w.x0, None, a)) / (2 * eps)).ravel()
    assert np.allclose(H, Hfd, rtol=1e-6, atol=1e-6 * np.abs(H).max())
    # dense Newton with numpy.linalg.solve lands on the same minimiser as the SuperLU Newton
    free = p.free
    xd = w.x0.copy()
    for _ in range(30):
        G = p.grad(xd, w.x0, None, a).ravel()[free]
        Hd = p.hessian(xd, w.x0, a).toarray()[np.ix_(free, free)]
        xd.reshape(-1)[free] -= np.linalg.solve(Hd, G)
    x1, _, _ = solve.step(p, w.x0, None, a, tol=1e-14)
    assert np.allclose(xd, x1, rtol=0, atol=1e-11 * np.abs(x1).max())


def test_adjoint_linear_loss_matches_dense_and_fd():
    w = scenes.qs_cantilever()
    p = Problem.from_workload(w)
    a = w.actions[0]
    x1, _, _ = solve.step(p, w.x0, None, a, tol=1e-14)
    rng = np.random.default_rng(4)
    c = rng.normal(size=x1.shape)
    wv = solve.adjoint(p, x1, w.x0, a, c)
    g = solve.vjp_params(p, wv, x1, w.x0, a)["a_bar"]
    # dense: dL/da_e = -c^T H^-1 dG/da_e with dG/da_e by central differences of G in a_e
    free = p.free
    Hd = p.hessian(x1, w.x0, a).toarray()[np.ix_(free, free)]
    z = np.linalg.solve(Hd, c.ravel()[free])
    for e in rng.choice(p.mesh.n_e, 6, replace=False):
        da = np.zeros_like(a)
        da[e] = 1e-6
        dG = (p.grad(x1, w.x0, None, a + da) - p.grad(x1, w.x0, None, a - da)).ravel()[free] / 2e-6
        assert -z @ dG == pytest.approx(g[e], rel=1e-6, abs=1e-9 * np.abs(g).max())
    # finite differences of whole solves along a random direction
    r = rng.choice([-1.0, 1.0], size=a.shape)
    eps = 1e-6
    xp, _, _ = solve.step(p, w.x0, None, a + eps * r, tol=1e-14)
    xm, _, _ = solve.step(p, w.x0, None, a - eps * r, tol=1e-14)
    fd = np.sum(c * (xp - xm)) / (2 * eps)
    assert fd == pytest.approx(g @ r, rel=1e-6)


def test_bptt_gradient_matches_fd_of_rollout():
    w = scenes.be_strip(nx=8, ny=2, steps=4)
    w.scene["k_friction"] = 1e3
    p = Problem.from_workload(w)
    x0, v0 = w.x0.copy(), w.v0.copy()
    v0[:, 0] = 0.3                         # sliding start: friction active from step 0
    states, _ = solve.rollout(p, x0, v0, w.actions)
    loss = solve.com_x_loss(p, states[-1][0])
    a_bar, x0_bar, v0_bar = solve.rollout_grad(p, states, w.actions, solve.com_x_loss_grad(p, states[-1][0]))
    assert np.abs(a_bar).max() > 1e-6
    rng = np.random.default_rng(9)
    eps = 1e-6
    for _ in range(3):
        r = rng.choice([-1.0, 1.0], size=w.actions.shape)
        Lp = solve.com_x_loss(p, solve.rollout(p, x0, v0, w.actions + eps * r)[0][-1][0])
        Lm = solve.com_x_loss(p, solve.rollout(p, x0, v0, w.actions - eps * r)[0][-1][0])
        fd = (Lp - Lm) / (2 * eps)
        ad = np.sum(a_bar * r)
        assert abs(fd - ad) <= 1e-5 * max(abs(fd), abs(ad)) + 1e-10 * abs(loss)
    # state cotangents by finite differences too
    for bar, which in ((x0_bar, "x"), (v0_bar, "v")):
        r = rng.normal(size=x0.shape)
        xp, vp = (x0 + eps * r, v0) if which == "x" else (x0, v0 + eps * r)
        xm, vm = (x0 - eps * r, v0) if which == "x" else (x0, v0 - eps * r)
        Lp = solve.com_x_loss(p, solve.rollout(p, xp, vp, w.actions)[0][-1][0])
        Lm = solve.com_x_loss(p, solve.rollout(p, xm, vm, w.actions)[0][-1][0])
        fd = (Lp - Lm) / (2 * eps)
        assert fd == pytest.approx(np.sum(bar * r), rel=1e-5, abs=1e-9)


def test_tet_grid_is_conforming_and_positive():
    X, T = meshes.tet_grid(3, 2, 2)
    assert T.shape == (6 * 12, 4)
    Dm = fem.edge_matrix(X, T)
    assert np.all(fem.det(Dm) > 0)
    assert np.allclose(fem.det(Dm) / 6.0, 1.0 / 6.0)
    # every interior face is shared by exactly two tets, boundary faces by one
    faces = np.sort(np.concatenate([T[:, [0, 1, 2]], T[:, [0, 1, 3]], T[:, [0, 2, 3]], T[:, [1, 2, 3]]]), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert set(counts.tolist()) <= {1, 2}
    n_boundary = 2 * 2 * (3 * 2 + 3 * 2 + 2 * 2)
    assert int((counts == 1).sum()) == n_boundary


def test_iterative_linear_solves_match_direct():
    """The large-system path (SciPy CG on the assembled matrix) agrees with the direct solves."""
    from tests.gpu_util import rand_workload
    w, rng = rand_workload(3, seed=5, shape=(4, 3, 3))
    p = Problem.from_workload(w)
    a = w.actions[0]
    xd, _, sd = solve.step(p, w.x0, w.v0, a, tol=1e-12, direct_max=10 ** 9)
    xi, _, si = solve.step(p, w.x0, w.v0, a, tol=1e-12, direct_max=0)
    assert np.linalg.norm(xi - xd) <= 1e-11 * np.linalg.norm(xd - w.x0)
    xbar = rng.normal(size=xd.shape)
    wd = solve.adjoint(p, xd, w.x0, a, xbar, direct_max=10 ** 9)
    wi = solve.adjoint(p, xd, w.x0, a, xbar, direct_max=0)
    assert np.linalg.norm(wi - wd) <= 1e-11 * np.linalg.norm(wd)
