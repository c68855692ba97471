"""Pins of the oracle's alternative isotropic element energies (St. Venant-Kirchhoff, corotated,
stable neo-Hookean; Sec. 3 names them next to the neo-Hookean density of Eq. 3), all CPU.

For every model: zero energy and stress at rest; the Hessian at rest equals the textbook linear
elastic stiffness (each model linearises to the same Lame pair); hand-derived energies and
stresses for stretched, rotated and inverted F; frame invariance; gradient, Hessian and the
Lame-pair cotangents against an independent torch autograd of the density (the corotated one
through torch's SVD); finite differences of the assembled objective; Newton on a step.
"""
import math

import numpy as np
import pytest

from oracle import fem, solve
from oracle.fem import Problem
from synth import meshes, scenes
from tests.test_oracle_pins import _cst_stiffness, _random_fd, _rotation, _tet_stiffness

ALT = ["stvk", "corot", "snh"]
ALL = ["nh"] + ALT


def _one(F):
    return np.asarray(F, float)[None]


def _parts(F, model, mu=2.0, lam=3.0):
    """(psi, P) of the isotropic density for one F."""
    pm, pl, Pm, Pl = fem.iso_param_parts(_one(F), model)
    return float(mu * pm[0] + lam * pl[0]), mu * Pm[0] + lam * Pl[0]


# ---------------------------------------------------------------------------------------------
# hand-derived values (mu = 2, lam = 3)
# ---------------------------------------------------------------------------------------------
def test_stvk_hand_values():
    # F = diag(1.5, 1): E = diag(0.625, 0): psi = mu e^2 + lam/2 e^2; P = F (2 mu E + lam tr E I)
    e, P = _parts(np.diag([1.5, 1.0]), "stvk")
    assert e == pytest.approx(2 * 0.625 ** 2 + 1.5 * 0.625 ** 2, abs=1e-14)
    assert np.allclose(P, np.diag([1.5 * (4 * 0.625 + 3 * 0.625), 3 * 0.625]), atol=1e-14)
    # uniform compression to half: E = -3/8 I (3D): psi = mu 3 (3/8)^2 + lam/2 (9/8)^2
    e, P = _parts(0.5 * np.eye(3), "stvk")
    assert e == pytest.approx(2 * 3 * (3 / 8) ** 2 + 1.5 * (9 / 8) ** 2, abs=1e-14)
    assert np.allclose(P, 0.5 * (2 * 2 * (-3 / 8) + 3 * (-9 / 8)) * np.eye(3), atol=1e-14)


def test_corotated_hand_values():
    # F = diag(1.5, 1): R = I, S = F: psi = mu (0.5)^2 + lam/2 (0.5)^2, P = 2 mu (F - I) + lam (0.5) I
    e, P = _parts(np.diag([1.5, 1.0]), "corot")
    assert e == pytest.approx(2 * 0.25 + 1.5 * 0.25, abs=1e-14)
    assert np.allclose(P, np.diag([2 * 2 * 0.5 + 3 * 0.5, 3 * 0.5]), atol=1e-14)
    # the same stretch after a rotation by 0.4 rad: energy unchanged, stress rotated with it
    c, s = math.cos(0.4), math.sin(0.4)
    Q = np.array([[c, -s], [s, c]])
    e2, P2 = _parts(Q @ np.diag([1.5, 1.0]), "corot")
    assert e2 == pytest.approx(e, abs=1e-13) and np.allclose(P2, Q @ P, atol=1e-13)
    # inverted: F = diag(-0.5, 1) keeps R = I (tr(R^T F) = 0.5 cos t is largest at t = 0),
    # S = F: psi = mu (1.5^2) + lam/2 (-1.5)^2
    e, P = _parts(np.diag([-0.5, 1.0]), "corot")
    assert e == pytest.approx(2 * 2.25 + 1.5 * 2.25, abs=1e-14)
    assert np.allclose(P, np.diag([2 * 2 * -1.5 + 3 * -1.5, 3 * -1.5]), atol=1e-14)
    # 3D: diag(2, 1, 1) rotated about z by 90 degrees
    Q = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    e, P = _parts(Q @ np.diag([2.0, 1.0, 1.0]), "corot")
    assert e == pytest.approx(2 * 1.0 + 1.5 * 1.0, abs=1e-13)
    assert np.allclose(P, Q @ np.diag([2 * 2 * 1 + 3, 3, 3]), atol=1e-13)


def test_stable_neohookean_hand_values():
    # psi = mu/2 (I1 - d) - mu (J - 1) + (lam + mu)/2 (J - 1)^2, P = mu F + ((lam + mu)(J - 1) - mu) cof F
    e, P = _parts(np.diag([1.5, 1.0]), "snh")
    assert e == pytest.approx(1.0 * 1.25 - 2 * 0.5 + 2.5 * 0.25, abs=1e-14)
    assert np.allclose(P, np.diag([3.0, 2.0]) + (5 * 0.5 - 2) * np.diag([1.0, 1.5]), atol=1e-14)
    # finite for inverted and collapsed elements (no logarithm): F = diag(-1, 1, 1), J = -1
    e, P = _parts(np.diag([-1.0, 1.0, 1.0]), "snh")
    assert e == pytest.approx(0.0 + 4.0 + 2.5 * 4.0, abs=1e-14)
    assert np.isfinite(_parts(np.zeros((3, 3)), "snh")[0])


# ---------------------------------------------------------------------------------------------
# rest state, rest stiffness, frame invariance
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("model", ALL)
@pytest.mark.parametrize("dim", [2, 3])
def test_rest_state_is_stress_free_and_linearises_to_lame_pair(model, dim):
    e, P = _parts(np.eye(dim), model)
    assert abs(e) <= 1e-14 and np.abs(P).max() <= 1e-14
    rng = np.random.default_rng(70 + dim)
    E, nu = 1e4, 0.3
    mu, lam = scenes.lame(E, nu)
    X = rng.normal(size=(dim + 1, dim))
    T = np.arange(dim + 1)[None, :]
    if fem.det(fem.edge_matrix(X, T))[0] < 0:
        X[[1, 2]] = X[[2, 1]]
    p = Problem(X, T, np.zeros(X.shape, np.uint8), [mu], [lam], [0.0], _random_fd(rng, 1, dim), np.ones(1),
                scenes.scene("qs", k_contact=0.0, k_friction=0.0, gravity=0.0), model=model)
    K = fem.element_hessians(p.mesh, X, p.mu, p.lam, p.kf, np.ones(1), p.fd, model)[0]
    Kref = _cst_stiffness(X, E, nu) if dim == 2 else _tet_stiffness(X, E, nu)
    assert np.allclose(K, Kref, rtol=1e-10, atol=1e-9 * np.abs(Kref).max())


@pytest.mark.parametrize("model", ALT)
@pytest.mark.parametrize("dim", [2, 3])
def test_frame_invariance(model, dim):
    rng = np.random.default_rng(80 + dim)
    F = np.eye(dim)[None] + 0.3 * rng.normal(size=(5, dim, dim))
    Q = _rotation(rng, dim)
    pm, pl, Pm, Pl = fem.iso_param_parts(F, model)
    qm, ql, Qm, Ql = fem.iso_param_parts(Q[None] @ F, model)
    assert np.allclose(pm, qm, rtol=1e-12, atol=1e-13) and np.allclose(pl, ql, rtol=1e-12, atol=1e-13)
    assert np.allclose(Qm, Q[None] @ Pm, atol=1e-12) and np.allclose(Ql, Q[None] @ Pl, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_closest_rotation_is_a_rotation_maximising_trace(dim):
    rng = np.random.default_rng(90 + dim)
    F = rng.normal(size=(40, dim, dim))             # about half of them inverted
    R = fem.closest_rotation(F)
    eye = np.eye(dim)[None]
    assert np.allclose(np.swapaxes(R, 1, 2) @ R, eye, atol=1e-12)
    assert np.allclose(fem.det(R), 1.0, atol=1e-12)
    S = np.swapaxes(R, 1, 2) @ F
    assert np.allclose(S, np.swapaxes(S, 1, 2), atol=1e-12)
    best = np.einsum("eij,eij->e", R, F)
    for _ in range(300):                             # brute force: no sampled rotation does better
        Qs = np.stack([_rotation(rng, dim) for _ in range(F.shape[0])])
        assert np.all(np.einsum("eij,eij->e", Qs, F) <= best + 1e-12)


# ---------------------------------------------------------------------------------------------
# derivatives against an independent torch autograd of each density (Sec. 4.1, Eq. 10)
# ---------------------------------------------------------------------------------------------
def _torch_density(torch, F, mu, lam, model):
    d = F.shape[-1]
    eye = torch.eye(d, dtype=F.dtype)
    if model == "stvk":
        E = 0.5 * (F.transpose(1, 2) @ F - eye)
        trE = E.diagonal(dim1=1, dim2=2).sum(-1)
        return mu * (E * E).sum((1, 2)) + 0.5 * lam * trE ** 2
    if model == "corot":
        U, sig, Vh = torch.linalg.svd(F)
        sign = torch.sign(torch.linalg.det(U @ Vh))
        ones = torch.ones_like(sig)
        D = torch.cat([ones[:, :-1], sign[:, None]], dim=1)
        R = U @ torch.diag_embed(D) @ Vh
        trS = (sig * D).sum(-1)                                  # tr(R^T F)
        return mu * ((F - R) ** 2).sum((1, 2)) + 0.5 * lam * (trS - d) ** 2
    if model == "snh":
        J = torch.linalg.det(F)
        I1 = (F * F).sum((1, 2))
        return 0.5 * mu * (I1 - d) - mu * (J - 1) + 0.5 * (lam + mu) * (J - 1) ** 2
    raise ValueError(model)


@pytest.mark.parametrize("model", ALT)
@pytest.mark.parametrize("dim", [2, 3])
def test_stress_and_differential_match_torch_autograd(model, dim):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(100 + dim)
    n = 12
    F_np = np.eye(dim)[None] + 0.35 * rng.normal(size=(n, dim, dim))
    if model == "corot":
        F_np[:3] = F_np[:3] @ np.diag([-1.0] + [1.0] * (dim - 1))   # inverted ones too
    mu_np, lam_np = rng.uniform(1.0, 3.0, n), rng.uniform(1.0, 3.0, n)
    dF_np = rng.normal(size=F_np.shape)
    F = torch.tensor(F_np, requires_grad=True)
    mu = torch.tensor(mu_np, requires_grad=True)
    lam = torch.tensor(lam_np, requires_grad=True)
    psi = _torch_density(torch, F, mu, lam, model)
    pm, pl, Pm, Pl = fem.iso_param_parts(F_np, model)
    assert np.allclose(psi.detach().numpy(), mu_np * pm + lam_np * pl, rtol=1e-12, atol=1e-12)
    (P,) = torch.autograd.grad(psi.sum(), F, create_graph=True)
    Pref = mu_np[:, None, None] * Pm + lam_np[:, None, None] * Pl
    assert np.allclose(P.detach().numpy(), Pref, rtol=1e-10, atol=1e-10)
    dF = torch.tensor(dF_np)
    dP, dmu, dlam = torch.autograd.grad((P * dF).sum(), (F, mu, lam))
    dPref = fem.iso_stress_diff(F_np, dF_np, mu_np, lam_np, model)
    assert np.allclose(dP.numpy(), dPref, rtol=1e-8, atol=1e-8 * np.abs(dPref).max())
    # P is linear in the Lame pair: d(P : dF)/dmu = P_mu : dF, d(P : dF)/dlam = P_lam : dF
    assert np.allclose(dmu.numpy(), np.sum(Pm * dF_np, axis=(1, 2)), rtol=1e-10, atol=1e-10)
    assert np.allclose(dlam.numpy(), np.sum(Pl * dF_np, axis=(1, 2)), rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------------------------------------
# the assembled objective and the step with each model
# ---------------------------------------------------------------------------------------------
def _strip(dim, model, seed):
    rng = np.random.default_rng(seed)
    X, T = meshes.tri_grid(4, 2) if dim == 2 else meshes.tet_grid(2, 2, 1)
    n_e = T.shape[0]
    mu, lam = scenes.lame(1e4 if dim == 2 else 1e5, 0.3 if dim == 2 else 0.45)
    sc = scenes.scene("be", h=0.05, k_contact=3e3, k_friction=50.0, eps_friction=0.3)
    p = Problem(X, T, np.zeros(X.shape, np.uint8), np.full(n_e, mu), np.full(n_e, lam),
                np.full(n_e, 1e4), _random_fd(rng, n_e, dim), np.ones(n_e), sc, model=model)
    return p, rng


@pytest.mark.parametrize("model", ALT)
@pytest.mark.parametrize("dim", [2, 3])
def test_model_gradient_hessian_vs_finite_differences(model, dim):
    p, rng = _strip(dim, model, 110 + dim)
    a = rng.uniform(0.7, 1.0, p.mesh.n_e)
    x0 = p.mesh.X + 0.05 * rng.normal(size=p.mesh.X.shape)
    x0[:, 1] -= 0.1
    v0 = rng.normal(size=x0.shape)
    x = x0 + 0.1 * rng.normal(size=x0.shape)
    G = p.grad(x, x0, v0, a)
    u = rng.normal(size=x.shape)
    eps = 1e-6
    fd = (p.energy(x + eps * u, x0, v0, a) - p.energy(x - eps * u, x0, v0, a)) / (2 * eps)
    assert fd == pytest.approx(np.sum(G * u), rel=1e-7, abs=1e-9)
    H = p.hessian(x, x0, a)
    fdH = (p.grad(x + eps * u, x0, v0, a) - p.grad(x - eps * u, x0, v0, a)) / (2 * eps)
    assert np.allclose((H @ u.ravel()).reshape(x.shape), fdH, rtol=1e-6, atol=1e-6 * np.abs(fdH).max())
    assert abs(H - H.T).max() <= 1e-11 * abs(H).max()


@pytest.mark.parametrize("model", ALT)
def test_model_step_converges_and_vjp_matches_fd(model):
    """Newton reaches the FP64 floor on a contact step, and the Lame-pair cotangents of Eq. 9
    match finite differences of whole solves."""
    p, rng = _strip(2, model, 120)
    a = rng.uniform(0.7, 1.0, p.mesh.n_e)
    x0 = p.mesh.X - np.array([0.0, 0.02])
    v0 = 0.3 * rng.normal(size=x0.shape)
    x1, _, st = solve.step(p, x0, v0, a, tol=1e-13)
    assert st["converged"]
    xbar = rng.normal(size=x1.shape)
    wv = solve.adjoint(p, x1, x0, a, xbar)
    out = solve.vjp_params(p, wv, x1, x0, a)
    for key, attr in (("mu_bar", "mu"), ("lam_bar", "lam")):
        for e in (0, 5):
            vals = []
            for sgn in (1, -1):
                arr = getattr(p, attr).copy()
                base = arr[e]
                arr[e] = base * (1 + sgn * 1e-6)
                setattr(p, attr, arr)
                xs, _, _ = solve.step(p, x0, v0, a, tol=1e-14)
                vals.append(float(np.sum(xbar * xs)))
                arr[e] = base
                setattr(p, attr, arr)
            fd = (vals[0] - vals[1]) / (2e-6 * getattr(p, attr)[e])
            assert out[key][e] == pytest.approx(fd, rel=1e-5, abs=1e-10)
