"""GPU parity of the single evaluations (energy, gradient, Hessian-vector product, Hessian
diagonal, parameter VJP) against the FP64 oracle at identical inputs, through the C ABI."""
import numpy as np
import pytest

from oracle import solve
from tests.gpu_util import abs_assembly, problems, rand_workload, rel, rel_inf

pytestmark = pytest.mark.gpu

CASES = [(2, "be", False, 1), (2, "qs", True, 1), (3, "be", False, 1), (2, "be", False, 3)]
IDS = ["2d-be", "2d-qs-pinned", "3d-be", "2d-be-3bodies"]


def _ctx(w, precision="fp64", scatter=0):
    from paper_2102_05791_amd import Context
    return Context.from_workload(w, precision=precision, scatter=scatter)


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _state(w, rng):
    x = w.x0 + 0.05 * rng.normal(size=w.x0.shape)
    x[w.pinned.astype(bool)] = w.x0[w.pinned.astype(bool)]
    return x


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("scatter", [0, 1, 2], ids=["atomic", "colour", "patch"])
def test_gradient_energy_parity_fp64(case, scatter):
    dim, integ, pin, nb = case
    w, rng = rand_workload(dim, seed=1, integrator=integ, pinned_left=pin, bodies=nb)
    ctx = _ctx(w, scatter=scatter)
    x = _state(w, rng)
    a = w.actions[0]
    G = ctx.gradient(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    E = ctx.energy(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    for b, p in enumerate(problems(w)):
        v0, v1 = w.body_v_off[b], w.body_v_off[b + 1]
        e0, e1 = w.body_e_off[b], w.body_e_off[b + 1]
        xb, x0b, vb, ab = x[v0:v1], w.x0[v0:v1], w.v0[v0:v1], a[e0:e1]
        Gref = p.grad(xb, x0b, vb, ab)
        Gref[p.pinned] = 0.0
        scale = abs_assembly(p, xb, x0b, vb, ab)
        assert rel(G[v0:v1], Gref, scale) <= 1e-13
        assert rel_inf(G[v0:v1], Gref, scale) <= 1e-13
        ee, ev = p.energy_terms(xb, x0b, vb, ab)
        assert abs(E[b] - (ee.sum() + ev.sum())) <= 1e-13 * (np.abs(ee).sum() + np.abs(ev).sum())


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
@pytest.mark.parametrize("scatter", [0, 1, 2], ids=["atomic", "colour", "patch"])
def test_hessvec_hessdiag_parity(case, precision, tol, scatter):
    dim, integ, pin, nb = case
    w, rng = rand_workload(dim, seed=2, integrator=integ, pinned_left=pin, bodies=nb)
    ctx = _ctx(w, precision=precision, scatter=scatter)
    x = _state(w, rng)
    a = w.actions[1]
    pv = rng.normal(size=x.shape)
    Hp = ctx.hessvec(_dev(x), _dev(w.x0), _dev(a), _dev(pv)).cpu().numpy()
    Hd = ctx.hessdiag(_dev(x), _dev(w.x0), _dev(a)).cpu().numpy()
    for b, p in enumerate(problems(w)):
        v0, v1 = w.body_v_off[b], w.body_v_off[b + 1]
        e0, e1 = w.body_e_off[b], w.body_e_off[b + 1]
        H = p.hessian(x[v0:v1], w.x0[v0:v1], a[e0:e1])
        free = p.free
        pm = pv[v0:v1].ravel() * free
        ref = (H @ pm) * free
        absref = (abs(H) @ np.abs(pm)) * free
        assert rel(Hp[v0:v1].ravel(), ref, absref) <= tol
        assert rel_inf(Hp[v0:v1].ravel(), ref, absref) <= tol
        dref = np.where(free, H.diagonal(), 1.0)
        assert rel(Hd[v0:v1].ravel(), dref) <= tol
        assert rel_inf(Hd[v0:v1].ravel(), dref) <= tol


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_vjp_parity_fp64(case):
    dim, integ, pin, nb = case
    w, rng = rand_workload(dim, seed=3, integrator=integ, pinned_left=pin, bodies=nb)
    ctx = _ctx(w)
    x1 = _state(w, rng)
    a = w.actions[2]
    wv = rng.normal(size=x1.shape)
    wv[w.pinned.astype(bool)] = 0.0
    vbar = rng.normal(size=x1.shape)
    out = ctx.vjp_params(_dev(wv), _dev(x1), _dev(w.x0), _dev(a), _dev(vbar))
    out = {k: v.cpu().numpy() for k, v in out.items()}
    for b, p in enumerate(problems(w)):
        v0, v1 = w.body_v_off[b], w.body_v_off[b + 1]
        e0, e1 = w.body_e_off[b], w.body_e_off[b + 1]
        ref = solve.vjp_params(p, wv[v0:v1], x1[v0:v1], w.x0[v0:v1], a[e0:e1], v1_bar=vbar[v0:v1])
        for k in ("a_bar", "mu_bar", "lam_bar", "kf_bar"):
            assert rel(out[k][e0:e1], ref[k]) <= 1e-12, k
            assert rel_inf(out[k][e0:e1], ref[k]) <= 1e-12, k
        for k in ("x0_bar", "v0_bar"):
            if integ == "qs" and k == "v0_bar":
                assert np.all(out[k][v0:v1] == 0.0)
                continue
            assert rel(out[k][v0:v1], ref[k]) <= 1e-12, k
            assert rel_inf(out[k][v0:v1], ref[k]) <= 1e-12, k


def test_mass_matches_oracle():
    w, _ = rand_workload(3, seed=4)
    ctx = _ctx(w, scatter=1)
    m = ctx.mass().cpu().numpy()
    ref = problems(w)[0].mesh.mass
    assert rel(m, ref) <= 1e-15
    assert rel_inf(m, ref) <= 1e-15


@pytest.mark.parametrize("order", ["given", "wave"])
@pytest.mark.parametrize("dim,shape", [(2, (130, 65)), (3, (16, 16, 11))], ids=["2d-16900", "3d-16896"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_patch_scatter_large_mesh(dim, shape, precision, tol, order):
    """Meshes above the patch threshold take the LDS-staged patch scatter (isb scatter mode 2), in
    the elements' given order and in the order isb_wave_order gives them."""
    from paper_2102_05791_amd import isb
    w, rng = rand_workload(dim, seed=6, shape=shape)
    assert w.n_e >= 16384
    if order == "wave":
        w = w.permute_elements(isb.wave_order(dim, w.n_v, w.T, w.body_e_off))
    ctx = _ctx(w, precision=precision, scatter=2)
    x = _state(w, rng)
    a = w.actions[0]
    pv = rng.normal(size=x.shape)
    p = problems(w)[0]
    G = ctx.gradient(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    Gref = p.grad(x, w.x0, w.v0, a)
    assert rel(G, Gref, abs_assembly(p, x, w.x0, w.v0, a)) <= 1e-13
    assert rel_inf(G, Gref, abs_assembly(p, x, w.x0, w.v0, a)) <= 1e-13
    H = p.hessian(x, w.x0, a)
    Hp = ctx.hessvec(_dev(x), _dev(w.x0), _dev(a), _dev(pv)).cpu().numpy().ravel()
    assert rel(Hp, H @ pv.ravel(), abs(H) @ np.abs(pv.ravel())) <= tol
    assert rel_inf(Hp, H @ pv.ravel(), abs(H) @ np.abs(pv.ravel())) <= tol
    Hd = ctx.hessdiag(_dev(x), _dev(w.x0), _dev(a)).cpu().numpy().ravel()
    assert rel(Hd, H.diagonal()) <= tol
    assert rel_inf(Hd, H.diagonal()) <= tol
    he = ctx.hessvec_elements(_dev(x), _dev(a), _dev(pv), _dev(np.zeros_like(x))).cpu().numpy().ravel()
    Hv_vertex = _elem_free_hessian(p, x, w.x0, a) @ pv.ravel()
    assert rel(he, H @ pv.ravel() - Hv_vertex, abs(H) @ np.abs(pv.ravel())) <= tol
    assert rel_inf(he, H @ pv.ravel() - Hv_vertex, abs(H) @ np.abs(pv.ravel())) <= tol


def _elem_free_hessian(p, x, x0, a):
    """The assembled Hessian with the element terms removed (vertex terms only)."""
    import scipy.sparse as sp
    from oracle import fem
    K = p.s_pot * fem.element_hessians(p.mesh, x, p.mu, p.lam, p.kf, a, p.fd)
    d = p.mesh.d
    dofs = (p.mesh.T[:, :, None] * d + np.arange(d)[None, None, :]).reshape(p.mesh.n_e, -1)
    rows = np.repeat(dofs, dofs.shape[1], axis=1).ravel()
    cols = np.tile(dofs, (1, dofs.shape[1])).ravel()
    n = p.mesh.n_v * d
    return p.hessian(x, x0, a) - sp.coo_matrix((K.ravel(), (rows, cols)), shape=(n, n)).tocsr()


@pytest.mark.parametrize("scatter", [0, 2], ids=["atomic", "patch"])
@pytest.mark.parametrize("dim,shape", [(2, (130, 65)), (3, (16, 16, 11))], ids=["2d", "3d"])
def test_mixed_hessvec_smooth_operand(dim, shape, scatter):
    """p = large constant + small smooth field: the element sees only differences of p, which must
    be formed in FP64 before rounding to the FP32 element precision (cancellation otherwise)."""
    w, rng = rand_workload(dim, seed=7, shape=shape)
    ctx = _ctx(w, precision="mixed", scatter=scatter)
    x = _state(w, rng)
    a = w.actions[0]
    pv = 1e3 + 1e-2 * np.sin(w.X @ np.arange(1, dim + 1) * 0.1)[:, None] * np.ones((1, dim))
    he = ctx.hessvec_elements(_dev(x), _dev(a), _dev(pv), _dev(np.zeros_like(x))).cpu().numpy().ravel()
    p = problems(w)[0]
    Hp = (p.hessian(x, w.x0, a) - _elem_free_hessian(p, x, w.x0, a)) @ pv.ravel()
    scale = abs(p.hessian(x, w.x0, a) - _elem_free_hessian(p, x, w.x0, a)) @ np.abs(pv - pv.mean()).ravel()
    assert rel(he, Hp, scale) <= 1e-5
    assert rel_inf(he, Hp, scale) <= 1e-5
