"""GPU parity of the alternative isotropic element energies (St. Venant-Kirchhoff, corotated,
stable neo-Hookean; Sec. 3) against the FP64 oracle through the C ABI: single evaluations in the
atomic and patch scatter modes, the Lame-pair VJPs, and the plain and batched step and adjoint.

Mixed precision is held to the 1e-5 bar for the step and for the adjoint, which solves with the FP32
operator (the error then follows the conditioning of H(x1): about 1e-7 on these triangles, 1e-6 on
these tetrahedra, for every model), in the 2-norm and in the worst entry."""
import numpy as np
import pytest

from oracle import fem, solve
from tests.gpu_util import abs_assembly, problems, rand_workload, rel, rel_inf

pytestmark = pytest.mark.gpu

MODELS = ["stvk", "corot", "snh"]


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _ctx(w, precision="fp64", scatter=0, solver=0):
    from paper_2102_05791_amd import Context
    return Context.from_workload(w, precision=precision, scatter=scatter, solver=solver)


def _workload(dim, model, seed, bodies=1, shape=None):
    w, rng = rand_workload(dim, seed=seed, bodies=bodies, shape=shape)
    w.model = model
    return w, rng


def _state(w, rng):
    return w.x0 + 0.05 * rng.normal(size=w.x0.shape)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_model_gradient_energy_vjp_parity_fp64(model, dim):
    w, rng = _workload(dim, model, 51)
    ctx = _ctx(w)
    from paper_2102_05791_amd import isb
    assert ctx.get_option(isb.OPT_ENERGY) == isb.ENERGY[model]
    p = problems(w)[0]
    assert p.model == model
    x = _state(w, rng)
    a = w.actions[0]
    G = ctx.gradient(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    E = ctx.energy(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    assert rel(G, p.grad(x, w.x0, w.v0, a), abs_assembly(p, x, w.x0, w.v0, a)) <= 1e-12
    assert rel_inf(G, p.grad(x, w.x0, w.v0, a), abs_assembly(p, x, w.x0, w.v0, a)) <= 1e-12
    ee, ev = p.energy_terms(x, w.x0, w.v0, a)
    assert abs(E[0] - (ee.sum() + ev.sum())) <= 1e-13 * (np.abs(ee).sum() + np.abs(ev).sum())
    wv = rng.normal(size=x.shape)
    out = {k: v.cpu().numpy() for k, v in ctx.vjp_params(_dev(wv), _dev(x), _dev(w.x0), _dev(a)).items()}
    ref = solve.vjp_params(p, wv, x, w.x0, a)
    for k in ("a_bar", "mu_bar", "lam_bar", "kf_bar", "x0_bar", "v0_bar"):
        assert rel(out[k], ref[k]) <= 1e-12, k
        assert rel_inf(out[k], ref[k]) <= 1e-12, k


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_model_hessvec_hessdiag_parity(model, dim, precision, tol):
    w, rng = _workload(dim, model, 52)
    ctx = _ctx(w, precision=precision)
    p = problems(w)[0]
    x = _state(w, rng)
    a = w.actions[1]
    pv = rng.normal(size=x.shape)
    Hp = ctx.hessvec(_dev(x), _dev(w.x0), _dev(a), _dev(pv)).cpu().numpy()
    Hd = ctx.hessdiag(_dev(x), _dev(w.x0), _dev(a)).cpu().numpy()
    H = p.hessian(x, w.x0, a)
    ref = H @ pv.ravel()
    assert rel(Hp.ravel(), ref, abs(H) @ np.abs(pv.ravel())) <= tol
    assert rel_inf(Hp.ravel(), ref, abs(H) @ np.abs(pv.ravel())) <= tol
    assert rel(Hd.ravel(), H.diagonal()) <= 1e-12
    assert rel_inf(Hd.ravel(), H.diagonal()) <= 1e-12


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("dim,shape", [(2, (130, 65)), (3, (16, 16, 11))], ids=["2d-16900", "3d-16896"])
def test_model_patch_scatter_large_mesh(model, dim, shape):
    """Bodies of >= 16,384 elements take the LDS-staged patch scatter."""
    w, rng = _workload(dim, model, 53, shape=shape)
    ctx = _ctx(w, scatter=2)
    p = problems(w)[0]
    x = _state(w, rng)
    a = w.actions[0]
    pv = rng.normal(size=x.shape)
    G = ctx.gradient(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    assert rel(G, p.grad(x, w.x0, w.v0, a), abs_assembly(p, x, w.x0, w.v0, a)) <= 1e-12
    assert rel_inf(G, p.grad(x, w.x0, w.v0, a), abs_assembly(p, x, w.x0, w.v0, a)) <= 1e-12
    hp = _dev(np.zeros_like(x))
    ctx.hessvec_elements(_dev(x), _dev(a), _dev(pv), hp)
    K = p.s_pot * fem.element_hessians(p.mesh, x, p.mu, p.lam, p.kf, a, p.fd, model)
    nd = (dim + 1) * dim
    loc = np.einsum("eij,ej->ei", K, pv[p.mesh.T].reshape(-1, nd)).reshape(-1, dim + 1, dim)
    ref = np.zeros_like(x)
    np.add.at(ref, p.mesh.T, loc)
    assert rel(hp.cpu().numpy(), ref) <= 1e-12
    assert rel_inf(hp.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("solver", [0, 1], ids=["plain", "batched"])
@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)], ids=["fp64", "mixed"])
def test_model_step_adjoint_parity(solver, model, dim, precision, tol):
    shape = (10, 3) if dim == 2 else (3, 3, 2)
    w, rng = _workload(dim, model, 54, bodies=3, shape=shape)
    w.scene.update(tol_rel=1e-13, adj_tol_rel=1e-13, max_newton=60, max_cg=4000)
    ctx = _ctx(w, precision=precision, solver=solver)
    a = w.actions[0]
    x1, v1, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(a))
    x1, v1 = x1.cpu().numpy(), v1.cpu().numpy()
    xs = []
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        xr, vr, _ = solve.step(p, w.x0[sv], w.v0[sv], a[se], tol=1e-13)
        xs.append(xr)
        print(b, model, "gpu", st[b])
        assert rel(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= tol
        assert rel_inf(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= tol
        assert rel(v1[sv], vr) <= tol
        assert rel_inf(v1[sv], vr) <= tol
    xs = np.concatenate(xs)
    xbar = rng.normal(size=xs.shape)
    vbar = rng.normal(size=xs.shape)
    wg, st, _ = ctx.solve_adjoint(_dev(xs), _dev(w.x0), _dev(a), _dev(xbar), _dev(vbar))
    wg = wg.cpu().numpy()
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        wr = solve.adjoint(p, xs[sv], w.x0[sv], a[se], xbar[sv], vbar[sv])
        print(b, model, "adjoint err", rel(wg[sv], wr), rel_inf(wg[sv], wr))
        assert rel(wg[sv], wr) <= tol
        assert rel_inf(wg[sv], wr) <= tol


def test_model_option_errors():
    from paper_2102_05791_amd import IsbError, isb
    w, _ = _workload(2, "stvk", 55, shape=(6, 2))
    ctx = _ctx(w, solver=1)
    with pytest.raises(IsbError) as e:
        ctx.set_option(isb.OPT_ENERGY, 7)
    assert e.value.status == isb.ISB_E_ARG
    ctx.set_option(isb.OPT_BLOCK, 512)   # not the default size of triangles: no kernel for this model
    with pytest.raises(IsbError) as e:
        ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0]))
    assert e.value.status == isb.ISB_E_ARG
    ctx.set_option(isb.OPT_BLOCK, 0)
    x1, _, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0]))
    assert all(s["flags"] & 1 for s in st)
