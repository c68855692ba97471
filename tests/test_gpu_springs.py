"""GPU parity of the vertex-pair springs (Eq. 2 between two vertices) against the FP64 oracle
through the C ABI: single evaluations in every scatter mode, the plain and batched step, adjoint
and VJPs (actions and stiffnesses), the spring strips at their real size, and the upload's error
paths."""
import numpy as np
import pytest

from oracle import fem, solve
from oracle.fem import Problem
from synth import scenes
from tests.gpu_util import abs_assembly, rand_workload, rel, rel_inf, with_springs

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _ctx(w, precision="fp64", scatter=0, solver=0):
    from paper_2102_05791_amd import Context
    return Context.from_workload(w, precision=precision, scatter=scatter, solver=solver)


def _spring_workload(dim, seed, bodies=1, shape=None, integrator="be", pinned_left=False):
    w, rng = rand_workload(dim, seed=seed, bodies=bodies, shape=shape, integrator=integrator,
                           pinned_left=pinned_left)
    return with_springs(w, rng), rng


def _tight(w):
    w.scene.update(tol_rel=1e-13, adj_tol_rel=1e-13, max_newton=60, max_cg=4000)
    return w


def _state(w, rng):
    x = w.x0 + 0.05 * rng.normal(size=w.x0.shape)
    x[w.pinned.astype(bool)] = w.x0[w.pinned.astype(bool)]
    return x


def _body_acts(w, a, b):
    """Body b's action vector (its elements' entries, then its springs')."""
    e0, e1 = w.body_e_off[b], w.body_e_off[b + 1]
    s0, s1 = w.body_s_off[b], w.body_s_off[b + 1]
    return np.concatenate([a[e0:e1], a[w.n_e + s0:w.n_e + s1]])


CASES = [(2, "be", False, 1), (2, "qs", True, 1), (3, "be", False, 1), (2, "be", False, 3)]
IDS = ["2d-be", "2d-qs-pinned", "3d-be", "2d-be-3bodies"]


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("scatter", [0, 1, 2], ids=["atomic", "colour", "patch"])
def test_spring_gradient_energy_parity_fp64(case, scatter):
    dim, integ, pin, nb = case
    w, rng = _spring_workload(dim, 41, bodies=nb, integrator=integ, pinned_left=pin)
    ctx = _ctx(w, scatter=scatter)
    assert ctx.n_s == w.n_s > 0
    x = _state(w, rng)
    a = w.actions[0]
    G = ctx.gradient(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    E = ctx.energy(_dev(x), _dev(w.x0), _dev(w.v0), _dev(a)).cpu().numpy()
    for b in range(nb):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        ab = _body_acts(w, a, b)
        assert np.array_equal(ab, wb.actions[0])
        xb = x[sv]
        Gref = p.grad(xb, wb.x0, wb.v0, ab)
        Gref[p.pinned] = 0.0
        assert rel(G[sv], Gref, abs_assembly(p, xb, wb.x0, wb.v0, ab)) <= 1e-13
        assert rel_inf(G[sv], Gref, abs_assembly(p, xb, wb.x0, wb.v0, ab)) <= 1e-13
        ee, ev = p.energy_terms(xb, wb.x0, wb.v0, ab)
        assert abs(E[b] - (ee.sum() + ev.sum())) <= 1e-13 * (np.abs(ee).sum() + np.abs(ev).sum())


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
@pytest.mark.parametrize("scatter", [0, 1, 2], ids=["atomic", "colour", "patch"])
def test_spring_hessvec_hessdiag_parity(case, precision, tol, scatter):
    dim, integ, pin, nb = case
    w, rng = _spring_workload(dim, 42, bodies=nb, integrator=integ, pinned_left=pin)
    ctx = _ctx(w, precision=precision, scatter=scatter)
    x = _state(w, rng)
    a = w.actions[1]
    pv = rng.normal(size=x.shape)
    Hp = ctx.hessvec(_dev(x), _dev(w.x0), _dev(a), _dev(pv)).cpu().numpy()
    Hd = ctx.hessdiag(_dev(x), _dev(w.x0), _dev(a)).cpu().numpy()
    for b in range(nb):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        H = p.hessian(x[sv], wb.x0, wb.actions[1])
        free = p.free
        pm = pv[sv].ravel() * free
        ref = (H @ pm) * free
        absref = (abs(H) @ np.abs(pm)) * free
        assert rel(Hp[sv].ravel(), ref, absref) <= tol
        assert rel_inf(Hp[sv].ravel(), ref, absref) <= tol
        # the diagonal is FP64 in both precisions
        assert rel(Hd[sv].ravel(), np.where(free, H.diagonal(), 1.0)) <= 1e-12
        assert rel_inf(Hd[sv].ravel(), np.where(free, H.diagonal(), 1.0)) <= 1e-12


def test_spring_hessvec_elements_includes_springs():
    """isb_hessvec_elements adds the springs' blocks besides the elements' (no vertex terms)."""
    w, rng = _spring_workload(2, 43)
    ctx = _ctx(w)
    x = _state(w, rng)
    a = w.actions[0]
    pv = rng.normal(size=x.shape)
    import torch
    hp = torch.zeros(w.n_v, 2, dtype=torch.float64, device="cuda:0")
    ctx.hessvec_elements(_dev(x), _dev(a), _dev(pv), hp)
    p = Problem.from_workload(w)
    sc = dict(w.scene, k_contact=0.0, k_friction=0.0)
    q = Problem(w.X, w.T, np.zeros_like(w.pinned), w.mu, w.lam, w.kf, w.fdir, w.rho, dict(sc, integrator="qs"),
                w.S, w.ks)
    ref = p.s_pot * (q.hessian(x, w.x0, a) @ pv.ravel())
    assert rel(hp.cpu().numpy().ravel(), ref) <= 1e-12
    assert rel_inf(hp.cpu().numpy().ravel(), ref) <= 1e-12
    # isb_gradient_elements: the element and spring forces alone, added into g
    g = torch.ones(w.n_v, 2, dtype=torch.float64, device="cuda:0")
    ctx.gradient_elements(_dev(x), _dev(a), g)
    ae, as_ = p.split(a)
    gref = 1.0 + p.s_pot * (p.element_grad(x, ae) + fem.spring_grad(x, p.S, p.ks, p.l0, as_))
    assert rel(g.cpu().numpy(), gref) <= 1e-13
    assert rel_inf(g.cpu().numpy(), gref) <= 1e-13


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_spring_vjp_parity_fp64(case):
    dim, integ, pin, nb = case
    w, rng = _spring_workload(dim, 44, bodies=nb, integrator=integ, pinned_left=pin)
    ctx = _ctx(w)
    x1 = _state(w, rng)
    a = w.actions[2]
    wv = rng.normal(size=x1.shape)
    wv[w.pinned.astype(bool)] = 0.0
    vbar = rng.normal(size=x1.shape)
    out = {k: v.cpu().numpy() for k, v in ctx.vjp_params(_dev(wv), _dev(x1), _dev(w.x0), _dev(a), _dev(vbar)).items()}
    kb = ctx.vjp_spring_stiffness(_dev(wv), _dev(x1), _dev(a)).cpu().numpy()
    assert out["a_bar"].shape == (w.n_e + w.n_s,)
    for b in range(nb):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        ref = solve.vjp_params(p, wv[sv], x1[sv], wb.x0, wb.actions[2], v1_bar=vbar[sv])
        assert rel(_body_acts(w, out["a_bar"], b), ref["a_bar"]) <= 1e-12
        assert rel_inf(_body_acts(w, out["a_bar"], b), ref["a_bar"]) <= 1e-12
        assert rel(kb[w.body_s_off[b]:w.body_s_off[b + 1]], ref["ks_bar"]) <= 1e-12
        assert rel_inf(kb[w.body_s_off[b]:w.body_s_off[b + 1]], ref["ks_bar"]) <= 1e-12
        for k in ("x0_bar",) + (("v0_bar",) if integ == "be" else ()):
            assert rel(out[k][sv], ref[k]) <= 1e-12, k
            assert rel_inf(out[k][sv], ref[k]) <= 1e-12, k


@pytest.mark.parametrize("solver", [0, 1], ids=["plain", "batched"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_spring_step_adjoint_vjp_parity(solver, dim, precision, tol):
    shape = (10, 3) if dim == 2 else (3, 3, 2)
    w, rng = _spring_workload(dim, 45, bodies=3, shape=shape)
    w = _tight(w)
    ctx = _ctx(w, precision=precision, solver=solver)
    a = w.actions[0]
    x1, v1, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(a))
    x1, v1 = x1.cpu().numpy(), v1.cpu().numpy()
    xs = []
    for b in range(w.n_bodies):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        xr, vr, _ = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=1e-13)
        xs.append(xr)
        print(b, "gpu", st[b])
        assert rel(x1[sv] - wb.x0, xr - wb.x0) <= tol
        assert rel(v1[sv], vr) <= tol
        assert rel_inf(x1[sv] - wb.x0, xr - wb.x0) <= tol
        assert rel_inf(v1[sv], vr) <= tol
        ee, ev = p.energy_terms(xr, wb.x0, wb.v0, wb.actions[0])
        assert st[b]["energy"] == pytest.approx(ee.sum() + ev.sum(), rel=1e-8)
    # adjoint and VJP at the oracle's x1, so that only they are compared
    xs = np.concatenate(xs)
    xbar = rng.normal(size=xs.shape)
    vbar = rng.normal(size=xs.shape)
    wg, st, _ = ctx.solve_adjoint(_dev(xs), _dev(w.x0), _dev(a), _dev(xbar), _dev(vbar))
    wg = wg.cpu().numpy()
    abar = ctx.vjp_params(_dev(wg), _dev(xs), _dev(w.x0), _dev(a), _dev(vbar), want=("a_bar",))["a_bar"].cpu().numpy()
    for b in range(w.n_bodies):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        wr = solve.adjoint(p, xs[sv], wb.x0, wb.actions[0], xbar[sv], vbar[sv])
        assert rel(wg[sv], wr) <= tol
        assert rel_inf(wg[sv], wr) <= tol
        ref = solve.vjp_params(p, wr, xs[sv], wb.x0, wb.actions[0], v1_bar=vbar[sv])
        assert rel(_body_acts(w, abar, b), ref["a_bar"]) <= tol
        assert rel_inf(_body_acts(w, abar, b), ref["a_bar"]) <= tol


def test_spring_colour_scatter_is_bitwise_reproducible():
    w, _ = _spring_workload(2, 46)
    ctx = _ctx(w, scatter=1)
    outs = []
    for _ in range(2):
        x1, v1, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0]))
        outs.append((x1.cpu().numpy(), v1.cpu().numpy(), st[0]["newton_iters"], st[0]["cg_iters"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2:] == outs[1][2:]


@pytest.mark.parametrize("solver,precision,tol", [(0, "fp64", 1e-10), (1, "fp64", 1e-10), (1, "mixed", 1e-5)],
                         ids=["plain-fp64", "batched-fp64", "batched-mixed"])
def test_spring_strip_full_size(solver, precision, tol):
    """The 64x16 spring strip (2048 passive triangles, 1088 springs) over two steps."""
    w = scenes.be_spring_strip(steps=2)
    w = _tight(w)
    ctx = _ctx(w, precision=precision, solver=solver)
    p = Problem.from_workload(w)
    x, v = w.x0, w.v0
    xg, vg = _dev(w.x0), _dev(w.v0)
    for t in range(2):
        xg, vg, st, _ = ctx.step(xg, vg, _dev(w.actions[t]))
        x, v, _ = solve.step(p, x, v, w.actions[t], tol=1e-13)
        assert rel(xg.cpu().numpy() - w.x0, x - w.x0) <= tol
        assert rel(vg.cpu().numpy(), v) <= tol
        assert rel_inf(xg.cpu().numpy() - w.x0, x - w.x0) <= tol
        assert rel_inf(vg.cpu().numpy(), v) <= tol


def test_batched_spring_strips_sampled_bodies():
    """Batched spring strips (64 bodies of U{4..32} scale) in one launch, at the bench's tolerance;
    sampled bodies against the oracle, all bodies converged."""
    sizes = scenes.batched_sizes(64)
    w = scenes.batched_spring_strips(64, steps=1, sizes=sizes)
    ctx = _ctx(w, precision="mixed", solver=1)
    x1, v1, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0]))
    x1 = x1.cpu().numpy()
    assert all(s["flags"] & 1 for s in st)
    for b in (0, int(np.argmax(sizes)), 63):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        xr, _, _ = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=1e-13)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        # a 1e-6 relative residual leaves an error of the same order in the step
        assert rel(x1[sv] - wb.x0, xr - wb.x0) <= 1e-4
        assert rel_inf(x1[sv] - wb.x0, xr - wb.x0) <= 1e-4


def test_spring_upload_errors_and_action_length():
    from paper_2102_05791_amd import IsbError, isb
    w, rng = _spring_workload(2, 47, bodies=2, shape=(6, 2))
    ctx = _ctx(w)
    S, ks, so = w.S.copy(), w.ks.copy(), w.body_s_off.copy()
    bad = S.copy()
    bad[0] = (int(w.body_v_off[1]), int(w.body_v_off[1]) + 1)   # body 0's spring joining body 1's vertices
    with pytest.raises(IsbError) as e:
        ctx.spring_upload(bad, ks, so)
    assert e.value.status == isb.ISB_E_MESH
    bad = S.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(IsbError) as e:
        ctx.spring_upload(bad, ks, so)
    assert e.value.status == isb.ISB_E_MESH
    kneg = ks.copy()
    kneg[1] = -1.0
    with pytest.raises(IsbError) as e:
        ctx.spring_upload(S, kneg, so)
    assert e.value.status == isb.ISB_E_ARG
    with pytest.raises(IsbError) as e:
        ctx.spring_upload(S, ks, None)                              # two bodies need the offsets
    assert e.value.status == isb.ISB_E_ARG
    # a failed upload keeps the previous springs; the action vector must cover them
    assert ctx.n_s == w.n_s
    with pytest.raises(ValueError):
        ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0][:w.n_e]))
    a = w.actions[0].copy()
    a[w.n_e + 2] = 0.0                                              # a spring action must be > 0 too
    with pytest.raises(IsbError) as e:
        ctx.step(_dev(w.x0), _dev(w.v0), _dev(a))
    assert e.value.status == isb.ISB_E_ARG
    # removing the springs brings back the element-only action vector
    ctx.spring_upload(np.zeros((0, 2), np.int32), np.zeros(0), np.zeros(3, np.int64))
    assert ctx.n_s == 0
    x1, _, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0][:w.n_e]))
    assert all(s["flags"] & 1 for s in st)
