"""The first-order forward solver (L-BFGS with the Armijo line search; the paper's kind of forward
pass, Sec. 6) through the C ABI: its step reaches the oracle's minimiser, the adjoint at its
solution matches the one at Newton's (Eq. 9 does not depend on how the minimiser was found), and
it composes with springs and the alternative energies."""
import numpy as np
import pytest

from oracle import solve
from oracle.fem import Problem
from tests.gpu_util import problems, rand_workload, rel, rel_inf, with_springs

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _ctx(w, forward, precision="fp64", solver=0):
    from paper_2102_05791_amd import Context, isb
    ctx = Context.from_workload(w, precision=precision, solver=solver)
    ctx.set_option(isb.OPT_FORWARD, forward)
    return ctx


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lbfgs_step_reaches_oracle_minimiser(dim, precision):
    from paper_2102_05791_amd import isb
    shape = (10, 3) if dim == 2 else (3, 3, 2)
    w, rng = rand_workload(dim, seed=61, bodies=2, shape=shape)
    w.scene.update(tol_rel=1e-10, max_newton=60)
    ctx = _ctx(w, isb.FORWARD_LBFGS, precision)
    a = w.actions[0]
    x1, v1, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(a))
    x1, v1 = x1.cpu().numpy(), v1.cpu().numpy()
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        xr, vr, sr = solve.step(p, w.x0[sv], w.v0[sv], a[se], tol=1e-13)
        print(b, "lbfgs", st[b], "oracle newton", sr["newton_iters"])
        assert st[b]["flags"] & 1 and st[b]["cg_iters"] == 0
        assert st[b]["res_final"] <= 1e-10 * st[b]["res0"]
        # a 1e-10 relative gradient leaves an error of about cond(H) 1e-10 in the step
        assert rel(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= 1e-7
        assert rel_inf(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= 1e-7
        assert rel(v1[sv], vr) <= 1e-7
        assert rel_inf(v1[sv], vr) <= 1e-7


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lbfgs_step_tight_at_the_fp64_bar(dim, precision):
    """Solved to a 1e-13 relative gradient, the L-BFGS step lands on the oracle's minimiser at the
    FP64 bar of 1e-10 (the first-order solver never applies the Hessian, so its arithmetic is FP64
    in either precision mode), in the 2-norm and in the worst entry."""
    from paper_2102_05791_amd import isb
    shape = (10, 3) if dim == 2 else (3, 3, 2)
    w, rng = rand_workload(dim, seed=65, bodies=2, shape=shape)
    w.scene.update(tol_rel=1e-13, max_newton=60)
    ctx = _ctx(w, isb.FORWARD_LBFGS, precision)
    a = w.actions[0]
    x1, v1, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(a), allow_not_converged=True)
    x1, v1 = x1.cpu().numpy(), v1.cpu().numpy()
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        xr, vr, _ = solve.step(p, w.x0[sv], w.v0[sv], a[se], tol=1e-13)
        err, err_inf = rel(x1[sv] - w.x0[sv], xr - w.x0[sv]), rel_inf(x1[sv] - w.x0[sv], xr - w.x0[sv])
        print(dim, precision, b, st[b]["newton_iters"], st[b]["res_final"] / st[b]["res0"], err, err_inf)
        assert st[b]["flags"] & (isb.FLAG_CONVERGED | isb.FLAG_STAGNATED)
        assert err <= 1e-10 and err_inf <= 1e-10
        assert rel(v1[sv], vr) <= 1e-10
        assert rel_inf(v1[sv], vr) <= 1e-10


def test_lbfgs_adjoint_matches_newton_adjoint():
    from paper_2102_05791_amd import isb
    w, rng = rand_workload(2, seed=62, shape=(12, 4))
    w.scene.update(tol_rel=1e-11, adj_tol_rel=1e-12, max_newton=60, max_cg=4000)
    a = w.actions[1]
    outs = {}
    for fwd in (isb.FORWARD_NEWTON, isb.FORWARD_LBFGS):
        ctx = _ctx(w, fwd)
        x1, _, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(a))
        xbar = np.random.default_rng(0).normal(size=w.x0.shape)
        wv, _, _ = ctx.solve_adjoint(x1, _dev(w.x0), _dev(a), _dev(xbar))
        outs[fwd] = (x1.cpu().numpy(), wv.cpu().numpy(), st[0])
    (xn, wn, sn), (xl, wl, sl) = outs[isb.FORWARD_NEWTON], outs[isb.FORWARD_LBFGS]
    print("newton", sn, "lbfgs", sl)
    assert sl["newton_iters"] > sn["newton_iters"]
    assert rel(xl - w.x0, xn - w.x0) <= 1e-7
    assert rel_inf(xl - w.x0, xn - w.x0) <= 1e-7
    assert rel(wl, wn) <= 1e-6
    assert rel_inf(wl, wn) <= 1e-6


def test_lbfgs_with_springs_and_corotated_energy():
    from paper_2102_05791_amd import isb
    w, rng = rand_workload(2, seed=63, shape=(8, 3))
    w = with_springs(w, rng)
    w.model = "corot"
    w.scene.update(tol_rel=1e-10, max_newton=60)
    ctx = _ctx(w, isb.FORWARD_LBFGS)
    a = w.actions[0]
    x1, _, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(a))
    p = Problem.from_workload(w)
    xr, _, _ = solve.step(p, w.x0, w.v0, a, tol=1e-13)
    assert st[0]["flags"] & 1
    assert rel(x1.cpu().numpy() - w.x0, xr - w.x0) <= 1e-7
    assert rel_inf(x1.cpu().numpy() - w.x0, xr - w.x0) <= 1e-7


def test_lbfgs_options_and_limits():
    from paper_2102_05791_amd import IsbError, isb
    w, _ = rand_workload(2, seed=64, shape=(8, 3))
    ctx = _ctx(w, isb.FORWARD_LBFGS, solver=1)
    with pytest.raises(IsbError) as e:                      # the batched solver runs Newton only
        ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0]))
    assert e.value.status == isb.ISB_E_ARG
    for key, bad in ((isb.OPT_FORWARD, 2), (isb.OPT_LBFGS_MEMORY, 0), (isb.OPT_LBFGS_MAX_ITERS, 0)):
        with pytest.raises(IsbError):
            ctx.set_option(key, bad)
    ctx.set_option(isb.OPT_SOLVER, 0)
    ctx.set_option(isb.OPT_LBFGS_MEMORY, 3)
    ctx.set_option(isb.OPT_LBFGS_MAX_ITERS, 5)
    w.scene.update(tol_rel=1e-12)
    ctx.set_scene(w.scene)
    x1, _, st, status = ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0]), allow_not_converged=True)
    assert status == isb.ISB_E_NOT_CONVERGED and st[0]["newton_iters"] == 5
    assert np.isfinite(x1.cpu().numpy()).all()
    assert ctx.get_option(isb.OPT_LBFGS_MEMORY) == 3 and ctx.get_option(isb.OPT_FORWARD) == isb.FORWARD_LBFGS
