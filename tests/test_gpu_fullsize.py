"""Full-size runs in the benchmark's launch configuration, checked on sampled outputs that the
oracle computes one body at a time (the batched-strips workload: 512 bodies, 1,541,840 triangles)."""
import numpy as np
import pytest

from oracle import solve
from oracle.fem import Problem
from synth import scenes

pytestmark = pytest.mark.gpu

SAMPLE = (0, 1, 137, 256, 400, 511)


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def batch():
    return scenes.batched_strips(512, steps=2)


@pytest.mark.parametrize("precision,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
def test_batched_strips_full_size_sampled(batch, precision, tol):
    from paper_2102_05791_amd import Context
    w = batch
    w.scene.update(tol_rel=1e-13, adj_tol_rel=1e-13, max_newton=80, max_cg=4000)
    ctx = Context.from_workload(w, precision=precision, solver=1)
    a = w.actions[0]
    x1, v1, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(a))
    x1 = x1.cpu().numpy()
    v1 = v1.cpu().numpy()
    assert all(s["flags"] & 3 for s in st)
    # adjoint of the batch loss at the GPU's own x1; references use the oracle's x1 per body
    m = ctx.mass().cpu().numpy()
    body = np.repeat(np.arange(w.n_bodies), np.diff(w.body_v_off))
    msum = np.bincount(body, weights=m)
    xbar = np.zeros_like(x1)
    xbar[:, 0] = -m / msum[body]
    wg, sta, _ = ctx.solve_adjoint(_dev(x1), _dev(w.x0), _dev(a), _dev(xbar))
    out = ctx.vjp_params(wg, _dev(x1), _dev(w.x0), _dev(a))
    wg = wg.cpu().numpy()
    abar = out["a_bar"].cpu().numpy()
    for b in SAMPLE:
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        xr, vr, sr = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=1e-13)
        ex = np.linalg.norm(x1[sv] - xr) / np.linalg.norm(xr - wb.x0)
        ev = np.linalg.norm(v1[sv] - vr) / np.linalg.norm(vr)
        wr = solve.adjoint(p, xr, wb.x0, wb.actions[0], xbar[sv])
        ar = solve.vjp_params(p, wr, xr, wb.x0, wb.actions[0])["a_bar"]
        ew = np.linalg.norm(wg[sv] - wr) / np.linalg.norm(wr)
        ea = np.linalg.norm(abar[se] - ar) / np.linalg.norm(ar)
        # the worst entry, over the largest reference entry
        exi = np.max(np.abs(x1[sv] - xr)) / np.max(np.abs(xr - wb.x0))
        evi = np.max(np.abs(v1[sv] - vr)) / np.max(np.abs(vr))
        ewi = np.max(np.abs(wg[sv] - wr)) / np.max(np.abs(wr))
        eai = np.max(np.abs(abar[se] - ar)) / np.max(np.abs(ar))
        print(f"body {b} ({wb.n_e} tris): x1 {ex:.2e} v1 {ev:.2e} w {ew:.2e} a_bar {ea:.2e} "
              f"(worst entry {exi:.2e} {evi:.2e} {ewi:.2e} {eai:.2e}) "
              f"newton {st[b]['newton_iters']} cg {st[b]['cg_iters']} adj_cg {sta[b]['adj_cg_iters']}")
        assert ex <= tol and ev <= tol and ew <= tol and ea <= tol
        assert exi <= tol and evi <= tol and ewi <= tol and eai <= tol


def test_batched_strips_metric_tolerance_error_reported(batch):
    """At the benchmark's 1e-6 relative residual the step error against the tight oracle is
    reported (the solve stops at 1e-6, so parity is not gated at 1e-10 here)."""
    from paper_2102_05791_amd import Context
    w = batch
    w.scene.update(tol_rel=1e-6, adj_tol_rel=1e-6, max_newton=50, max_cg=1000)
    ctx = Context.from_workload(w, precision="mixed", solver=1)
    x1, _, st, _ = ctx.step(_dev(w.x0), _dev(w.v0), _dev(w.actions[0]))
    x1 = x1.cpu().numpy()
    errs = []
    for b in SAMPLE:
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        xr, _, _ = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=1e-13)
        errs.append(np.linalg.norm(x1[sv] - xr) / np.linalg.norm(xr - wb.x0))
        assert st[b]["res_final"] <= 1e-6 * st[b]["res0"]
    print("x1 error vs oracle at tol 1e-6:", ["%.2e" % e for e in errs])
    assert max(errs) <= 1e-4
