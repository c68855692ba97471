"""CPU tests of the batched persistent solver's body logic (isb_body.hpp) run by host threads
as one emulated workgroup, against the FP64 oracle. Covers the control flow (static body
assignment, Newton / CG / line-search loops, adjoint) without a GPU."""
import numpy as np
import pytest

from oracle import solve
from tests.gpu_util import problems, rand_workload, rel


@pytest.fixture(scope="module")
def emu_mod():
    from tests.emu import emu
    try:
        emu.build()
    except Exception as e:  # pragma: no cover
        pytest.skip(f"g++ emulator build failed: {e}")
    return emu


def _tight(w):
    w.scene.update(tol_rel=1e-13, adj_tol_rel=1e-13, max_newton=60, max_cg=4000)
    return w


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_emulated_batched_step_and_adjoint(emu_mod, precision, tol):
    w, rng = rand_workload(2, seed=21, bodies=3, shape=(5, 2))
    w = _tight(w)
    eb = emu_mod.EmuBatch(w, precision)
    a = w.actions[0]
    x1, v1, st = eb.step(w.x0, w.v0, a, block=64)
    assert np.all(st["flags"] & 1)
    xs = []
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        xr, vr, _ = solve.step(p, w.x0[sv], w.v0[sv], a[se], tol=1e-13)
        xs.append(xr)
        assert rel(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= tol
        assert rel(v1[sv], vr) <= tol
    xs = np.concatenate(xs)
    xbar = rng.normal(size=xs.shape)
    vbar = rng.normal(size=xs.shape)
    wv, st = eb.adjoint(xs, w.x0, a, xbar, vbar, block=64)
    assert np.all(st["flags"] & 8)
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        wr = solve.adjoint(p, xs[sv], w.x0[sv], a[se], xbar[sv], vbar[sv])
        assert rel(wv[sv], wr) <= tol


def test_emulated_static_assignment_covers_every_body_once(emu_mod):
    """With more bodies than rounds x workgroups boundaries, every body is solved exactly once."""
    w, _ = rand_workload(2, seed=22, bodies=5, shape=(3, 2))
    eb = emu_mod.EmuBatch(w, "fp64")
    x1, v1, st = eb.step(w.x0, w.v0, w.actions[0], block=64)
    assert np.all(st["newton_iters"] > 0) and np.all(st["flags"] & 1)
    assert np.all(x1 != 0.0)
