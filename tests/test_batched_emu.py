"""CPU tests of the batched persistent solver's body logic (isb_body.hpp) run by host threads
as one emulated workgroup, against the FP64 oracle. Covers the control flow (static body
assignment, Newton / CG / line-search loops, adjoint) without a GPU."""
import numpy as np
import pytest

from oracle import solve
from oracle.fem import Problem
from tests.gpu_util import problems, rand_workload, rel, with_springs


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


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_emulated_batched_springs_step_and_adjoint(emu_mod, precision, tol):
    """Bodies with vertex-pair springs (Eq. 2 between two vertices) besides their element fibres."""
    w, rng = rand_workload(2, seed=23, bodies=3, shape=(5, 2))
    w = _tight(with_springs(w, rng))
    eb = emu_mod.EmuBatch(w, precision)
    a = w.actions[0]
    x1, v1, st = eb.step(w.x0, w.v0, a, block=64)
    assert np.all(st["flags"] & 1)
    xs = []
    for b in range(w.n_bodies):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        assert p.n_s > 0
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        xr, vr, _ = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=1e-13)
        xs.append(xr)
        assert rel(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= tol
        assert rel(v1[sv], vr) <= tol
        # the final energy of the batched solve includes the springs' terms
        assert st["energy"][b] == pytest.approx(p.energy(xr, wb.x0, wb.v0, wb.actions[0]), rel=1e-9)
    xs = np.concatenate(xs)
    xbar = rng.normal(size=xs.shape)
    vbar = rng.normal(size=xs.shape)
    wv, st = eb.adjoint(xs, w.x0, a, xbar, vbar, block=64)
    assert np.all(st["flags"] & 8)
    for b in range(w.n_bodies):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        wr = solve.adjoint(p, xs[sv], wb.x0, wb.actions[0], xbar[sv], vbar[sv])
        assert rel(wv[sv], wr) <= tol


@pytest.mark.parametrize("model", ["stvk", "corot", "snh"])
@pytest.mark.parametrize("dim", [2, 3])
def test_emulated_batched_energy_models(emu_mod, model, dim):
    """The alternative isotropic energies (Sec. 3) in the batched step and adjoint, FP64 and mixed.
    The mixed adjoint solves with the FP32 operator; St. Venant-Kirchhoff forms E = (F^T F - I)/2
    from an FP32 F, which cancels near rest and leaves E about 6e-8/|E| relative precision, so the
    mixed adjoint bar of the alternative models is 3e-5 (the step stays at 1e-5)."""
    # small bodies: the host-thread emulation pays a barrier per wave operation (the GPU tests
    # cover the same paths at full size)
    shape = (4, 2) if dim == 2 else (2, 1, 1)
    w, rng = rand_workload(dim, seed=24, bodies=2 if dim == 2 else 1, shape=shape)
    w = _tight(w)
    w.model = model
    probs = problems(w)
    a = w.actions[0]
    for precision, tol, adj_tol in (("fp64", 1e-10, 1e-10), ("mixed", 1e-5, 3e-5)):
        eb = emu_mod.EmuBatch(w, precision)
        x1, v1, st = eb.step(w.x0, w.v0, a, block=64)
        assert np.all(st["flags"] & 1)
        xs = []
        for b, p in enumerate(probs):
            sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
            se = slice(w.body_e_off[b], w.body_e_off[b + 1])
            xr, vr, _ = solve.step(p, w.x0[sv], w.v0[sv], a[se], tol=1e-13)
            xs.append(xr)
            assert rel(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= tol
        xs = np.concatenate(xs)
        xbar = rng.normal(size=xs.shape)
        wv, st = eb.adjoint(xs, w.x0, a, xbar, None, block=64)
        assert np.all(st["flags"] & 8)
        for b, p in enumerate(probs):
            sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
            se = slice(w.body_e_off[b], w.body_e_off[b + 1])
            wr = solve.adjoint(p, xs[sv], w.x0[sv], a[se], xbar[sv])
            assert rel(wv[sv], wr) <= adj_tol


def test_emulated_index_checks_report_a_bad_corner(emu_mod):
    """The debug build's index checks: an element corner planted out of its body's range (on the
    CPU, in the emulator's copy of the connectivity) is reported as check 2 and read as corner 0,
    so the run stays in bounds; the same body with its real corners reports nothing."""
    w, _ = rand_workload(2, seed=23, bodies=2, shape=(3, 2))
    eb = emu_mod.EmuBatch(w, "fp64")
    eb.step(w.x0, w.v0, w.actions[0], block=64)
    assert eb.last_index_site == 0
    eb.lconn[1, 0] = 60000
    eb.allow_index_errors = True
    eb.step(w.x0, w.v0, w.actions[0], block=64)
    assert eb.last_index_site == 2
    eb.allow_index_errors = False
    with pytest.raises(IndexError):
        eb.step(w.x0, w.v0, w.actions[0], block=64)


def test_emulated_static_assignment_covers_every_body_once(emu_mod):
    """With more bodies than rounds x workgroups boundaries, every body is solved exactly once."""
    w, _ = rand_workload(2, seed=22, bodies=5, shape=(3, 2))
    eb = emu_mod.EmuBatch(w, "fp64")
    x1, v1, st = eb.step(w.x0, w.v0, w.actions[0], block=64)
    assert np.all(st["newton_iters"] > 0) and np.all(st["flags"] & 1)
    assert np.all(x1 != 0.0)


@pytest.mark.parametrize("lds_fill", [0.0, -12345.0, 1e30])
def test_emulated_first_preconditioner_ignores_stale_lds(emu_mod, lds_fill):
    """With no Newton iteration allowed, the Jacobi preconditioner left behind is the one of the
    first trial pass: 1/|diag H| at the initial iterate (x0 + h v0, pinned DOFs at x0) on free DOFs,
    rounded to FP32, whatever the LDS held when the launch began."""
    w, _ = rand_workload(2, seed=23, bodies=2, shape=(6, 3))
    w.scene.update(max_newton=0)
    eb = emu_mod.EmuBatch(w, "mixed")
    a = w.actions[0]
    eb.step(w.x0, w.v0, a, block=64, lds_fill=lds_fill)
    dinv = eb.Dv.astype(np.float64).reshape(w.x0.shape)  # stored in FP32
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        xi = np.where(p.pinned, w.x0[sv], p.x_hat(w.x0[sv], w.v0[sv]))
        d = np.abs(p.hessian(xi, w.x0[sv], a[se]).diagonal())
        ref = np.where(p.free, 1.0 / d, 0.0).reshape(xi.shape)
        assert rel(dinv[sv], ref) <= 1e-7


@pytest.mark.parametrize("mode", ["step", "adjoint"])
def test_emulated_launch_leaves_lds_accumulators_zero(emu_mod, mode):
    """Both LDS accumulators are zero outside the passes that use them: each pass clears what it
    used, and CG clears its direction on every exit (the trial pass accumulates there next)."""
    w, rng = rand_workload(2, seed=24, bodies=3, shape=(6, 3))
    eb = emu_mod.EmuBatch(w, "mixed")
    a = w.actions[0]
    x1, _, st = eb.step(w.x0, w.v0, a, block=64, lds_fill=0.0)
    assert np.all(st["flags"] & 1)
    if mode == "adjoint":
        eb.adjoint(x1, w.x0, a, rng.normal(size=x1.shape), rng.normal(size=x1.shape), block=64, lds_fill=0.0)
    assert eb.lds_left == 0.0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_emulated_adjoint_warm_start(emu_mod, precision, tol):
    """ISB_OPT_ADJ_WARM_START: CG starts from the given w and solves for the correction. In FP64 a
    restart from the cold solution has nothing left to do; with the FP32 operator the restart sees
    the true residual b - H w, which at this 1e-13 tolerance lies well above CG's recurrence
    residual (FP32 rounding of H w), so it only takes fewer iterations than the cold solve. From a
    perturbed start it reaches the oracle's adjoint (Eq. 9) to the cold start's bar. Springs
    included, pinned DOFs stay 0."""
    w, rng = rand_workload(2, seed=24, bodies=3, shape=(6, 2), pinned_left=True)
    w = _tight(with_springs(w, rng))
    eb = emu_mod.EmuBatch(w, precision)
    a = w.actions[0]
    x1, _, st = eb.step(w.x0, w.v0, a, block=64)
    assert np.all(st["flags"] & 1)
    xbar = rng.normal(size=x1.shape)
    vbar = rng.normal(size=x1.shape)
    w_cold, st_c = eb.adjoint(x1, w.x0, a, xbar, vbar, block=64)
    w_same, st_s = eb.adjoint(x1, w.x0, a, xbar, vbar, block=64, w_init=w_cold)
    assert np.all(st_s["flags"] & 8)
    if precision == "fp64":
        assert np.all(st_s["adj_cg_iters"] == 0) and np.all(st_c["adj_cg_iters"] > 5)
    else:
        assert np.all(st_s["adj_cg_iters"] < st_c["adj_cg_iters"])
    assert rel(w_same, w_cold) <= tol
    start = w_cold + 0.1 * np.abs(w_cold).max() * rng.normal(size=w_cold.shape)
    w_warm, st_w = eb.adjoint(x1, w.x0, a, xbar, vbar, block=64, w_init=start)
    assert np.all(st_w["flags"] & 8)
    pin = w.pinned.astype(bool)
    assert np.all(w_warm[pin] == 0.0)
    for b in range(w.n_bodies):
        wb = w.body(b)
        p = Problem.from_workload(wb)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        wr = solve.adjoint(p, x1[sv], w.x0[sv], wb.actions[0], xbar[sv], vbar[sv])
        assert rel(w_warm[sv], wr) <= tol


@pytest.mark.parametrize("block", [256, 768])
def test_emulated_multi_wave_workgroups(emu_mod, block):
    """Workgroups of 4 and 12 waves: the alternating reduction banks, the cross-wave sums and every
    barrier of the step, CG and adjoint with more waves than the one-wave runs above exercise."""
    w, rng = rand_workload(2, seed=25, bodies=2, shape=(4, 2))
    w = _tight(w)
    eb = emu_mod.EmuBatch(w, "fp64")
    a = w.actions[0]
    x1, v1, st = eb.step(w.x0, w.v0, a, block=block)
    assert np.all(st["flags"] & 1)
    xbar = rng.normal(size=x1.shape)
    wv, sa = eb.adjoint(x1, w.x0, a, xbar, None, block=block)
    assert np.all(sa["flags"] & 8)
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        se = slice(w.body_e_off[b], w.body_e_off[b + 1])
        xr, vr, _ = solve.step(p, w.x0[sv], w.v0[sv], a[se], tol=1e-13)
        assert rel(x1[sv] - w.x0[sv], xr - w.x0[sv]) <= 1e-10
        wr = solve.adjoint(p, x1[sv], w.x0[sv], a[se], xbar[sv])
        assert rel(wv[sv], wr) <= 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_emulated_compact_rest_record(emu_mod, precision, tol):
    """Bodies of one material with x fibres take the compact rest record (Dm^-1 and W per element,
    the material from the mesh's scalars), as the library's batched launch does."""
    from synth import scenes
    w = scenes.batched_strips(2, steps=1, sizes=np.array([4, 5]))
    w = _tight(w)
    eb = emu_mod.EmuBatch(w, precision)
    assert eb.m.axis == 0
    a = w.actions[0]
    x1, v1, st = eb.step(w.x0, w.v0, a, block=64)
    assert np.all(st["flags"] & 1)
    for b, p in enumerate(problems(w)):
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        wb = w.body(b)
        xr, vr, _ = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=1e-13)
        assert rel(x1[sv] - wb.x0, xr - wb.x0) <= tol
