"""isb_autotune through the C ABI: it keeps one of its candidate configurations, the solver still
matches the oracle afterwards, and the Python JSON cache answers a repeated question without
timing."""
import json

import numpy as np
import pytest

from oracle import solve
from oracle.fem import Problem
from synth import scenes
from tests.gpu_util import rand_workload, rel, rel_inf

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def test_autotune_batched_block_and_cache(tmp_path):
    from paper_2102_05791_amd import Context, isb
    w = scenes.batched_strips(48, steps=1)
    ctx = Context.from_workload(w, precision="mixed", solver=1)
    x0, v0, a = _dev(w.x0), _dev(w.v0), _dev(w.actions[0])
    cache = str(tmp_path / "tune.json")
    chosen = ctx.autotune(x0, v0, a, cache_path=cache)
    assert list(chosen) == [isb.OPT_BLOCK] and chosen[isb.OPT_BLOCK] in (512, 768, 1024)
    assert ctx.get_option(isb.OPT_BLOCK) == chosen[isb.OPT_BLOCK]
    doc = json.load(open(cache))
    assert len(doc) == 1 and list(doc.values())[0] == [isb.OPT_BLOCK, chosen[isb.OPT_BLOCK]]
    # the step with the chosen size still solves the bodies (sampled against the oracle)
    x1, _, st, _ = ctx.step(x0, v0, a)
    assert all(s["flags"] & 1 for s in st)
    x1 = x1.cpu().numpy()
    for b in (0, 47):
        wb = w.body(b)
        xr, _, _ = solve.step(Problem.from_workload(wb), wb.x0, wb.v0, wb.actions[0], tol=1e-13)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        assert rel(x1[sv] - wb.x0, xr - wb.x0) <= 1e-4
        assert rel_inf(x1[sv] - wb.x0, xr - wb.x0) <= 1e-4
    # a second context answers from the cache: it takes the cached value even when it differs
    doc[list(doc)[0]] = [isb.OPT_BLOCK, 512]
    json.dump(doc, open(cache, "w"))
    ctx2 = Context.from_workload(w, precision="mixed", solver=1)
    assert ctx2.autotune(x0, v0, a, cache_path=cache) == {isb.OPT_BLOCK: 512}
    assert ctx2.get_option(isb.OPT_BLOCK) == 512


def test_autotune_plain_scatter():
    from paper_2102_05791_amd import Context, isb
    w, rng = rand_workload(2, seed=81, shape=(130, 65))          # 16,900 triangles: patches apply
    w.scene.update(tol_rel=1e-10)
    ctx = Context.from_workload(w, precision="fp64", solver=0)
    x0, v0, a = _dev(w.x0), _dev(w.v0), _dev(w.actions[0])
    chosen = ctx.autotune(x0, v0, a)
    assert list(chosen) == [isb.OPT_SCATTER] and chosen[isb.OPT_SCATTER] in (0, 2)
    assert ctx.get_option(isb.OPT_SCATTER) == chosen[isb.OPT_SCATTER]
    x1, _, st, _ = ctx.step(x0, v0, a)
    xr, _, _ = solve.step(Problem.from_workload(w), w.x0, w.v0, w.actions[0], tol=1e-13)
    assert rel(x1.cpu().numpy() - w.x0, xr - w.x0) <= 1e-8
    assert rel_inf(x1.cpu().numpy() - w.x0, xr - w.x0) <= 1e-8
