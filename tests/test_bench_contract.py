"""CPU checks of bench.py's contract pieces: it refuses more than one GPU, its algorithmic byte
model gives the per-element figures the roofline is quoted with, and measured traffic is only
reported for the library sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_element_byte_model():
    # the general per-element record of a tetrahedron: connectivity 16 B, Dm^-1 (9), gf (3), W mu,
    # W lam, W k_f, actuation: 144 B in FP64; 80 + the FP64 actuation's extra 4 B = 84 B mixed
    assert bench.elem_bytes(3, 8) == 144
    assert bench.elem_bytes(3, 4) + 4 == 84
    assert bench.elem_bytes(2, 8) == 4 * 3 + 8 * (4 + 2 + 3 + 1)
    # the compact record of a uniform material with axis fibres: Dm^-1 and W (104 B, 60 B mixed)
    assert bench.elem_bytes(3, 8, compact=True) == 104 and bench.elem_bytes(3, 4, compact=True) == 60
    # batched triangles: 16-bit body-local connectivity and the 10-word edge Hessian
    assert bench.hv_elem_bytes(2, 4) == 2 * 3 + 40
    # a trial pass reads the FP64 rest data: 4 words fewer per triangle with the compact record
    assert bench.trial_bytes(2, 1, 0, 4) - bench.trial_bytes(2, 1, 0, 4, compact=True) == 8 * 4


def test_adjoint_warm_start_adds_one_hessian_vector_pass():
    st = {"adj_cg_iters": 40}
    ne, nv = 1000, 550
    cold = bench.adjoint_launch_bytes(2, ne, nv, st, 4)
    warm = bench.adjoint_launch_bytes(2, ne, nv, st, 4, warm=True)
    assert warm - cold == bench.hv_elem_bytes(2, 4) * ne + (8 + 16 + 4 + 8 + 24) * nv * 2
    one_more = bench.adjoint_launch_bytes(2, ne, nv, {"adj_cg_iters": 41}, 4)
    assert cold < warm < one_more + (8 + 16 + 4 + 8 + 24) * nv * 2


def test_traffic_record_is_ignored_for_other_sources(tmp_path, monkeypatch):
    rec = {"source_hash": bench.kernel_source_hash(), "bytes_per_launch": {"0": 123, "1": 45}}
    f = tmp_path / "counters.md"
    f.write_text("# counters\n\ntraffic-record: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(f))
    assert bench.measured_traffic(0) == 123 and bench.measured_traffic(1) == 45
    rec["source_hash"] = "0" * 64
    f.write_text("traffic-record: " + json.dumps(rec) + "\n")
    assert bench.measured_traffic(0) is None


def test_octile_pick_takes_equal_shares_of_each_size_octile():
    import numpy as np
    sizes = np.random.default_rng(0).integers(128, 8193, size=512)
    pick = bench.octile_pick(sizes, 64)
    assert len(pick) == 64 and len(set(pick.tolist())) == 64
    order = np.argsort(sizes, kind="stable")
    rank = np.empty(512, int)
    rank[order] = np.arange(512)
    assert np.array_equal(np.bincount(rank[pick] // 64, minlength=8), np.full(8, 8))


def test_bench_reference_matches_the_workloads_it_was_written_for():
    """The stored oracle results bench.py compares against: one per leg, for the workloads the bench
    builds (same vertex counts), with sampled vertices inside each body."""
    from synth import scenes
    g = bench.golden()
    w = scenes.batched_strips(512, steps=1)
    for ref in g["batched_strips_512"]:
        b = ref["body"]
        assert ref["n_v"] == w.body_v_off[b + 1] - w.body_v_off[b]
        assert max(ref["vertices"]) < ref["n_v"] and len(ref["x1"]) == len(ref["vertices"])
    assert set(g["energies"]) == {"stvk", "corot", "snh"}
    assert g["be_strip_64x16_5_steps"]["steps"] == 5
    assert g["policy_strip_64x16"]["horizon"] == 100 and g["policy_strip_64x16"]["grad_norm"] > 0


def test_sampled_error_is_relative_to_the_displacement():
    import numpy as np
    x0 = np.zeros((10, 2))
    ref = {"vertices": [1, 3], "x1": [[1.0, 0.0], [0.0, 1.0]]}
    x = x0.copy()
    x[1] = [1.0, 0.0]
    x[3] = [0.0, 1.001]
    assert abs(bench.sampled_error(x, ref, x0) - 0.001 / np.sqrt(2.0)) < 1e-15
