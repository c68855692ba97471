"""CPU tests of the C ABI: the library loads, exports every declared symbol, and its host-only
entry points (mesh validation, element colouring) behave. No GPU call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth import meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isb.h")


def _lib():
    from paper_2102_05791_amd import isb
    return isb, isb.load_library()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(isb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    isb, lib = _lib()
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(isb.EXPORTED)
    assert lib.isb_version().startswith(b"isb")


def test_header_struct_layouts_match_binding():
    isb, _ = _lib()
    assert ctypes.sizeof(isb.Stats) == 6 * 4 + 6 * 8
    assert ctypes.sizeof(isb.Scene) == 4 * 4 + 7 * 8


def test_validate_mesh_accepts_grids():
    isb, _ = _lib()
    X, T = meshes.tri_grid(5, 3)
    assert isb.validate_mesh(2, X, T)[0] == isb.ISB_OK
    X, T = meshes.tet_grid(3, 2, 2)
    assert isb.validate_mesh(3, X, T)[0] == isb.ISB_OK


@pytest.mark.parametrize("case", ["inverted", "out_of_range", "repeat", "body_cross", "nan"])
def test_validate_mesh_rejects(case):
    isb, _ = _lib()
    X, T = meshes.tri_grid(4, 2)
    T = T.copy()
    X = X.copy()
    vo = eo = None
    if case == "inverted":
        T[3, [1, 2]] = T[3, [2, 1]]
    elif case == "out_of_range":
        T[2, 0] = X.shape[0]
    elif case == "repeat":
        T[1, 2] = T[1, 0]
    elif case == "nan":
        X[4, 1] = np.nan
    elif case == "body_cross":
        # two bodies: the second body's element refers to a vertex of the first
        X2, T2 = meshes.tri_grid(2, 2)
        X, T, P, vo, eo = meshes.concat_bodies([(X, T, np.zeros(X.shape, np.uint8)),
                                                (X2, T2, np.zeros(X2.shape, np.uint8))])
        T[-1, 0] = 0
    st, msg = isb.validate_mesh(2, X, T, vo, eo)
    assert st == isb.ISB_E_MESH, (case, st, msg)
    assert msg


def _check_colouring(T, col, nc):
    assert col.min() == 0 and col.max() == nc - 1
    for c in range(nc):
        verts = T[col == c].ravel()
        assert len(np.unique(verts)) == len(verts), f"colour {c} shares a vertex"


def test_colouring_valid_2d_3d():
    isb, _ = _lib()
    X, T = meshes.tri_grid(64, 16)
    col, nc = isb.colour_elements(2, X.shape[0], T)
    _check_colouring(T, col, nc)
    assert 6 <= nc <= 13
    X, T = meshes.tet_grid(6, 5, 4)
    col, nc = isb.colour_elements(3, X.shape[0], T)
    _check_colouring(T, col, nc)
    assert nc <= 64
    col2, nc2 = isb.colour_elements(3, X.shape[0], T)
    assert nc2 == nc and np.array_equal(col, col2)


def test_colouring_rejects_bad_index():
    isb, _ = _lib()
    X, T = meshes.tri_grid(3, 2)
    T = T.copy()
    T[0, 0] = 10 ** 6
    with pytest.raises(isb.IsbError):
        isb.colour_elements(2, X.shape[0], T)


def test_library_missing_raises(tmp_path):
    isb, _ = _lib()
    with pytest.raises(ImportError):
        isb.load_library(str(tmp_path / "nope.so"))


def test_stream_copy_rejects_bad_arguments_before_any_gpu_call():
    """isb_stream_copy checks its arguments on the host: negative n, NULL or misaligned buffers and
    overlapping ranges fail with ISB_E_ARG without touching a device (pointer values only)."""
    import ctypes
    isb, _ = _lib()
    lib = isb.load_library()
    vp = ctypes.c_void_p
    cases = [(vp(4096), vp(8192), -1), (None, vp(8192), 4), (vp(4096), None, 4),
             (vp(4104), vp(8192), 4), (vp(4096), vp(4096 + 16), 8)]
    for src, dst, n in cases:
        assert lib.isb_stream_copy(None, src, dst, n) == isb.ISB_E_ARG
        assert lib.isb_last_error()


def _patch_duplication(T, n_v, size=1024):
    """Sum over runs of `size` consecutive elements of their distinct vertices, over n_v."""
    return sum(np.unique(T[s:s + size]).size for s in range(0, T.shape[0], size)) / n_v


def test_locality_order_is_a_per_body_permutation_that_compacts_patches():
    from paper_2102_05791_amd import isb
    X, T = meshes.tet_grid(96, 8, 8, block=1)           # cubes x fastest: long thin runs
    perm = isb.locality_order(3, X, T)
    assert np.array_equal(np.sort(perm), np.arange(T.shape[0]))
    assert np.array_equal(perm, isb.locality_order(3, X, T))          # deterministic
    before, after = _patch_duplication(T, X.shape[0]), _patch_duplication(T[perm], X.shape[0])
    assert after < 0.7 * before, (before, after)
    # two bodies: every body's elements stay in its own range
    X2, T2 = meshes.tri_grid(40, 30)
    Xb = np.concatenate([X2, X2 + 100.0])
    Tb = np.concatenate([T2, T2 + X2.shape[0]])
    eoff = np.array([0, T2.shape[0], 2 * T2.shape[0]])
    pb = isb.locality_order(2, Xb, Tb, eoff)
    assert np.array_equal(np.sort(pb[:T2.shape[0]]), np.arange(T2.shape[0]))
    assert np.array_equal(np.sort(pb[T2.shape[0]:]), np.arange(T2.shape[0], 2 * T2.shape[0]))


def _patch_bounds(T, n_v, eoff, dim):
    """Patch boundaries by the plan's rule: per body, runs of min(2048, max(256, n_b/1024 rounded
    up to a multiple of 64)) elements, cut early where the distinct vertices would exceed what
    three FP64 vectors and a 4-byte vertex id fit in 64 KB of LDS."""
    budget = 64 * 1024 // (3 * dim * 8 + 4)
    out = [0]
    for b in range(len(eoff) - 1):
        n_b = eoff[b + 1] - eoff[b]
        me = min(2048, max(256, -(-(n_b // 1024) // 64) * 64))
        e = eoff[b]
        while e < eoff[b + 1]:
            seen, start = set(), e
            while e < eoff[b + 1] and e - start < me:
                fresh = set(T[e].tolist()) - seen
                if len(seen) + len(fresh) > budget:
                    break
                seen |= fresh
                e += 1
            out.append(e)
    return np.array(out)


def _half_wave_bank_load(T, bounds, dim):
    """Mean over (half-wavefront group of 32 consecutive elements from a patch's first, corner slot)
    of the most lanes whose vertex falls in one LDS bank class: the plan numbers a patch's vertices
    by sorted global id, and FP64 [vertex][dim] rows put local id v in class v mod 32 (3D) or
    v mod 16 (2D)."""
    nc = 32 if dim == 3 else 16
    loads = []
    for s, e in zip(bounds[:-1], bounds[1:]):
        P = T[s:e]
        loc = np.searchsorted(np.unique(P), P) % nc
        g = np.arange(e - s) // 32
        for k in range(T.shape[1]):
            cnt = np.bincount(g * nc + loc[:, k], minlength=(g[-1] + 1) * nc).reshape(-1, nc)
            loads.append(cnt.max(axis=1))
    return float(np.mean(np.concatenate(loads)))


def _slot_clashes(T, bounds, wave=64):
    """Lanes of a wavefront group (64 consecutive elements from a patch's first) whose vertex in
    some corner slot another lane of the group already has there, per element corner."""
    c = 0
    for s, e in zip(bounds[:-1], bounds[1:]):
        for w in range(s, e, wave):
            g = T[w:min(w + wave, e)]
            c += sum(g.shape[0] - np.unique(g[:, k]).size for k in range(T.shape[1]))
    return c / T.size


def test_wave_order_keeps_patches_and_separates_slot_vertices():
    from paper_2102_05791_amd import isb
    X, T = meshes.tet_grid(48, 32, 16)                 # 147,456 tets in 4x4x4-cube blocks
    n_e, n_v = T.shape[0], X.shape[0]
    bounds = _patch_bounds(T, n_v, [0, n_e], 3)
    assert np.all(np.diff(bounds)[:-1] == 256)         # n_e/1024 = 144: the 256 floor
    perm = isb.wave_order(3, n_v, T)
    assert np.array_equal(np.sort(perm), np.arange(n_e))
    assert np.array_equal(perm, isb.wave_order(3, n_v, T))           # deterministic
    for s, e in zip(bounds[:-1], bounds[1:]):          # a permutation inside each patch
        assert np.array_equal(np.sort(perm[s:e]), np.arange(s, e))
    assert np.array_equal(_patch_bounds(T[perm], n_v, [0, n_e], 3), bounds)
    # the six tetrahedra of a cube share two corners in fixed slots, so a patch of four wavefront
    # groups cannot separate them all: fewer clashes, not none
    before, after = _slot_clashes(T, bounds), _slot_clashes(T[perm], bounds)
    assert before > 0.5 and after < 0.5 * before, (before, after)
    # and each half-wavefront's corners spread over the LDS bank classes (ideal 1 lane per class)
    lb, la = _half_wave_bank_load(T, bounds, 3), _half_wave_bank_load(T[perm], bounds, 3)
    assert lb > 2.9 and la < 2.2, (lb, la)
    # 393,216 tets: 384-element patches of six groups, one per tetrahedron of a cube: no clash left
    X6, T6 = meshes.tet_grid(64, 32, 32)
    b6 = _patch_bounds(T6, X6.shape[0], [0, T6.shape[0]], 3)
    assert np.all(np.diff(b6) == 384)
    p6 = isb.wave_order(3, X6.shape[0], T6)
    assert all(np.array_equal(np.sort(p6[s:e]), np.arange(s, e)) for s, e in zip(b6[:-1], b6[1:]))
    assert _slot_clashes(T6, b6) > 0.5 and _slot_clashes(T6[p6], b6) == 0.0
    # two bodies of triangles, the second large enough for 256-element patches: ranges kept
    X1, T1 = meshes.tri_grid(20, 10)
    X2, T2 = meshes.tri_grid(130, 65)
    Tb = np.concatenate([T1, T2 + X1.shape[0]])
    eoff = np.array([0, T1.shape[0], T1.shape[0] + T2.shape[0]])
    nvb = X1.shape[0] + X2.shape[0]
    pb = isb.wave_order(2, nvb, Tb, eoff)
    bb = _patch_bounds(Tb, nvb, eoff, 2)
    for s, e in zip(bb[:-1], bb[1:]):
        assert np.array_equal(np.sort(pb[s:e]), np.arange(s, e))
    assert _slot_clashes(Tb[pb], bb) < 0.5 * _slot_clashes(Tb, bb)
    # 304,000 triangles: n_e/1024 = 296 rounds up to 320 elements, five whole wavefronts
    X3, T3 = meshes.tri_grid(400, 380)
    b3 = _patch_bounds(T3, X3.shape[0], [0, T3.shape[0]], 2)
    assert np.all(np.diff(b3)[:-1] == 320)
    p3 = isb.wave_order(2, X3.shape[0], T3)
    assert all(np.array_equal(np.sort(p3[s:e]), np.arange(s, e)) for s, e in zip(b3[:-1], b3[1:]))
    assert isb.wave_order(2, nvb, Tb[:0]).size == 0


def test_wave_order_rejects_bad_input():
    from paper_2102_05791_amd import IsbError, isb
    X, T = meshes.tri_grid(3, 2)
    bad = T.copy()
    bad[1, 2] = X.shape[0]
    with pytest.raises(IsbError) as e:
        isb.wave_order(2, X.shape[0], bad)
    assert e.value.status == isb.ISB_E_MESH
    with pytest.raises(IsbError) as e:
        isb.wave_order(2, X.shape[0], T, np.array([0, 3, 2]))
    assert e.value.status == isb.ISB_E_ARG
    with pytest.raises(IsbError) as e:
        isb.wave_order(4, X.shape[0], T)
    assert e.value.status == isb.ISB_E_ARG


def test_locality_order_rejects_bad_input():
    from paper_2102_05791_amd import IsbError, isb
    X, T = meshes.tri_grid(3, 2)
    bad = T.copy()
    bad[1, 2] = X.shape[0]
    with pytest.raises(IsbError) as e:
        isb.locality_order(2, X, bad)
    assert e.value.status == isb.ISB_E_MESH
    with pytest.raises(IsbError) as e:
        isb.locality_order(2, X, T, np.array([0, 3, 2]))
    assert e.value.status == isb.ISB_E_ARG


def test_permute_elements_moves_every_per_element_array_together():
    """A workload in wave order is the same problem: the oracle's total energy (a sum over elements
    and vertices) is unchanged, and each body keeps its elements and its actions."""
    from oracle.fem import Problem
    from paper_2102_05791_amd import isb
    from synth import scenes
    w = scenes.batched_strips(6, steps=2)
    perm = isb.wave_order(2, w.n_v, w.T, w.body_e_off)
    assert not np.array_equal(perm, np.arange(w.n_e))
    wp = w.permute_elements(perm)
    rng = np.random.default_rng(5)
    x = w.x0 + 0.01 * rng.standard_normal(w.x0.shape)
    for b in (0, 5):
        p, pp = Problem.from_workload(w.body(b)), Problem.from_workload(wp.body(b))
        wb, wpb = w.body(b), wp.body(b)
        sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
        e = sum(t.sum() for t in p.energy_terms(x[sv], wb.x0, wb.v0, wb.actions[1]))
        ep = sum(t.sum() for t in pp.energy_terms(x[sv], wpb.x0, wpb.v0, wpb.actions[1]))
        assert abs(e - ep) <= 1e-12 * abs(e)
    with pytest.raises(ValueError):
        w.permute_elements(np.roll(np.arange(w.n_e), 1))   # moves elements across bodies
