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
