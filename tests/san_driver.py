"""Drivers the sanitizer tests run in a child process with the sanitizer runtime preloaded (test
infrastructure only; the module name keeps pytest from collecting it).

  python -m tests.san_driver host <libisb_host built with -fsanitize=address,undefined>
  python -m tests.san_driver emu <libisb_emu built with -fsanitize=thread>

`host` drives the host-only C ABI (mesh validation, colouring, locality and wave orders) over valid
and invalid meshes; `emu` runs the batched solver's body logic on host threads (2 emulated waves on
triangles with springs in mixed precision, 4 on tetrahedra in FP64, warm-started adjoints) and checks it against the
FP64 oracle. Each exits non-zero on a failed check; the sanitizers abort on the first report."""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def host(path):
    from synth import meshes
    lib = ctypes.CDLL(path)
    lib.isb_last_error.restype = ctypes.c_char_p
    lib.isb_version.restype = ctypes.c_char_p
    assert lib.isb_version().startswith(b"isb")
    checks = 0
    for dim, (X, T) in ((2, meshes.tri_grid(9, 4)), (3, meshes.tet_grid(4, 3, 3))):
        parts = [(X, T, np.zeros(X.shape, np.uint8))] * 3
        Xb, Tb, _, vo, eo = meshes.concat_bodies(parts)
        Xb = np.ascontiguousarray(Xb, np.float64)
        Tb = np.ascontiguousarray(Tb, np.int32)
        vo = np.ascontiguousarray(vo, np.int64)
        eo = np.ascontiguousarray(eo, np.int64)
        n_v, n_e = Xb.shape[0], Tb.shape[0]
        assert lib.isb_validate_mesh(dim, n_v, _p(Xb), n_e, _p(Tb), 3, _p(vo), _p(eo)) == 0
        col = np.zeros(n_e, np.int32)
        nc = ctypes.c_int32(0)
        assert lib.isb_colour_elements(dim, n_v, n_e, _p(Tb), _p(col), ctypes.byref(nc)) == 0
        for k in range(nc.value):   # no two elements of a colour share a vertex
            v = Tb[col == k].ravel()
            assert np.unique(v).size == v.size
        perm = np.zeros(n_e, np.int64)
        assert lib.isb_locality_order(dim, n_v, _p(Xb), n_e, _p(Tb), 3, _p(eo), _p(perm)) == 0
        assert np.array_equal(np.sort(perm), np.arange(n_e))
        assert lib.isb_wave_order(dim, n_v, n_e, _p(Tb), 3, _p(eo), _p(perm)) == 0
        assert np.array_equal(np.sort(perm), np.arange(n_e))
        # invalid meshes: index out of the body's range, a repeated vertex, an inverted element,
        # broken offsets; each must be rejected without touching memory outside the arrays
        bad = []
        t = Tb.copy(); t[0, 0] = n_v + 5; bad.append((t, vo, eo))
        t = Tb.copy(); t[1, 1] = t[1, 0]; bad.append((t, vo, eo))
        t = Tb.copy(); t[2, [0, 1]] = t[2, [1, 0]]; bad.append((t, vo, eo))
        t = Tb.copy(); t[eo[1], 0] = vo[1] - 1; bad.append((t, vo, eo))   # body 1 element using body 0's vertex
        v2 = vo.copy(); v2[1] = v2[2] + 1; bad.append((Tb, v2, eo))
        e2 = eo.copy(); e2[1] = e2[2] + 1; bad.append((Tb, vo, e2))
        for k, (t, v_, e_) in enumerate(bad):
            t = np.ascontiguousarray(t, np.int32)
            st = lib.isb_validate_mesh(dim, int(v_[-1]), _p(Xb), int(e_[-1]), _p(t), 3, _p(v_), _p(e_))
            assert st != 0 and lib.isb_last_error(), (dim, k)
            checks += 1
        t = Tb.copy(); t[0, 0] = -1
        t = np.ascontiguousarray(t, np.int32)
        assert lib.isb_colour_elements(dim, n_v, n_e, _p(t), _p(col), ctypes.byref(nc)) != 0
        assert lib.isb_locality_order(dim, n_v, _p(Xb), n_e, _p(t), 3, _p(eo), _p(perm)) != 0
        assert lib.isb_wave_order(dim, n_v, n_e, _p(t), 3, _p(eo), _p(perm)) != 0
        checks += 3
    # a mesh of 72 patches, so that the wave order's per-patch balance runs on several threads
    X, T = meshes.tet_grid(24, 16, 8)
    T = np.ascontiguousarray(T, np.int32)
    perm = np.zeros(T.shape[0], np.int64)
    assert lib.isb_wave_order(3, X.shape[0], T.shape[0], _p(T), 1, None, _p(perm)) == 0
    assert np.array_equal(np.sort(perm), np.arange(T.shape[0]))
    print(f"host ABI checks passed ({checks} rejections)")


def emu(path):
    from oracle import solve
    from oracle.fem import Problem
    from tests.emu import emu as em
    from tests.gpu_util import rand_workload, rel, with_springs
    em.OUT = path
    em.build = lambda: path
    # (dim, body shape, precision, bar, threads per emulated workgroup)
    cases = [(2, (3, 2), "mixed", 1e-5, 128), (3, (2, 2, 1), "fp64", 1e-10, 256)]
    for dim, shape, precision, tol, block in cases:
        w, rng = rand_workload(dim, seed=31 + dim, bodies=2, shape=shape)
        if dim == 2:
            w = with_springs(w, rng)
        w.scene.update(tol_rel=1e-13, adj_tol_rel=1e-13, max_newton=60, max_cg=4000)
        eb = em.EmuBatch(w, precision)
        a = w.actions[0]
        x1, v1, st = eb.step(w.x0, w.v0, a, block=block)
        assert np.all(st["flags"] & 1), st["flags"]
        xbar, vbar = rng.normal(size=x1.shape), rng.normal(size=x1.shape)
        wv, sa = eb.adjoint(x1, w.x0, a, xbar, vbar, block=block, w_init=0.5 * np.ones_like(x1))
        assert np.all(sa["flags"] & 8), sa["flags"]
        for b in range(w.n_bodies):
            wb = w.body(b)
            p = Problem.from_workload(wb)
            sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
            xr, _, _ = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=1e-13)
            assert rel(x1[sv] - wb.x0, xr - wb.x0) <= tol, (dim, precision, block, b)
            wr = solve.adjoint(p, x1[sv], wb.x0, wb.actions[0], xbar[sv], vbar[sv])
            assert rel(wv[sv], wr) <= tol, (dim, precision, block, b)
    print(f"emulated batched solver checks passed ({len(cases)} runs)")


if __name__ == "__main__":
    {"host": host, "emu": emu}[sys.argv[1]](sys.argv[2])
