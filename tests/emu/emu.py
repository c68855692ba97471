"""ctypes driver of the CPU-emulated batched solver (tests/emu/batched_emu.cpp).

Builds libisb_emu.so with g++ on first use (into tests/emu/_build, git-ignored) and runs
isb_body.hpp's body logic with host threads as one workgroup. Test infrastructure only: it
checks the persistent solver's control flow and arithmetic on the CPU; the GPU tests check
the same code on the device.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2102_05791_amd", "csrc")
OUT = os.path.join(HERE, "_build", "libisb_emu.so")
SRCS = [os.path.join(HERE, "batched_emu.cpp"), os.path.join(CSRC, "isb_body.hpp"),
        os.path.join(CSRC, "isb_elem.hpp"), os.path.join(CSRC, "isb_device.hpp"), os.path.join(CSRC, "isb_spring.hpp"),
        os.path.join(HERE, "include", "hip", "hip_runtime.h")]

vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double


class DevMesh(ctypes.Structure):
    _fields_ = [("dim", ci), ("n_v", ci), ("n_e", ci), ("conn", vp), ("Dinv", vp), ("gf", vp), ("W", vp),
                ("wmu", vp), ("wlam", vp), ("wkf", vp), ("Dinv32", vp), ("gf32", vp), ("wmu32", vp),
                ("wlam32", vp), ("wkf32", vp), ("mass", vp), ("pinned", vp), ("model", ci), ("axis", ci),
                ("mu_u", cd), ("lam_u", cd), ("kf_u", cd), ("W32", vp)]


class DevScene(ctypes.Structure):
    _fields_ = [("be", ci), ("h", cd), ("s_pot", cd), ("grav", cd), ("kc", cd), ("kfr", cd), ("eps", cd), ("ih2", cd)]


class BatchArgs(ctypes.Structure):
    _fields_ = [("order", vp), ("wg_off", vp), ("voff", vp), ("eoff", vp), ("n_bodies", ci),
                ("x0", vp), ("v0", vp), ("a", vp), ("a32", vp), ("x1", vp), ("v1", vp), ("xbar", vp),
                ("vbar", vp), ("w", vp), ("xhat", vp), ("G", vp), ("Gt", vp), ("dx", vp), ("r", vp), ("cv", vp),
                ("xt", vp), ("Dv", vp), ("vdT", vp), ("lconn", vp), ("stats", vp), ("tol", cd), ("adj_tol", cd),
                ("max_newton", ci), ("max_cg", ci), ("want_tail", ci), ("nacc", ci), ("Fbuf", vp), ("E0", vp), ("E1", vp),
                ("soff", vp), ("slconn", vp), ("sk", vp), ("sil0", vp), ("Sbuf", vp), ("n_s", ci),
                ("adj_warm", ci)]


STATS_DTYPE = np.dtype([("newton_iters", "<i4"), ("cg_iters", "<i4"), ("adj_cg_iters", "<i4"),
                        ("ls_backtracks", "<i4"), ("negcurv_exits", "<i4"), ("flags", "<i4"),
                        ("res0", "<f8"), ("res_final", "<f8"), ("adj_res_final", "<f8"), ("energy", "<f8"),
                        ("min_J", "<f8"), ("max_J", "<f8")])


def build():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    if os.path.exists(OUT) and all(os.path.getmtime(OUT) >= os.path.getmtime(s) for s in SRCS):
        return OUT
    tmp = f"{OUT}.{os.getpid()}.tmp"  # parallel test workers build apart, then one rename wins
    cmd = ["g++", "-std=c++20", "-O1", "-fPIC", "-shared", "-pthread", "-DISB_DEBUG", "-I",
           os.path.join(HERE, "include"), "-I", CSRC, SRCS[0], "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(tmp, OUT)
    return OUT


def _p(a):
    return a.ctypes.data_as(vp)


def compact_axis(w):
    """The library's test for the compact rest record: one (mu, lam, k_f) for every element and every
    fibre along one coordinate axis; returns that axis, or -1."""
    if w.n_e == 0:
        return -1
    d0 = w.fdir[0]
    axes = [k for k in range(w.dim) if d0[k] == 1.0]
    if not axes:
        return -1
    ax = axes[-1]
    unit = np.zeros(w.dim)
    unit[ax] = 1.0
    same = (np.all(w.mu == w.mu[0]) and np.all(w.lam == w.lam[0]) and np.all(w.kf == w.kf[0])
            and np.all(w.fdir == unit))
    return ax if same else -1


class EmuBatch:
    """Host arrays laid out exactly as the device arrays of the library (SoA element data)."""

    def __init__(self, w, precision="fp64"):
        self.lib = ctypes.CDLL(build())
        self.allow_index_errors = False
        self.last_index_site = 0
        self._left = ctypes.c_double(0.0)
        self.lds_left = None
        sizes = (ci * 4)()
        self.lib.emu_sizes(sizes)
        assert list(sizes) == [ctypes.sizeof(DevMesh), ctypes.sizeof(DevScene), ctypes.sizeof(BatchArgs), 72]
        offs = (ci * len(BatchArgs._fields_))()
        assert self.lib.emu_batchargs_offsets(offs) == len(BatchArgs._fields_)
        assert list(offs) == [getattr(BatchArgs, f).offset for f, _ in BatchArgs._fields_], "BatchArgs layout"
        self.w = w
        d = w.dim
        self.prec = 1 if precision == "mixed" else 0
        X, T = w.X, w.T.astype(np.int64)
        Dm = np.swapaxes(X[T[:, 1:]] - X[T[:, :1]], 1, 2)
        Dinv = np.linalg.inv(Dm)
        W = np.linalg.det(Dm) / math.factorial(d)
        gf = np.einsum("ejc,ec->ej", Dinv, w.fdir)
        self.keep = []

        def k(a):
            a = np.ascontiguousarray(a)
            self.keep.append(a)
            return a
        self.conn = k(np.ascontiguousarray(w.T.T, dtype=np.int32))
        self.Dinv = k(Dinv.reshape(len(T), d * d).T.astype(np.float64))
        self.gf = k(gf.T.astype(np.float64))
        self.W = k(W)
        self.wmu, self.wlam, self.wkf = k(W * w.mu), k(W * w.lam), k(W * w.kf)
        mass = np.zeros(w.n_v)
        np.add.at(mass, T, (w.rho * W / (d + 1))[:, None])
        self.mass = k(mass)
        self.pinned = k(w.pinned.astype(np.uint8))
        f32 = lambda a: k(a.astype(np.float32))
        self.m = DevMesh(d, w.n_v, w.n_e, _p(self.conn), _p(self.Dinv), _p(self.gf), _p(self.W), _p(self.wmu),
                         _p(self.wlam), _p(self.wkf), _p(f32(self.Dinv)), _p(f32(self.gf)), _p(f32(self.wmu)),
                         _p(f32(self.wlam)), _p(f32(self.wkf)), _p(self.mass), _p(self.pinned),
                         {"nh": 0, "stvk": 1, "corot": 2, "snh": 3}[getattr(w, "model", "nh")],
                         compact_axis(w), float(w.mu[0]), float(w.lam[0]), float(w.kf[0]), _p(f32(self.W)))
        sc = w.scene
        be = sc["integrator"] == "be"
        self.sc = DevScene(int(be), sc["h"], sc["h"] ** 2 if be else 1.0, sc["gravity"], sc["k_contact"],
                           sc["k_friction"], sc["eps_friction"], 1.0 / (sc["h"] * sc["h"]))
        nb = w.n_bodies
        ne_b = np.diff(w.body_e_off)
        self.order = k(np.argsort(-ne_b, kind="stable").astype(np.int32))
        self.wg_off = k(np.array([0, nb], dtype=np.int32))  # one workgroup takes every body
        self.voff = k(w.body_v_off.astype(np.int32))
        self.eoff = k(w.body_e_off.astype(np.int32))
        self.nacc = int((np.diff(w.body_v_off) * d).max())
        nd = w.n_v * d
        self.ws = {n: k(np.zeros(nd)) for n in ("xhat", "G", "Gt", "dx", "r", "xt")}
        self.Dv = k(np.zeros(nd, dtype=np.float32))  # FP32 preconditioner
        self.vdT = k(np.zeros(nd, dtype=np.float64))  # element precision (FP32 uses the first half)
        body = np.repeat(np.arange(nb), ne_b)
        self.lconn = k((self.conn - w.body_v_off[body][None, :]).astype(np.uint16))
        self.cv = k(np.zeros(w.n_v))
        self.stats = k(np.zeros(nb, dtype=STATS_DTYPE))
        self.Fbuf = k(np.zeros((10 if d == 2 else d * d + d) * w.n_e, dtype=np.float64))  # hv_state_words
        n_s = getattr(w, "n_s", 0)
        self.n_s = n_s
        self.E0 = k(np.zeros(w.n_e + n_s))
        self.E1 = k(np.zeros(w.n_e + n_s))
        if n_s:
            S = w.S.astype(np.int64)
            sbody = np.repeat(np.arange(nb), np.diff(w.body_s_off))
            self.soff = k(w.body_s_off.astype(np.int32))
            self.slconn = k((S.T - w.body_v_off[sbody][None, :]).astype(np.uint16))
            self.sk = k(w.ks.astype(np.float64))
            self.sil0 = k(1.0 / np.linalg.norm(X[S[:, 1]] - X[S[:, 0]], axis=1))
            self.Sbuf = k(np.zeros(d * (d + 1) // 2 * n_s, dtype=np.float64))  # spring_state_words
        self.be = be

    def _args(self, **kw):
        A = BatchArgs()
        sc = self.w.scene
        A.order, A.wg_off, A.voff, A.eoff = _p(self.order), _p(self.wg_off), _p(self.voff), _p(self.eoff)
        A.n_bodies = self.w.n_bodies
        for n in ("xhat", "G", "Gt", "dx", "r", "xt"):
            setattr(A, n, _p(self.ws[n]))
        A.cv = _p(self.cv)
        A.Dv, A.vdT, A.lconn = _p(self.Dv), _p(self.vdT), _p(self.lconn)
        A.stats = _p(self.stats)
        A.tol, A.adj_tol = sc["tol_rel"], sc["adj_tol_rel"]
        A.max_newton, A.max_cg = sc["max_newton"], sc["max_cg"]
        A.nacc = self.nacc
        A.Fbuf = _p(self.Fbuf)
        A.E0, A.E1 = _p(self.E0), _p(self.E1)
        A.n_s = self.n_s
        if self.n_s:
            A.soff, A.slconn, A.sk, A.sil0, A.Sbuf = (_p(self.soff), _p(self.slconn), _p(self.sk), _p(self.sil0),
                                                      _p(self.Sbuf))
        for key, val in kw.items():
            setattr(A, key, val)
        return A

    def step(self, x0, v0, a, block=128, want_tail=1, lds_fill=-12345.0):
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        a = np.ascontiguousarray(a, dtype=np.float64)
        a32 = a.astype(np.float32)
        x1 = np.zeros_like(x0)
        v1 = np.zeros_like(x0)
        A = self._args(x0=_p(x0), v0=_p(v0) if self.be else None, a=_p(a), a32=_p(a32), x1=_p(x1),
                       v1=_p(v1) if self.be else None, want_tail=want_tail)
        self.lib.emu_batched(self.w.dim, self.prec, 0, block, ctypes.byref(self.m), ctypes.byref(self.sc),
                             ctypes.byref(A), ctypes.c_double(lds_fill), ctypes.byref(self._left))
        self.lds_left = self._left.value
        self._check_indices()
        return x1, (v1 if self.be else None), self.stats.copy()

    def _check_indices(self):
        """The body logic's index checks (built with ISB_DEBUG): raise IndexError naming the check
        that saw an index out of range during the last launch (1: LDS vertex, 2: element corner,
        3: spring end); the check resets."""
        site = self.lib.emu_debug_site(1)
        if site != 0 and not self.allow_index_errors:
            raise IndexError(f"index check {site} saw an index out of range")
        self.last_index_site = site

    def adjoint(self, x1, x0, a, xbar, vbar=None, block=128, lds_fill=-12345.0, w_init=None):
        """w_init: the starting point of the adjoint CG (ISB_OPT_ADJ_WARM_START), else zero."""
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (x1, x0, a, xbar)]
        vb = None if vbar is None else np.ascontiguousarray(vbar, dtype=np.float64)
        a32 = arrs[2].astype(np.float32)
        wv = np.zeros_like(arrs[0]) if w_init is None else np.array(w_init, dtype=np.float64)
        A = self._args(x1=_p(arrs[0]), x0=_p(arrs[1]), a=_p(arrs[2]), a32=_p(a32), xbar=_p(arrs[3]),
                       vbar=None if vb is None else _p(vb), w=_p(wv), adj_warm=int(w_init is not None))
        self.lib.emu_batched(self.w.dim, self.prec, 1, block, ctypes.byref(self.m), ctypes.byref(self.sc),
                             ctypes.byref(A), ctypes.c_double(lds_fill), ctypes.byref(self._left))
        self.lds_left = self._left.value
        self._check_indices()
        return wv, self.stats.copy()
