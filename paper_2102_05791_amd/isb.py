"""ctypes binding of libisb.so (the C ABI in include/isb.h).

Argument marshalling only: every computation runs in the HIP library. Methods of `Context`
carry the C names without the `isb_` prefix (isb_step -> Context.step, ...). Device arrays
are torch CUDA tensors (float64, contiguous, on the context's device); PyTorch supplies
device memory and the current stream, nothing else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisb.so")

ISB_OK, ISB_E_ARG, ISB_E_MESH, ISB_E_HIP, ISB_E_NOT_CONVERGED, ISB_E_NONFINITE, ISB_E_STATE = range(7)
STATUS_NAMES = {0: "ISB_OK", 1: "ISB_E_ARG", 2: "ISB_E_MESH", 3: "ISB_E_HIP", 4: "ISB_E_NOT_CONVERGED",
                5: "ISB_E_NONFINITE", 6: "ISB_E_STATE"}
ISB_FP64, ISB_MIXED = 0, 1
ISB_QUASISTATIC, ISB_BACKWARD_EULER = 0, 1
(OPT_SOLVER, OPT_SCATTER, OPT_GRAPH_SAFE, OPT_BLOCK, OPT_CG_CHECK, OPT_PRECISION, OPT_ENERGY, OPT_FORWARD,
 OPT_LBFGS_MEMORY, OPT_LBFGS_MAX_ITERS, OPT_CG_GRAPH, OPT_FP64_FALLBACK, OPT_ADJ_WARM_START,
 OPT_COMPACT_REST, OPT_PATCH_BLOCK, OPT_CG_SINGLE_REDUCTION, OPT_CG_RESIDENT,
 OPT_CG_BARRIER_LIMIT_US) = range(18)
FLAG_CONVERGED, FLAG_STAGNATED, FLAG_NONFINITE, FLAG_ADJ_CONVERGED, FLAG_FP64_FALLBACK = 1, 2, 4, 8, 16
FLAG_INVALID_ACTION = 32
FORWARD_NEWTON, FORWARD_LBFGS = 0, 1
# isotropic element energies (ISB_ENERGY_*), by the names the synthetic workloads use
ENERGY = {"nh": 0, "stvk": 1, "corot": 2, "snh": 3}
(INFO_N_VERTICES, INFO_N_ELEMENTS, INFO_N_BODIES, INFO_DIM, INFO_N_COLOURS, INFO_LDS_BYTES,
 INFO_COMPACT_AXIS, INFO_RESIDENT) = range(100, 108)

EXPORTED = ("isb_create", "isb_destroy", "isb_last_error", "isb_version", "isb_validate_mesh",
            "isb_colour_elements", "isb_mesh_upload", "isb_material_upload", "isb_set_scene",
            "isb_set_option", "isb_get_option", "isb_get_mass", "isb_step", "isb_solve_adjoint",
            "isb_vjp_params", "isb_energy", "isb_gradient", "isb_hessvec", "isb_hessvec_elements",
            "isb_hessdiag", "isb_stream_copy", "isb_spring_upload", "isb_vjp_spring_stiffness",
            "isb_gradient_elements", "isb_locality_order", "isb_wave_order", "isb_autotune",
            "isb_hessvec_noalloc")


class IsbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("adj_cg_iters", ctypes.c_int32), ("ls_backtracks", ctypes.c_int32),
                ("negcurv_exits", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("res0", ctypes.c_double), ("res_final", ctypes.c_double),
                ("adj_res_final", ctypes.c_double), ("energy", ctypes.c_double),
                ("min_J", ctypes.c_double), ("max_J", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Scene(ctypes.Structure):
    _fields_ = [("integrator", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("max_cg", ctypes.c_int32), ("pad_", ctypes.c_int32), ("h", ctypes.c_double),
                ("gravity", ctypes.c_double), ("k_contact", ctypes.c_double),
                ("k_friction", ctypes.c_double), ("eps_friction", ctypes.c_double),
                ("tol_rel", ctypes.c_double), ("adj_tol_rel", ctypes.c_double)]

    @classmethod
    def from_dict(cls, d: dict) -> "Scene":
        integ = d["integrator"]
        if isinstance(integ, str):
            integ = {"qs": ISB_QUASISTATIC, "be": ISB_BACKWARD_EULER}[integ]
        return cls(int(integ), int(d["max_newton"]), int(d["max_cg"]), 0, float(d["h"]),
                   float(d["gravity"]), float(d["k_contact"]), float(d["k_friction"]),
                   float(d["eps_friction"]), float(d["tol_rel"]), float(d["adj_tol_rel"]))


_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load the in-tree libisb.so (or the build at `path`, which is not cached); raises ImportError
    when it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    # torch ships its own HIP runtime under the same soname; loading torch first makes the library
    # bind to that one copy, so that both share one runtime, one device context and its streams
    import torch  # noqa: F401
    if not os.path.exists(p):
        raise ImportError(f"libisb.so not found at {p}; build it with "
                          "`python -m paper_2102_05791_amd.build_lib`")
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sigs = {
        "isb_create": [ctypes.c_int, ctypes.c_int, P(vp)],
        "isb_destroy": [vp],
        "isb_validate_mesh": [ctypes.c_int, i64, vp, i64, vp, i32, vp, vp],
        "isb_colour_elements": [ctypes.c_int, i64, i64, vp, vp, P(i32)],
        "isb_locality_order": [ctypes.c_int, i64, vp, i64, vp, i32, vp, vp],
        "isb_wave_order": [ctypes.c_int, i64, i64, vp, i32, vp, vp],
        "isb_autotune": [vp, vp, vp, vp, vp, vp],
        "isb_mesh_upload": [vp, ctypes.c_int, i32, vp, vp, vp, vp, vp],
        "isb_material_upload": [vp, vp, vp, vp, vp, vp, P(Scene)],
        "isb_set_scene": [vp, P(Scene)],
        "isb_set_option": [vp, ctypes.c_int, i64],
        "isb_get_option": [vp, ctypes.c_int, P(i64)],
        "isb_get_mass": [vp, vp, vp],
        "isb_step": [vp, vp, vp, vp, vp, vp, vp, vp],
        "isb_solve_adjoint": [vp, vp, vp, vp, vp, vp, vp, vp, vp],
        "isb_vjp_params": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
        "isb_energy": [vp, vp, vp, vp, vp, vp, vp],
        "isb_gradient": [vp, vp, vp, vp, vp, vp, vp],
        "isb_hessvec": [vp, vp, vp, vp, vp, vp, vp],
        "isb_hessvec_noalloc": [vp, vp, vp, vp, vp, vp, vp],
        "isb_hessvec_elements": [vp, vp, vp, vp, vp, vp],
        "isb_hessdiag": [vp, vp, vp, vp, vp, vp],
        "isb_gradient_elements": [vp, vp, vp, vp, vp],
        "isb_stream_copy": [vp, vp, vp, i64],
        "isb_spring_upload": [vp, i64, vp, vp, vp],
        "isb_vjp_spring_stiffness": [vp, vp, vp, vp, vp, vp],
    }
    for name, argtypes in sigs.items():
        f = getattr(lib, name)
        f.argtypes = argtypes
        f.restype = ctypes.c_int
    lib.isb_last_error.restype = ctypes.c_char_p
    lib.isb_last_error.argtypes = []
    lib.isb_version.restype = ctypes.c_char_p
    lib.isb_version.argtypes = []
    if path is None:
        _lib = lib
    return lib


def _check(lib, status: int, allow=()):
    if status != ISB_OK and status not in allow:
        raise IsbError(status, lib.isb_last_error().decode())
    return status


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def validate_mesh(dim, X, T, body_v_off=None, body_e_off=None):
    """isb_validate_mesh on host arrays; returns (status, message)."""
    lib = load_library()
    X, pX = _host(X, np.float64)
    T, pT = _host(T, np.int32)
    vo = np.array([0, X.shape[0]] if body_v_off is None else body_v_off, dtype=np.int64)
    eo = np.array([0, T.shape[0]] if body_e_off is None else body_e_off, dtype=np.int64)
    vo, pvo = _host(vo, np.int64)
    eo, peo = _host(eo, np.int64)
    st = lib.isb_validate_mesh(dim, X.shape[0], pX, T.shape[0], pT, len(vo) - 1, pvo, peo)
    return st, lib.isb_last_error().decode()


def colour_elements(dim, n_v, T):
    """isb_colour_elements: (colour per element, number of colours)."""
    lib = load_library()
    T, pT = _host(T, np.int32)
    col = np.zeros(T.shape[0], dtype=np.int32)
    nc = ctypes.c_int32(0)
    _check(lib, lib.isb_colour_elements(dim, n_v, T.shape[0], pT, col.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(nc)))
    return col, nc.value


def locality_order(dim, X, T, body_e_off=None):
    """isb_locality_order: the element permutation (new position -> element) of a locality order."""
    lib = load_library()
    X, pX = _host(X, np.float64)
    T, pT = _host(T, np.int32)
    perm = np.zeros(T.shape[0], dtype=np.int64)
    if body_e_off is None:
        _check(lib, lib.isb_locality_order(dim, X.shape[0], pX, T.shape[0], pT, 1, None,
                                           perm.ctypes.data_as(ctypes.c_void_p)))
    else:
        eo, peo = _host(body_e_off, np.int64)
        _check(lib, lib.isb_locality_order(dim, X.shape[0], pX, T.shape[0], pT, len(eo) - 1, peo,
                                           perm.ctypes.data_as(ctypes.c_void_p)))
    return perm


def wave_order(dim, n_v, T, body_e_off=None):
    """isb_wave_order: the element permutation (new position -> element) that packs each patch's
    wavefront groups with distinct vertices per corner slot; it keeps the patches."""
    lib = load_library()
    T, pT = _host(T, np.int32)
    perm = np.zeros(T.shape[0], dtype=np.int64)
    if body_e_off is None:
        _check(lib, lib.isb_wave_order(dim, int(n_v), T.shape[0], pT, 1, None,
                                       perm.ctypes.data_as(ctypes.c_void_p)))
    else:
        eo, peo = _host(body_e_off, np.int64)
        _check(lib, lib.isb_wave_order(dim, int(n_v), T.shape[0], pT, len(eo) - 1, peo,
                                       perm.ctypes.data_as(ctypes.c_void_p)))
    return perm


def _dev(t, name="tensor"):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def stream_copy(src, dst):
    """isb_stream_copy: dst[:] = src[:] by the library's streaming copy kernel (bandwidth probe)."""
    lib = load_library()
    if src.numel() != dst.numel():
        raise ValueError("stream_copy: sizes differ")
    _check(lib, lib.isb_stream_copy(_stream(), _dev(src, "src"), _dev(dst, "dst"), src.numel()))
    return dst


class Context:
    """One isb_ctx: a mesh of independent bodies on one GPU, plus material and scene."""

    def __init__(self, device: int = 0, precision: str | int = "fp64"):
        self.lib = load_library()
        prec = {"fp64": ISB_FP64, "mixed": ISB_MIXED}.get(precision, precision)
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.isb_create(int(device), int(prec), ctypes.byref(h)))
        self.h = h
        self.device = device
        self.precision = prec
        self.dim = self.n_v = self.n_e = self.n_bodies = self.n_s = 0
        self.scene = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.isb_destroy(h)
            self.h = None

    def close(self):
        self.__del__()

    # ---- upload ----
    def mesh_upload(self, dim, X, T, pinned=None, body_v_off=None, body_e_off=None):
        X, pX = _host(X, np.float64)
        T, pT = _host(T, np.int32)
        P = np.zeros(X.shape, np.uint8) if pinned is None else pinned
        P, pP = _host(P, np.uint8)
        vo, pvo = _host([0, X.shape[0]] if body_v_off is None else body_v_off, np.int64)
        eo, peo = _host([0, T.shape[0]] if body_e_off is None else body_e_off, np.int64)
        _check(self.lib, self.lib.isb_mesh_upload(self.h, int(dim), len(vo) - 1, pvo, peo, pX, pT, pP))
        self.dim, self.n_v, self.n_e, self.n_bodies = int(dim), X.shape[0], T.shape[0], len(vo) - 1
        self.body_v_off, self.body_e_off = vo.copy(), eo.copy()
        self.n_s = 0

    def spring_upload(self, pairs, k, body_s_off=None):
        """isb_spring_upload: vertex-pair springs (i, j) = pairs[s] with stiffness k[s]; their actions
        follow the elements' in every action vector, which then has n_e + n_s entries."""
        S, pS = _host(np.asarray(pairs).reshape(-1, 2), np.int32)
        K, pK = _host(k, np.float64)
        if K.shape != (S.shape[0],):
            raise ValueError("one stiffness per spring")
        so, pso = (None, None) if body_s_off is None else _host(body_s_off, np.int64)
        _check(self.lib, self.lib.isb_spring_upload(self.h, S.shape[0], pso, pS, pK))
        self.n_s = S.shape[0]

    @property
    def n_act(self):
        """Length of an action vector: one per element, then one per spring."""
        return self.n_e + self.n_s

    def _a(self, a, name="a"):
        if a.numel() != self.n_act:
            raise ValueError(f"{name} must have n_e + n_s = {self.n_act} entries, got {a.numel()}")
        return _dev(a, name)

    def material_upload(self, mu, lam, kf, fdir, rho, scene: dict):
        arrs = [_host(a, np.float64) for a in (mu, lam, kf, fdir, rho)]
        sc = Scene.from_dict(scene)
        _check(self.lib, self.lib.isb_material_upload(self.h, *[p for _, p in arrs], ctypes.byref(sc)))
        self.scene = dict(scene)
        # host copies: the differentiable step re-uploads the Lame pair and k_f when they change
        self.material = {k: a.copy() for k, (a, _) in zip(("mu", "lam", "kf", "fdir", "rho"), arrs)}

    def set_material_params(self, mu, lam, kf):
        """Upload a new Lame pair and fibre stiffness per element (host or device arrays [n_e]),
        keeping the fibre directions, densities and scene; no-op when the values are unchanged."""
        new = [np.ascontiguousarray(v.detach().cpu().numpy() if hasattr(v, "detach") else v, dtype=np.float64)
               for v in (mu, lam, kf)]
        old = self.material
        if all(np.array_equal(n, old[k]) for n, k in zip(new, ("mu", "lam", "kf"))):
            return False
        self.material_upload(new[0], new[1], new[2], old["fdir"], old["rho"], self.scene)
        return True

    def set_scene(self, scene: dict):
        sc = Scene.from_dict(scene)
        _check(self.lib, self.lib.isb_set_scene(self.h, ctypes.byref(sc)))
        self.scene = dict(scene)

    def set_option(self, key: int, value: int):
        _check(self.lib, self.lib.isb_set_option(self.h, int(key), int(value)))

    def get_option(self, key: int) -> int:
        v = ctypes.c_int64(0)
        _check(self.lib, self.lib.isb_get_option(self.h, int(key), ctypes.byref(v)))
        return v.value

    @classmethod
    def from_workload(cls, w, device=0, precision="fp64", solver=0, scatter=2):
        ctx = cls(device, precision)
        ctx.set_option(OPT_SCATTER, scatter)
        ctx.set_option(OPT_ENERGY, ENERGY[getattr(w, "model", "nh")])
        ctx.mesh_upload(w.dim, w.X, w.T, w.pinned, w.body_v_off, w.body_e_off)
        ctx.material_upload(w.mu, w.lam, w.kf, w.fdir, w.rho, w.scene)
        if getattr(w, "S", None) is not None and len(w.S) > 0:
            ctx.spring_upload(w.S, w.ks, w.body_s_off)
        ctx.set_option(OPT_SOLVER, solver)
        return ctx

    # ---- launch configuration ----
    def autotune(self, x0, v0, a, cache_path=None):
        """isb_autotune on (x0, v0, a): keeps the fastest workgroup size (batched) or scatter (plain)
        and returns {option key: value}. With cache_path, a JSON file keyed by device architecture,
        dimension, precision, solver, energy model and element-count bucket (powers of two) answers
        repeated questions without timing."""
        import json
        import math
        import torch
        key = None
        if cache_path:
            arch = getattr(torch.cuda.get_device_properties(self.device), "gcnArchName", "unknown")
            bucket = int(math.log2(max(self.n_e, 1)))
            key = (f"{arch}|dim{self.dim}|prec{self.precision}|solver{self.get_option(OPT_SOLVER)}|"
                   f"energy{self.get_option(OPT_ENERGY)}|ne2^{bucket}")
            try:
                with open(cache_path) as fh:
                    cache = json.load(fh)
            except (OSError, ValueError):
                cache = {}
            if key in cache:
                opt, val = cache[key]
                self.set_option(int(opt), int(val))
                return {int(opt): int(val)}
        chosen = (ctypes.c_int64 * 2)()
        _check(self.lib, self.lib.isb_autotune(self.h, _stream(), _dev(x0, "x0"), _dev(v0, "v0"), self._a(a),
                                               chosen))
        if key is not None:
            cache[key] = [int(chosen[0]), int(chosen[1])]
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        return {int(chosen[0]): int(chosen[1])}

    # ---- device helpers ----
    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float64, device=f"cuda:{self.device}")

    def _stats_buf(self, want):
        return (Stats * self.n_bodies)() if want else None

    def mass(self):
        m = self._empty(self.n_v)
        _check(self.lib, self.lib.isb_get_mass(self.h, _stream(), _dev(m)))
        return m

    # ---- the step and its adjoint ----
    def step(self, x0, v0, a, x1=None, v1=None, stats=True, allow_not_converged=False):
        """isb_step. Returns (x1, v1, [per-body stats dicts] or None, status)."""
        be = self.scene["integrator"] in ("be", ISB_BACKWARD_EULER)
        x1 = self._empty(self.n_v, self.dim) if x1 is None else x1
        if be and v1 is None:
            v1 = self._empty(self.n_v, self.dim)
        sb = self._stats_buf(stats)
        allow = (ISB_E_NOT_CONVERGED,) if allow_not_converged else ()
        st = _check(self.lib, self.lib.isb_step(self.h, _stream(), _dev(x0, "x0"), _dev(v0, "v0"), self._a(a),
                                                _dev(x1, "x1"), _dev(v1, "v1") if be else None, sb), allow)
        return x1, (v1 if be else None), ([s.as_dict() for s in sb] if sb is not None else None), st

    def solve_adjoint(self, x1, x0, a, x1_bar, v1_bar=None, w=None, stats=True, allow_not_converged=False,
                      w_init=None):
        """isb_solve_adjoint. Returns (w, per-body stats or None, status). w_init (device [n_v][dim]):
        the starting point of the adjoint CG for this call (ISB_OPT_ADJ_WARM_START), e.g. the adjoint
        of the step after in a backward pass through time; None starts from zero."""
        w = self._empty(self.n_v, self.dim) if w is None else w
        sb = self._stats_buf(stats)
        allow = (ISB_E_NOT_CONVERGED,) if allow_not_converged else ()
        prev = None
        if w_init is not None:
            _dev(w_init, "w_init")
            if w_init.data_ptr() != w.data_ptr():
                w.copy_(w_init)
            prev = self.get_option(OPT_ADJ_WARM_START)
            self.set_option(OPT_ADJ_WARM_START, 1)
        try:
            st = _check(self.lib, self.lib.isb_solve_adjoint(self.h, _stream(), _dev(x1, "x1"), _dev(x0, "x0"),
                                                             self._a(a), _dev(x1_bar, "x1_bar"),
                                                             _dev(v1_bar, "v1_bar"), _dev(w, "w"), sb), allow)
        finally:
            if prev is not None:
                self.set_option(OPT_ADJ_WARM_START, prev)
        return w, ([s.as_dict() for s in sb] if sb is not None else None), st

    def vjp_params(self, w, x1, x0, a, v1_bar=None, want=("a_bar", "x0_bar", "v0_bar", "mu_bar", "lam_bar",
                                                          "kf_bar")):
        """isb_vjp_params. Returns a dict of the requested cotangents."""
        out = {"a_bar": self._empty(self.n_act) if "a_bar" in want else None}
        for k in ("mu_bar", "lam_bar", "kf_bar"):
            out[k] = self._empty(self.n_e) if k in want else None
        for k in ("x0_bar", "v0_bar"):
            out[k] = self._empty(self.n_v, self.dim) if k in want else None
        _check(self.lib, self.lib.isb_vjp_params(
            self.h, _stream(), _dev(w), _dev(x1), _dev(x0), self._a(a), _dev(v1_bar), _dev(out["a_bar"]),
            _dev(out["x0_bar"]), _dev(out["v0_bar"]), _dev(out["mu_bar"]), _dev(out["lam_bar"]),
            _dev(out["kf_bar"])))
        return {k: v for k, v in out.items() if v is not None}

    def vjp_spring_stiffness(self, w, x1, a):
        """isb_vjp_spring_stiffness: k_bar [n_s] = -w^T dG/dk at x1."""
        kb = self._empty(self.n_s)
        if self.n_s:
            _check(self.lib, self.lib.isb_vjp_spring_stiffness(self.h, _stream(), _dev(w), _dev(x1), self._a(a),
                                                               _dev(kb)))
        return kb

    # ---- single evaluations ----
    def energy(self, x, x0, v0, a):
        e = self._empty(self.n_bodies)
        _check(self.lib, self.lib.isb_energy(self.h, _stream(), _dev(x), _dev(x0), _dev(v0), self._a(a), _dev(e)))
        return e

    def gradient(self, x, x0, v0, a):
        g = self._empty(self.n_v, self.dim)
        _check(self.lib, self.lib.isb_gradient(self.h, _stream(), _dev(x), _dev(x0), _dev(v0), self._a(a), _dev(g)))
        return g

    def hessvec(self, x, x0, a, p):
        hp = self._empty(self.n_v, self.dim)
        _check(self.lib, self.lib.isb_hessvec(self.h, _stream(), _dev(x), _dev(x0), self._a(a), _dev(p), _dev(hp)))
        return hp

    def hessvec_noalloc(self, x, x0, a, p, hp):
        """isb_hessvec_noalloc: hp = P H(x) P p into the caller's hp, staged in the library's fixed
        device scratch (no allocation, here or in the library)."""
        _check(self.lib, self.lib.isb_hessvec_noalloc(self.h, _stream(), _dev(x), _dev(x0), self._a(a), _dev(p),
                                                      _dev(hp)))
        return hp

    def hessvec_elements(self, x, a, p, hp):
        """isb_hessvec_elements: hp += element part of H(x) p (no vertex terms, no projection)."""
        _check(self.lib, self.lib.isb_hessvec_elements(self.h, _stream(), _dev(x), self._a(a), _dev(p), _dev(hp)))
        return hp

    def gradient_elements(self, x, a, g):
        """isb_gradient_elements: g += element (and spring) part of grad g(x) (no vertex terms)."""
        _check(self.lib, self.lib.isb_gradient_elements(self.h, _stream(), _dev(x), self._a(a), _dev(g)))
        return g

    def hessdiag(self, x, x0, a):
        d = self._empty(self.n_v, self.dim)
        _check(self.lib, self.lib.isb_hessdiag(self.h, _stream(), _dev(x), _dev(x0), self._a(a), _dev(d)))
        return d
