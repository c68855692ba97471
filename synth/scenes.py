"""The five synthetic workloads, with every constant and seed in one place.

Each builder returns a `Workload`: mesh, per-element material arrays, scene
constants, initial state and the per-step actuation draws. Material parameters
are plain inputs here (Lame pair from Young's modulus and Poisson ratio, fibre
stiffness k_f = E, density 1); no energy or derivative is evaluated.

Sizes:
  qs_cantilever   10x4 quads, 80 triangles, 55 vertices, quasistatic, left column pinned
  be_strip        64x16 quads, 2048 triangles, 1105 vertices, backward Euler, 100 steps
  batched_strips  512 bodies, s ~ U{4..32}, grid 4s x s, 50 steps
  tet_block       64x32x32 cubes, 393216 Kuhn tets, 70785 vertices, 20 steps
  be_spring_strip, batched_spring_strips: the strips with the fibres as vertex-pair springs on
                  the horizontal grid edges (k = E per unit quad) and passive triangles (k_f = 0)

Action arrays hold, per step, the elements' actions and then the springs'.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import meshes

SCENE_KEYS = ("integrator", "h", "gravity", "k_contact", "k_friction", "eps_friction",
              "tol_rel", "adj_tol_rel", "max_newton", "max_cg")


def lame(E: float, nu: float):
    """Lame parameters (mu, lambda) of Young's modulus E and Poisson ratio nu."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def scene(integrator="be", h=1.0 / 60.0, gravity=9.8, k_contact=1e5, k_friction=1e3,
          eps_friction=1e-2, tol_rel=1e-6, adj_tol_rel=1e-6, max_newton=50, max_cg=1000):
    return dict(integrator=integrator, h=float(h), gravity=float(gravity),
                k_contact=float(k_contact), k_friction=float(k_friction),
                eps_friction=float(eps_friction), tol_rel=float(tol_rel),
                adj_tol_rel=float(adj_tol_rel), max_newton=int(max_newton), max_cg=int(max_cg))


@dataclass
class Workload:
    name: str
    dim: int
    X: np.ndarray            # [n_v, d] rest positions
    T: np.ndarray            # [n_e, d+1] int32
    pinned: np.ndarray       # [n_v, d] uint8
    mu: np.ndarray           # [n_e]
    lam: np.ndarray          # [n_e]
    kf: np.ndarray           # [n_e]
    fdir: np.ndarray         # [n_e, d] unit
    rho: np.ndarray          # [n_e]
    scene: dict
    x0: np.ndarray           # [n_v, d]
    v0: np.ndarray           # [n_v, d]
    actions: np.ndarray      # [steps, n_e + n_s]
    body_v_off: np.ndarray = field(default=None)
    body_e_off: np.ndarray = field(default=None)
    S: np.ndarray = field(default=None)           # [n_s, 2] int32 vertex pairs (global ids)
    ks: np.ndarray = field(default=None)          # [n_s] spring stiffness
    body_s_off: np.ndarray = field(default=None)  # [n_bodies + 1]
    model: str = "nh"  # isotropic element energy: nh (Eq. 3), stvk, corot, snh

    def __post_init__(self):
        if self.body_v_off is None:
            self.body_v_off = np.array([0, self.X.shape[0]], dtype=np.int64)
        if self.body_e_off is None:
            self.body_e_off = np.array([0, self.T.shape[0]], dtype=np.int64)
        if self.S is None:
            self.S = np.zeros((0, 2), np.int32)
            self.ks = np.zeros(0)
        if self.body_s_off is None:
            self.body_s_off = np.zeros(len(self.body_v_off), dtype=np.int64)
            self.body_s_off[-1] = self.S.shape[0]

    @property
    def n_s(self):
        return self.S.shape[0]

    @property
    def n_v(self):
        return self.X.shape[0]

    @property
    def n_e(self):
        return self.T.shape[0]

    @property
    def n_bodies(self):
        return len(self.body_v_off) - 1

    def body(self, b: int) -> "Workload":
        """The b-th body as a stand-alone single-body workload."""
        v0, v1 = int(self.body_v_off[b]), int(self.body_v_off[b + 1])
        e0, e1 = int(self.body_e_off[b]), int(self.body_e_off[b + 1])
        s0, s1 = int(self.body_s_off[b]), int(self.body_s_off[b + 1])
        acts = np.concatenate([self.actions[:, e0:e1], self.actions[:, self.n_e + s0:self.n_e + s1]], axis=1)
        return Workload(f"{self.name}[{b}]", self.dim, self.X[v0:v1].copy(),
                        (self.T[e0:e1] - v0).astype(np.int32), self.pinned[v0:v1].copy(),
                        self.mu[e0:e1].copy(), self.lam[e0:e1].copy(), self.kf[e0:e1].copy(),
                        self.fdir[e0:e1].copy(), self.rho[e0:e1].copy(), dict(self.scene),
                        self.x0[v0:v1].copy(), self.v0[v0:v1].copy(), acts,
                        S=(self.S[s0:s1] - v0).astype(np.int32), ks=self.ks[s0:s1].copy(), model=self.model)

    def permute_elements(self, perm) -> "Workload":
        """The same workload with its elements in the order `perm` (new position -> element),
        which must keep each body's elements in that body's range: connectivity, per-element
        material and the elements' actions move together; vertices and springs stay."""
        perm = np.asarray(perm, dtype=np.int64)
        if perm.shape != (self.n_e,) or not np.array_equal(np.sort(perm), np.arange(self.n_e)):
            raise ValueError("perm is not a permutation of the elements")
        for b in range(self.n_bodies):
            e0, e1 = int(self.body_e_off[b]), int(self.body_e_off[b + 1])
            if e1 > e0 and (perm[e0:e1].min() < e0 or perm[e0:e1].max() >= e1):
                raise ValueError(f"perm moves an element out of body {b}")
        acts = self.actions.copy()
        acts[:, :self.n_e] = self.actions[:, perm]
        return Workload(self.name, self.dim, self.X, np.ascontiguousarray(self.T[perm]), self.pinned,
                        self.mu[perm], self.lam[perm], self.kf[perm], np.ascontiguousarray(self.fdir[perm]),
                        self.rho[perm], dict(self.scene), self.x0, self.v0, acts,
                        body_v_off=self.body_v_off, body_e_off=self.body_e_off, S=self.S, ks=self.ks,
                        body_s_off=self.body_s_off, model=self.model)


def _material(n_e, dim, E, nu):
    mu, lam = lame(E, nu)
    return (np.full(n_e, mu), np.full(n_e, lam), np.full(n_e, float(E)),
            meshes.x_fibres(n_e, dim), np.ones(n_e))


def qs_cantilever(tol_rel=1e-10, steps=1) -> Workload:
    """10x4 quasistatic cantilever: E=1e4, nu=0.3, gravity, left column pinned."""
    X, T = meshes.tri_grid(10, 4)
    mu, lam, kf, fd, rho = _material(T.shape[0], 2, 1e4, 0.3)
    acts = meshes.contraction_actuation(meshes.rng(1), (steps, T.shape[0]))
    sc = scene("qs", h=1.0 / 60.0, k_contact=0.0, k_friction=0.0, tol_rel=tol_rel, adj_tol_rel=1e-12)
    return Workload("qs_cantilever_10x4", 2, X, T, meshes.left_column_pins(X), mu, lam, kf, fd,
                    rho, sc, X.copy(), np.zeros_like(X), acts)


def be_strip(nx=64, ny=16, steps=100, seed_cfg=2, tol_rel=1e-6) -> Workload:
    """Backward-Euler strip resting on the ground: h=1/60, k_c=1e5, k_fr=1e3, eps=1e-2."""
    X, T = meshes.tri_grid(nx, ny)
    mu, lam, kf, fd, rho = _material(T.shape[0], 2, 1e4, 0.3)
    acts = meshes.contraction_actuation(meshes.rng(seed_cfg), (steps, T.shape[0]))
    sc = scene("be", h=1.0 / 60.0, tol_rel=tol_rel)
    return Workload(f"be_strip_{nx}x{ny}", 2, X, T, np.zeros(X.shape, np.uint8), mu, lam, kf, fd,
                    rho, sc, X.copy(), np.zeros_like(X), acts)


def batched_sizes(n_bodies=512):
    """Body scale s_b ~ U{4..32}; body b is a (4 s_b) x s_b strip."""
    return meshes.rng(4).integers(4, 33, size=n_bodies)


def batched_strips(n_bodies=512, steps=50, tol_rel=1e-6, sizes=None) -> Workload:
    """Many strips of uneven size, concatenated with body offsets (C2 physics)."""
    if sizes is None:
        sizes = batched_sizes(n_bodies)
    bodies, acts = [], []
    for b, s in enumerate(sizes):
        X, T = meshes.tri_grid(4 * int(s), int(s))
        bodies.append((X, T, np.zeros(X.shape, np.uint8)))
        acts.append(meshes.contraction_actuation(meshes.rng(4, b), (steps, T.shape[0])))
    X, T, P, voff, eoff = meshes.concat_bodies(bodies)
    mu, lam, kf, fd, rho = _material(T.shape[0], 2, 1e4, 0.3)
    sc = scene("be", h=1.0 / 60.0, tol_rel=tol_rel)
    return Workload(f"batched_strips_{len(sizes)}", 2, X, T, P, mu, lam, kf, fd, rho, sc,
                    X.copy(), np.zeros_like(X), np.concatenate(acts, axis=1), voff, eoff)


def tet_block(nx=64, ny=32, nz=32, steps=20, tol_rel=1e-6) -> Workload:
    """3D block of Kuhn tets: E=1e5, nu=0.45, h=1/30, contact and friction on the floor."""
    X, T = meshes.tet_grid(nx, ny, nz)
    mu, lam, kf, fd, rho = _material(T.shape[0], 3, 1e5, 0.45)
    acts = meshes.contraction_actuation(meshes.rng(5), (steps, T.shape[0]))
    sc = scene("be", h=1.0 / 30.0, tol_rel=tol_rel)
    return Workload(f"tet_block_{nx}x{ny}x{nz}", 3, X, T, np.zeros(X.shape, np.uint8), mu, lam,
                    kf, fd, rho, sc, X.copy(), np.zeros_like(X), acts)


def be_spring_strip(nx=64, ny=16, steps=100, seed_cfg=6, tol_rel=1e-6) -> Workload:
    """be_strip with the fibres moved to springs: passive triangles (k_f = 0) and one spring of
    stiffness E on each horizontal grid edge (the fibre of one unit quad), actuated at random."""
    w = be_strip(nx, ny, steps, tol_rel=tol_rel)
    S = meshes.grid_springs(nx, ny)
    E = float(w.kf[0])
    acts = np.concatenate([np.ones((steps, w.n_e)),
                           meshes.contraction_actuation(meshes.rng(seed_cfg), (steps, S.shape[0]))], axis=1)
    return Workload(f"be_spring_strip_{nx}x{ny}", 2, w.X, w.T, w.pinned, w.mu, w.lam, np.zeros(w.n_e),
                    w.fdir, w.rho, w.scene, w.x0, w.v0, acts, S=S, ks=np.full(S.shape[0], E))


def batched_spring_strips(n_bodies=512, steps=50, tol_rel=1e-6, sizes=None) -> Workload:
    """batched_strips with spring fibres: body b is a (4 s_b) x s_b strip, s_b ~ U{4..32}, with
    passive triangles and a spring on each horizontal grid edge."""
    if sizes is None:
        sizes = batched_sizes(n_bodies)
    bodies, springs, eacts, sacts = [], [], [], []
    for b, s in enumerate(sizes):
        X, T = meshes.tri_grid(4 * int(s), int(s))
        bodies.append((X, T, np.zeros(X.shape, np.uint8)))
        springs.append(meshes.grid_springs(4 * int(s), int(s)))
        eacts.append(np.ones((steps, T.shape[0])))
        sacts.append(meshes.contraction_actuation(meshes.rng(7, b), (steps, springs[-1].shape[0])))
    X, T, P, voff, eoff = meshes.concat_bodies(bodies)
    soff = np.concatenate([[0], np.cumsum([sp.shape[0] for sp in springs])]).astype(np.int64)
    S = np.concatenate([sp + voff[b] for b, sp in enumerate(springs)]).astype(np.int32)
    mu, lam, kf, fd, rho = _material(T.shape[0], 2, 1e4, 0.3)
    sc = scene("be", h=1.0 / 60.0, tol_rel=tol_rel)
    return Workload(f"batched_spring_strips_{len(sizes)}", 2, X, T, P, mu, lam, np.zeros_like(kf), fd, rho,
                    sc, X.copy(), np.zeros_like(X), np.concatenate(eacts + sacts, axis=1), voff, eoff,
                    S=S, ks=np.full(S.shape[0], 1e4), body_s_off=soff)
