"""Shared helpers of the GPU parity tests (seeded inputs, oracle-side reference quantities)."""
import numpy as np

from oracle import fem
from oracle.fem import Problem
from synth import meshes, scenes
from synth.scenes import Workload


def rand_workload(dim, seed=0, integrator="be", pinned_left=False, bodies=1, shape=None):
    """Small body (or bodies) with per-element material variation and contact/friction active.

    2D default 40x13 quads (1040 triangles: four full 256-thread tiles plus a ragged tail);
    3D default 6x5x4 cubes (720 tets)."""
    rng = np.random.default_rng([20210211, dim, seed])
    parts = []
    for b in range(bodies):
        if dim == 2:
            nx, ny = shape or (40, 13)
            X, T = meshes.tri_grid(nx + 3 * b, ny)
        else:
            nx, ny, nz = shape or (6, 5, 4)
            X, T = meshes.tet_grid(nx + b, ny, nz)
        P = meshes.left_column_pins(X) if pinned_left else np.zeros(X.shape, np.uint8)
        parts.append((X, T, P))
    X, T, P, vo, eo = meshes.concat_bodies(parts)
    n_e = T.shape[0]
    E, nu = (1e4, 0.3) if dim == 2 else (1e5, 0.45)
    mu, lam = scenes.lame(E, nu)
    f = rng.normal(size=(n_e, dim))
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    sc = scenes.scene(integrator, h=1.0 / 60.0 if dim == 2 else 1.0 / 30.0)
    x0 = X + 0.02 * rng.normal(size=X.shape)
    x0[:, 1] -= 0.03                            # bottom row below ground: contact and friction active
    v0 = 0.5 * rng.normal(size=X.shape)
    acts = rng.uniform(0.7, 1.0, size=(4, n_e))
    w = Workload(f"rand{dim}d", dim, X, T, P, mu * rng.uniform(0.8, 1.2, n_e), lam * rng.uniform(0.8, 1.2, n_e),
                 E * rng.uniform(0.8, 1.2, n_e), f, rng.uniform(0.5, 1.5, n_e), sc, x0, v0, acts, vo, eo)
    return w, rng


def with_springs(w, rng, frac=0.5, extra=4, ks_scale=1.0):
    """The workload plus vertex-pair springs in every body: the first edge of a random `frac` of its
    elements (distinct pairs) and `extra` random pairs of its vertices (longer reaches), stiffness
    ~ U(0.5, 1.5) E (E = the elements' mean fibre stiffness), spring actions ~ U(0.7, 1) appended
    to every step's actions."""
    S, soff = [], [0]
    E = float(np.mean(w.kf)) if np.mean(w.kf) > 0 else 1e4
    for b in range(w.n_bodies):
        v0, v1 = int(w.body_v_off[b]), int(w.body_v_off[b + 1])
        e0, e1 = int(w.body_e_off[b]), int(w.body_e_off[b + 1])
        pick = rng.choice(np.arange(e0, e1), size=max(1, int(frac * (e1 - e0))), replace=False)
        pairs = {tuple(sorted((int(w.T[e, 0]), int(w.T[e, 1])))) for e in pick}
        while len(pairs) < len(pick) + extra:
            i, j = rng.integers(v0, v1, size=2)
            if i != j:
                pairs.add((int(i), int(j)))
        pairs = sorted(pairs)
        S.extend(pairs)
        soff.append(len(S))
    S = np.asarray(S, np.int32)
    ks = ks_scale * E * rng.uniform(0.5, 1.5, size=S.shape[0])
    acts = np.concatenate([w.actions, rng.uniform(0.7, 1.0, size=(w.actions.shape[0], S.shape[0]))], axis=1)
    return Workload(w.name + "+springs", w.dim, w.X, w.T, w.pinned, w.mu, w.lam, w.kf, w.fdir, w.rho, w.scene,
                    w.x0, w.v0, acts, w.body_v_off, w.body_e_off, S=S, ks=ks,
                    body_s_off=np.asarray(soff, np.int64))


def problems(w):
    """Oracle Problem per body."""
    return [Problem.from_workload(w.body(b)) for b in range(w.n_bodies)]


def abs_assembly(prob: Problem, x, x0, v0, a):
    """|contributions| assembled per DOF: the scale of the gradient's rounding (A17-style measure)."""
    ae, as_ = prob.split(a)
    F = prob.mesh.F(x)
    cg = np.abs(fem.corner_grads(prob.mesh, fem.stress(F, prob.mu, prob.lam, prob.kf, ae, prob.fd)))
    G = np.zeros_like(x)
    np.add.at(G, prob.mesh.T, cg)
    if prob.n_s:
        n, _, _, f = fem.spring_force_terms(x, prob.S, prob.ks, prob.l0, as_)
        np.add.at(G, prob.S[:, 0], np.abs(f[:, None] * n))
        np.add.at(G, prob.S[:, 1], np.abs(f[:, None] * n))
    G = prob.s_pot * (G + np.abs(prob.vertex_grad(x, x0)))
    if prob.be:
        G += np.abs(prob.mesh.mass[:, None] * (x - prob.x_hat(x0, v0)))
    return G


def rel(a, b, scale=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b if scale is None else scale)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def rel_inf(a, b, scale=None):
    """max |a - b| over max |b| (or over max |scale|): the worst entry, which a 2-norm measure can
    hide when a handful of entries (a ragged tail, a patch boundary) are wrong."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b if scale is None else scale)) if b.size else 0.0
    num = np.max(np.abs(a - b)) if a.size else 0.0
    return float(num / den) if den > 0 else float(num)
