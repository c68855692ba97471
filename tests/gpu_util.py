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


def problems(w):
    """Oracle Problem per body."""
    return [Problem.from_workload(w.body(b)) for b in range(w.n_bodies)]


def abs_assembly(prob: Problem, x, x0, v0, a):
    """|contributions| assembled per DOF: the scale of the gradient's rounding (A17-style measure)."""
    F = prob.mesh.F(x)
    cg = np.abs(fem.corner_grads(prob.mesh, fem.stress(F, prob.mu, prob.lam, prob.kf, a, prob.fd)))
    G = np.zeros_like(x)
    np.add.at(G, prob.mesh.T, cg)
    G = prob.s_pot * (G + np.abs(prob.vertex_grad(x, x0)))
    if prob.be:
        G += np.abs(prob.mesh.mass[:, None] * (x - prob.x_hat(x0, v0)))
    return G


def rel(a, b, scale=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b if scale is None else scale)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))
