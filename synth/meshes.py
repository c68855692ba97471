"""Seeded synthetic meshes and inputs shared by the oracle and the GPU path.

This module only lays out geometry, connectivity, masks and random draws. It
holds none of the simulation's arithmetic (no energies, no derivatives, no
solver), so that the oracle and the HIP path can both consume its output
without sharing any of the method.

Mesh conventions (the paper fixes none of them; they are readings):
  * 2D: unit quads, vertex id = j*(nx+1) + i, position (i, j); each quad
    (v00, v10, v11, v01) is split into (v00, v10, v11) and (v00, v11, v01),
    both counter-clockwise, so every triangle has positive signed area.
  * 3D: unit cubes, vertex id = (k*(ny+1) + j)*(nx+1) + i, position (i, j, k)
    with y up; each cube is split into the six Kuhn tetrahedra that share the
    main diagonal v000-v111, each reordered to positive orientation.
  * The body's lowest row/face sits on the ground plane y = 0.
"""
from __future__ import annotations

import itertools

import numpy as np

SEED_ROOT = 210205791


def rng(*sub: int) -> np.random.Generator:
    """Seeded generator for one config / sub-stream: default_rng([root, *sub])."""
    return np.random.default_rng([SEED_ROOT, *sub])


def tri_grid(nx: int, ny: int, origin=(0.0, 0.0)):
    """Regular triangulation of an nx-by-ny block of unit quads.

    Returns X (float64 [(nx+1)(ny+1), 2]) and T (int32 [2*nx*ny, 3]).
    """
    if nx < 1 or ny < 1:
        raise ValueError("tri_grid needs nx, ny >= 1")
    j, i = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = np.stack([i.ravel(), j.ravel()], axis=1).astype(np.float64)
    X += np.asarray(origin, dtype=np.float64)
    vid = lambda ii, jj: jj * (nx + 1) + ii
    qj, qi = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    qi = qi.ravel()
    qj = qj.ravel()
    v00 = vid(qi, qj)
    v10 = vid(qi + 1, qj)
    v11 = vid(qi + 1, qj + 1)
    v01 = vid(qi, qj + 1)
    T = np.empty((2 * nx * ny, 3), dtype=np.int32)
    T[0::2] = np.stack([v00, v10, v11], axis=1)
    T[1::2] = np.stack([v00, v11, v01], axis=1)
    return X, T


def _kuhn_paths():
    """The six monotone lattice paths from corner 000 to 111 (one per axis order)."""
    paths = []
    for perm in itertools.permutations(range(3)):
        c = [0, 0, 0]
        corners = [tuple(c)]
        for ax in perm:
            c[ax] += 1
            corners.append(tuple(c))
        sign = np.linalg.det(np.eye(3)[list(perm)])
        if sign < 0:
            corners[1], corners[2] = corners[2], corners[1]
        paths.append(corners)
    return paths


def tet_grid(nx: int, ny: int, nz: int, origin=(0.0, 0.0, 0.0), block: int = 4):
    """Kuhn (Freudenthal) split of an nx-by-ny-by-nz block of unit cubes.

    Returns X (float64 [(nx+1)(ny+1)(nz+1), 3]) and T (int32 [6*nx*ny*nz, 4]),
    every tetrahedron positively oriented. Vertices are numbered x fastest; the cubes (six
    tetrahedra each, consecutive) come in block x block x block groups, the groups in x-fastest
    order and the cubes x-fastest inside a group: a locality order, so that runs of consecutive
    elements cover compact regions (block = 1 gives plain x-fastest cube order).
    """
    if min(nx, ny, nz) < 1:
        raise ValueError("tet_grid needs nx, ny, nz >= 1")
    if block < 1:
        raise ValueError("tet_grid needs block >= 1")
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    X += np.asarray(origin, dtype=np.float64)
    vid = lambda ii, jj, kk: (kk * (ny + 1) + jj) * (nx + 1) + ii
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    B = int(block)
    order = np.lexsort((ci.ravel() % B, cj.ravel() % B, ck.ravel() % B,
                        ci.ravel() // B, cj.ravel() // B, ck.ravel() // B))
    ci = ci.ravel()[order]
    cj = cj.ravel()[order]
    ck = ck.ravel()[order]
    tets = []
    for corners in _kuhn_paths():
        tets.append(np.stack([vid(ci + a, cj + b, ck + c) for (a, b, c) in corners], axis=1))
    T = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return X, T


def left_column_pins(X: np.ndarray) -> np.ndarray:
    """Dirichlet mask [n_v, d] (uint8): every DOF of the vertices with X_x == min X_x."""
    pinned = np.zeros(X.shape, dtype=np.uint8)
    pinned[np.isclose(X[:, 0], X[:, 0].min())] = 1
    return pinned


def grid_springs(nx: int, ny: int) -> np.ndarray:
    """The horizontal edges of tri_grid(nx, ny) as vertex pairs (left, right): int32 [nx (ny+1), 2]."""
    j, i = np.meshgrid(np.arange(ny + 1), np.arange(nx), indexing="ij")
    left = (j * (nx + 1) + i).ravel()
    return np.stack([left, left + 1], axis=1).astype(np.int32)


def contraction_actuation(gen: np.random.Generator, shape, umax: float = 0.3) -> np.ndarray:
    """Actuation a = 1 - u with u ~ U[0, umax): a = 1 relaxed, a < 1 contracts."""
    return 1.0 - gen.uniform(0.0, umax, size=shape)


def x_fibres(n_e: int, dim: int) -> np.ndarray:
    """Unit material-space fibre direction e_x for every element."""
    f = np.zeros((n_e, dim), dtype=np.float64)
    f[:, 0] = 1.0
    return f


def concat_bodies(bodies):
    """Concatenate (X, T, pinned) bodies into one mesh with body offsets.

    Returns X, T (global vertex ids), pinned, body_v_off, body_e_off.
    """
    Xs, Ts, Ps = [], [], []
    v_off = [0]
    e_off = [0]
    for X, T, P in bodies:
        Xs.append(X)
        Ts.append(T + v_off[-1])
        Ps.append(P)
        v_off.append(v_off[-1] + X.shape[0])
        e_off.append(e_off[-1] + T.shape[0])
    return (np.concatenate(Xs), np.concatenate(Ts).astype(np.int32), np.concatenate(Ps),
            np.asarray(v_off, dtype=np.int64), np.asarray(e_off, dtype=np.int64))
