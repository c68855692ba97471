"""Write tests/golden/tet_block_step.json: one backward-Euler step of the 64x32x32 Kuhn-tet block
(393,216 tets, 70,785 vertices; E = 1e5, nu = 0.45, h = 1/30, contact and friction) and the adjoint
of L = -COM_x(x1), computed by the FP64 oracle only, stored at sampled vertices and elements.

Run from the repository root: python -m tests.golden.make_tet_block_golden
Inputs come from synth/ (seeded); every stored value comes from oracle/.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import solve  # noqa: E402
from oracle.fem import Problem  # noqa: E402
from synth import meshes, scenes  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tet_block_step.json")
TOL = 1e-12


def main():
    t0 = time.time()
    w = scenes.tet_block()
    p = Problem.from_workload(w)
    a = w.actions[0]
    x1, v1, st = solve.step(p, w.x0, w.v0, a, tol=TOL)
    print(f"step done in {time.time() - t0:.0f} s: {st['newton_iters']} Newton iterations", flush=True)
    xbar = solve.com_x_loss_grad(p, x1)
    wv = solve.adjoint(p, x1, w.x0, a, xbar)
    out = solve.vjp_params(p, wv, x1, w.x0, a)
    print(f"adjoint done in {time.time() - t0:.0f} s", flush=True)
    gen = meshes.rng(5, 99)
    vs = np.sort(gen.choice(w.n_v, 256, replace=False))
    es = np.sort(gen.choice(w.n_e, 256, replace=False))
    doc = {
        "_about": "Oracle-only reference for the tet-block workload (one backward-Euler step, Eq. 14, and the "
                  "adjoint of Eq. 9 for L = -COM_x(x1)), sampled. Written by tests/golden/make_tet_block_golden.py.",
        "workload": w.name, "n_v": int(w.n_v), "n_e": int(w.n_e), "tol_rel": TOL,
        "newton_iters": int(st["newton_iters"]), "res0": st["res0"], "res_final": st["res_final"],
        "loss": solve.com_x_loss(p, x1),
        "norm_dx": float(np.linalg.norm(x1 - w.x0)), "norm_v1": float(np.linalg.norm(v1)),
        "norm_w": float(np.linalg.norm(wv)), "norm_a_bar": float(np.linalg.norm(out["a_bar"])),
        "vertices": vs.tolist(), "x1": x1[vs].tolist(), "v1": v1[vs].tolist(), "w": wv[vs].tolist(),
        "elements": es.tolist(), "a_bar": out["a_bar"][es].tolist(), "mu_bar": out["mu_bar"][es].tolist(),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
