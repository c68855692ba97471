"""Write tests/golden/bench_reference.json: the FP64 oracle's results for the benchmark's parity
checks, so that bench.py states the error of each leg against the oracle without running it:

* batched strips (512 bodies): the first backward-Euler step (Eq. 14 with contact and friction,
  Eq. 15-17) of bodies 0, 256 and 511;
* the same strips with the fibres as vertex-pair springs (Eq. 2 between two vertices): bodies 0, 511;
* the alternative element energies of Sec. 3 (St. Venant-Kirchhoff, corotated, stable neo-Hookean)
  on the batched strips: body 0;
* the 64x16 strip after 5 steps (the first-order solver leg);
* the 64x16 strip under the seeded 32-unit policy over a 100-step episode (Sec. 5.1): the reward
  and two projections of its gradient with respect to the policy's parameters.

Every stored state is the oracle's at relative residual 1e-13, sampled at up to 128 vertices per
body (seeded), with the norm of the full displacement for relative errors. The policy network is
plain PyTorch on the CPU on both sides; the steps of its episode are the oracle's (Newton with a
direct solve forward, the direct adjoint of Eq. 9 backward).

Run from the repository root: python -m tests.golden.make_bench_golden
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_reference.json")
TOL = 1e-13
N_SAMPLE = 128


def _sample(n_v, key):
    gen = meshes.rng(7, key)
    return np.sort(gen.choice(n_v, min(N_SAMPLE, n_v), replace=False))


def first_step(w, b, key):
    """The oracle's first step of body b of workload w, sampled."""
    wb = w.body(b)
    p = Problem.from_workload(wb)
    x1, v1, st = solve.step(p, wb.x0, wb.v0, wb.actions[0], tol=TOL)
    vs = _sample(wb.n_v, key)
    return {"body": int(b), "n_v": int(wb.n_v), "newton_iters": int(st["newton_iters"]),
            "vertices": vs.tolist(), "x1": x1[vs].tolist(), "v1": v1[vs].tolist(),
            "norm_dx": float(np.linalg.norm(x1 - wb.x0)), "norm_v1": float(np.linalg.norm(v1))}


def policy_episode(H=100, seed=0):
    import torch
    from paper_2102_05791_amd.policy import FibrePolicy, episode_reward
    from tests.oracle_layers import oracle_step
    w = scenes.be_strip(64, 16, steps=1)
    p = Problem.from_workload(w)
    pol = FibrePolicy(torch.from_numpy(p.mesh.mass.copy()), 2, w.n_e, seed=seed)
    r = episode_reward(p, pol, torch.from_numpy(w.x0.copy()), torch.from_numpy(np.zeros_like(w.x0)), H,
                       step=oracle_step)
    r.backward()
    g = np.concatenate([t.grad.numpy().ravel() for t in pol.parameters()])
    d = meshes.rng(7, 1000).standard_normal(g.size)
    return {"horizon": H, "seed": seed, "reward": float(r.detach()), "grad_norm": float(np.linalg.norm(g)),
            "grad_dot_probe": float(g @ d), "probe": "numpy default_rng([210205791, 7, 1000]).standard_normal(n)"}


def main():
    t0 = time.time()
    doc = {"_about": "Oracle-only references for bench.py's parity checks (tol 1e-13, sampled vertices). Written by "
                     "tests/golden/make_bench_golden.py.", "tol_rel": TOL}
    w = scenes.batched_strips(512, steps=1)
    doc["batched_strips_512"] = [first_step(w, b, 10 + b) for b in (0, 256, 511)]
    print(f"batched strips done, {time.time() - t0:.0f} s", flush=True)
    ws = scenes.batched_spring_strips(512, steps=1)
    doc["batched_spring_strips_512"] = [first_step(ws, b, 2000 + b) for b in (0, 511)]
    print(f"spring strips done, {time.time() - t0:.0f} s", flush=True)
    doc["energies"] = {}
    for model in ("stvk", "corot", "snh"):
        wm = scenes.batched_strips(512, steps=1)
        wm.model = model
        doc["energies"][model] = first_step(wm, 0, 3000)
    print(f"energies done, {time.time() - t0:.0f} s", flush=True)
    S = 5
    wf = scenes.be_strip(64, 16, steps=S)
    pf = Problem.from_workload(wf)
    states, _ = solve.rollout(pf, wf.x0, wf.v0, wf.actions, tol=TOL)
    vs = _sample(wf.n_v, 4000)
    doc["be_strip_64x16_5_steps"] = {"steps": S, "vertices": vs.tolist(), "x": states[-1][0][vs].tolist(),
                                      "norm_dx": float(np.linalg.norm(states[-1][0] - wf.x0))}
    print(f"strip rollout done, {time.time() - t0:.0f} s", flush=True)
    doc["policy_strip_64x16"] = policy_episode()
    print(f"policy episode done, {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
