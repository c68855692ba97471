"""CPU check of the oracle-backed policy rollout that the GPU policy test compares against: the
autograd gradient of the episode reward (policy -> oracle step -> ... -> reward) against central
finite differences of whole oracle rollouts along random parameter directions."""
import numpy as np
import torch

from oracle.fem import Problem
from synth import scenes
from tests.oracle_layers import oracle_step


def test_oracle_policy_gradient_matches_finite_differences():
    from paper_2102_05791_amd.policy import FibrePolicy, episode_reward
    w = scenes.be_strip(6, 2, steps=1)
    prob = Problem.from_workload(w)
    H = 3
    x0 = torch.from_numpy(w.x0.copy())
    v0 = torch.zeros_like(x0)
    v0[:, 0], v0[:, 1] = 0.2, -0.1
    pol = FibrePolicy(torch.from_numpy(prob.mesh.mass.copy()), 2, w.n_e, seed=7)
    r = episode_reward(prob, pol, x0, v0, H, step=oracle_step)
    r.backward()
    params = list(pol.parameters())
    grads = [p.grad.clone() for p in params]
    rng = np.random.default_rng(11)
    for _ in range(3):
        dirs = [torch.from_numpy(rng.standard_normal(p.shape)) for p in params]
        analytic = sum(float((g * d).sum()) for g, d in zip(grads, dirs))
        eps = 1e-5
        vals = []
        for sgn in (1.0, -1.0):
            with torch.no_grad():
                for p, d in zip(params, dirs):
                    p.add_(sgn * eps * d)
                vals.append(float(episode_reward(prob, pol, x0, v0, H, step=oracle_step)))
                for p, d in zip(params, dirs):
                    p.sub_(sgn * eps * d)
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - analytic) <= 1e-5 * max(abs(analytic), 1e-8), (fd, analytic)
