"""Locomotion control trained by backpropagation through time over the implicit step (Sec. 5.1).

A deterministic policy with one hidden layer of 32 ReLU units maps the current state (vertex
positions and velocities) to one actuation per element's contractile fibre (Eq. 2); an episode
runs H backward-Euler steps (Eq. 14) with ground contact and friction (Eq. 15-17); the reward is
the horizontal displacement of the body at the end of the episode, and each training iteration
takes one Adam step on the gradient of one episode (batch size 1).

Readings of the paper fixed here:
* state features: positions relative to the body's mass-weighted centre (so the policy does not
  see how far the body has already travelled) and velocities, both flattened;
* actuation range: a = 1 - 0.3 sigmoid(z) in (0.7, 1), the contraction range of the workloads;
* reward: displacement of the mass-weighted centre along x between the first and the last state.
The physics runs in the library (ImplicitStep: isb_step forward, the adjoint of Eq. 9 and
isb_vjp_params backward); the network itself is a plain PyTorch module in FP64.
"""
from __future__ import annotations

import torch

from .autograd import implicit_step


class FibrePolicy(torch.nn.Module):
    """pi_theta(x, v) -> a, one actuation per element, a in (1 - max_contraction, 1).

    mass: lumped vertex masses [n_v] (isb_get_mass), which weight the centre; dim: 2 or 3; n_e:
    actions per step, one per element (plus one per spring when the body has springs, whose
    actions follow the elements'). Weights start uniform in +-1/sqrt(fan_in) from a seeded generator, so
    two policies built with the same arguments are identical (on any device)."""

    def __init__(self, mass, dim: int, n_e: int, hidden: int = 32, max_contraction: float = 0.3, seed: int = 0):
        super().__init__()
        self.register_buffer("w", (mass / mass.sum()).detach().to(torch.float64))
        self.max_contraction = max_contraction
        n_in = 2 * mass.numel() * dim
        self.l1 = torch.nn.Linear(n_in, hidden, dtype=torch.float64, device=mass.device)
        self.l2 = torch.nn.Linear(hidden, n_e, dtype=torch.float64, device=mass.device)
        g = torch.Generator().manual_seed(seed)
        with torch.no_grad():
            for lin in (self.l1, self.l2):
                bound = 1.0 / lin.in_features ** 0.5
                for t in (lin.weight, lin.bias):
                    t.copy_(torch.rand(t.shape, dtype=torch.float64, generator=g) * (2 * bound) - bound)

    def features(self, x, v):
        com = (self.w[:, None] * x).sum(0)
        return torch.cat([(x - com).reshape(-1), v.reshape(-1)])

    def forward(self, x, v):
        z = self.l2(torch.relu(self.l1(self.features(x, v))))
        return (1.0 - self.max_contraction * torch.sigmoid(z)).contiguous()


def centre_x(weights, x):
    """Centre of the body along x with normalised vertex weights (mass / total mass)."""
    return (weights * x[:, 0]).sum()


def episode_reward(ctx, policy: FibrePolicy, x0, v0, horizon: int, step=implicit_step):
    """Horizontal displacement of the centre after `horizon` steps under the policy (differentiable
    in the policy's parameters, and in x0 and v0)."""
    x, v = x0, v0
    for _ in range(horizon):
        a = policy(x, v)
        x, v = step(ctx, x, v, a)
    return centre_x(policy.w, x) - centre_x(policy.w, x0)


def train_locomotion(ctx, policy: FibrePolicy, x0, v0, horizon: int, iterations: int, lr: float = 1e-3,
                     step=implicit_step, callback=None):
    """One Adam step per episode; returns the reward of every episode (before its update)."""
    opt = torch.optim.Adam(policy.parameters(), lr=lr)
    rewards = []
    for it in range(iterations):
        opt.zero_grad()
        r = episode_reward(ctx, policy, x0, v0, horizon, step)
        (-r).backward()
        opt.step()
        rewards.append(float(r.detach()))
        if callback is not None:
            callback(it, rewards[-1])
    return rewards
