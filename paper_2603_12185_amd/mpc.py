"""Sampling-based model-predictive control of the hand (the application of the
paper's Sec. V): model-predictive path integral (MPPI) control with batched
rollouts of the library's step.

Every iteration draws N noisy control sequences around the nominal one, runs
them as N worlds for H steps with one cf_rollout call (the persistent
kernel), scores each trajectory, and moves the nominal sequence by the
cost-weighted average of the noise.  The rollouts run in the library's
kernels; sampling, costs and the weighted average are a few tensor operations
on the same stream.
"""
from __future__ import annotations

import math

import numpy as np

from . import cfsim, scenes


def quat_yaw(q):
    """Yaw angle of (w, x, y, z) quaternions (rotation about z of the body x axis)."""
    import torch
    w, x, y, z = q.unbind(-1)
    return torch.atan2(2 * (w * z + x * y), 1 - 2 * (y * y + z * z))


class HandMPPI:
    """MPPI on the hand-and-cube scene: turn the cube to `target_yaw` about the
    vertical while keeping it at its start position.

    nroll rollouts of horizon H; Gaussian noise of standard deviation sigma
    (rad) on the 16 finger targets; temperature lam; targets clipped to
    +-clip around the rest pose.  autotune: let the library pick the rollout's
    launch shape for this scene first."""

    def __init__(self, nroll=2048, H=20, sigma=0.1, lam=0.01, clip=0.6, target_yaw=0.5, seed=0,
                 scene_kw=None, autotune=True):
        import torch
        kw = dict(scene_kw or {})
        self.scene = scenes.hand_cube(nworld=nroll, seed=seed, **kw)
        self.plant_scene = scenes.select_worlds(self.scene, [0])
        self.model = cfsim.Model(self.scene)
        self.plant = cfsim.Model(self.plant_scene)
        self.nroll, self.H, self.sigma, self.lam, self.clip = nroll, H, sigma, lam, clip
        self.nv, self.nq = self.model.nv, self.model.nq
        dev = torch.device("cuda")
        self.dev = dev
        self.rest = torch.tensor(np.tile(scenes.HAND_Q0, 4), dtype=torch.float32, device=dev)
        self.U = self.rest.repeat(H, 1).contiguous()                 # nominal [H][16]
        self.q = torch.from_numpy(self.plant_scene["q0"]).to(dev)     # plant state [1][nq]
        self.v = torch.from_numpy(self.plant_scene["v0"]).to(dev)
        self.p0 = self.q[0, 0:3].clone()
        self.target_yaw = target_yaw
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        self.tau_seq = torch.zeros((H, nroll, self.nv), dtype=torch.float32, device=dev)
        self.q_traj = torch.empty((H + 1, nroll, self.nq), dtype=torch.float32, device=dev)
        self.v_traj = torch.empty((H + 1, nroll, self.nv), dtype=torch.float32, device=dev)
        self.q0s = torch.empty((nroll, self.nq), dtype=torch.float32, device=dev)
        self.v0s = torch.empty((nroll, self.nv), dtype=torch.float32, device=dev)
        if autotune:
            # workgroup size and persistent kernel vs step launches for this scene
            self.q0s.copy_(self.q.expand(nroll, -1))
            self.v0s.copy_(self.v.expand(nroll, -1))
            self.model.autotune(self.q0s, self.v0s, steps=H)

    def costs(self, q_traj):
        """Per-rollout cost of the trajectories [H+1][N][nq]: squared yaw error
        and squared displacement of the cube, summed over the horizon."""
        cube = q_traj[1:, :, 0:7]
        yaw = quat_yaw(cube[..., 3:7])
        err = torch_wrap(yaw - self.target_yaw)
        pos = ((cube[..., 0:3] - self.p0) ** 2).sum(-1)
        return (err * err + 100.0 * pos).sum(0)

    def sample(self):
        import torch
        eps = torch.randn((self.nroll, self.H, 16), generator=self.gen, device=self.dev) * self.sigma
        u = torch.clamp(self.U[None] + eps, self.rest - self.clip, self.rest + self.clip)
        return u, u - self.U[None]

    def rollouts(self, u):
        """Run the sampled control sequences u [N][H][16] from the plant state."""
        self.tau_seq[:, :, 6:] = u.transpose(0, 1)
        self.q0s.copy_(self.q.expand(self.nroll, -1))
        self.v0s.copy_(self.v.expand(self.nroll, -1))
        self.model.rollout(self.H, self.q0s, self.v0s, tau_seq=self.tau_seq, q_traj=self.q_traj,
                           v_traj=self.v_traj)
        return self.q_traj

    def update(self, u, eps, cost):
        import torch
        w = torch.softmax(-(cost - cost.min()) / self.lam, 0)
        self.U = (self.U + (w[:, None, None] * eps).sum(0)).contiguous()
        return w

    def iterate(self):
        """One MPC iteration: sample, roll out, weight, update, apply the first
        control to the plant for one step and shift the nominal sequence.
        Returns the cost of the mean rollout estimate (weighted cost)."""
        import torch
        u, eps = self.sample()
        q_traj = self.rollouts(u)
        cost = self.costs(q_traj)
        w = self.update(u, eps, cost)
        tau = torch.zeros((1, self.nv), dtype=torch.float32, device=self.dev)
        tau[0, 6:] = self.U[0]
        self.q, self.v = self.plant.step(self.q, self.v, tau=tau)
        self.U = torch.cat([self.U[1:], self.U[-1:]], 0).contiguous()
        return float((w * cost).sum())

    def cube_yaw(self):
        return float(quat_yaw(self.q[0, 3:7]))


def torch_wrap(a):
    """Angles wrapped to (-pi, pi]."""
    import torch
    return torch.remainder(a + math.pi, 2 * math.pi) - math.pi
