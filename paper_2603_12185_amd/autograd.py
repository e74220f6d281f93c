"""torch.autograd bindings of the step and of rollouts.

`step(model, q, v, tau)` and `rollout(model, T, q0, v0, tau_seq)` return
tensors that carry gradients back through the library's hand-written adjoint
(`cf_step_backward`).  A rollout keeps every step's state (the trajectory it
returns anyway) as its checkpoint; its backward walks the steps in reverse,
each call recomputing its step's forward pass on the GPU from the stored
(q_t, v_t, tau_t).  Gradients are those of the piecewise-smooth step on the
piece that contains the forward trajectory (contact sets and facet activity
held fixed).  Only argument marshalling happens here; all arithmetic runs in
the HIP library.
"""
from __future__ import annotations

import torch


class _Step(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, q, v, tau):
        q, v = q.contiguous(), v.contiguous()
        tau = None if tau is None else tau.contiguous()
        q1, v1 = model.step(q, v, tau)
        ctx.model = model
        ctx.has_tau = tau is not None
        ctx.save_for_backward(q, v, tau if tau is not None else q.new_empty(0))
        return q1, v1

    @staticmethod
    def backward(ctx, gq1, gv1):
        q, v, tau = ctx.saved_tensors
        tau = tau if ctx.has_tau else None
        gq1 = None if gq1 is None else gq1.contiguous()
        gv1 = None if gv1 is None else gv1.contiguous()
        gq, gv, gtau = ctx.model.step_backward(q, v, tau, gq1, gv1)
        return None, gq, gv, (gtau if ctx.has_tau else None)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, T, q0, v0, tau_seq):
        q0, v0 = q0.contiguous(), v0.contiguous()
        tau_seq = None if tau_seq is None else tau_seq.contiguous()
        q_traj, v_traj = model.rollout(T, q0, v0, tau_seq)
        ctx.model, ctx.T = model, T
        ctx.has_tau = tau_seq is not None
        ctx.save_for_backward(q_traj, v_traj, tau_seq if tau_seq is not None else q0.new_empty(0))
        return q_traj, v_traj

    @staticmethod
    def backward(ctx, gq_traj, gv_traj):
        q_traj, v_traj, tau_seq = ctx.saved_tensors
        model, T = ctx.model, ctx.T
        nw = model.nworld
        if gq_traj is None:
            gq_traj = torch.zeros_like(q_traj)
        if gv_traj is None:
            gv_traj = torch.zeros_like(v_traj)
        gq = gq_traj[T].clone()
        gv = gv_traj[T].clone()
        gtau_seq = torch.empty((T, nw, model.nv), dtype=torch.float32, device=q_traj.device) \
            if ctx.has_tau else None
        gq_t, gv_t = torch.empty_like(gq), torch.empty_like(gv)
        scratch_tau = torch.empty_like(gv)
        for t in range(T - 1, -1, -1):
            tau_t = tau_seq[t] if ctx.has_tau else None
            gtau_t = gtau_seq[t] if ctx.has_tau else scratch_tau
            model.step_backward(q_traj[t], v_traj[t], tau_t, gq, gv, gq=gq_t, gv=gv_t, gtau=gtau_t)
            gq = gq_t + gq_traj[t]
            gv = gv_t + gv_traj[t]
        return None, None, gq, gv, gtau_seq


def step(model, q, v, tau=None):
    """(q+, v+) of one step, differentiable in q, v and tau."""
    return _Step.apply(model, q, v, tau)


def rollout(model, T, q0, v0, tau_seq=None):
    """Trajectories [T+1][nworld][nq], [T+1][nworld][nv], differentiable in q0,
    v0 and tau_seq [T][nworld][nv]."""
    return _Rollout.apply(model, int(T), q0, v0, tau_seq)
