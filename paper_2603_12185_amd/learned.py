"""Learned per-contact impedance: training data, training and evaluation.

The network and its gradient run in the library's kernels (cf_mlp_*); the
step exports each contact's features and the training target through
cf_contacts: the log of the gain multiplier that, for the contact alone along
its normal, closes its gap within the step as far as the fallback rule's
energy margin allows (half-way to the largest accepted normal velocity).
This module only moves tensors between those calls.
"""
from __future__ import annotations

import math

import numpy as np

from . import cfsim

NIN, NH, NOUT = 8, 64, 16


def init_params(feats, seed=0):
    """Feature normalisation from the training features (mean, std of the 7
    used columns, on the host), Glorot-uniform weights, zero biases; the flat
    layout of cf_mlp_nparam()."""
    f = feats[:, :7].double()
    mean = f.mean(0).cpu().numpy()
    std = f.std(0).cpu().numpy()
    std = np.where(std > 1e-12, std, 1.0)
    rng = np.random.default_rng(seed)

    def glorot(a, b):
        r = math.sqrt(6.0 / (a + b))
        return rng.uniform(-r, r, (a, b))

    p = np.concatenate([np.r_[mean, 0.0], np.r_[std, 1.0], glorot(NIN, NH).ravel(), np.zeros(NH),
                        glorot(NH, NH).ravel(), np.zeros(NH), glorot(NH, NOUT).ravel(), np.zeros(NOUT)])
    assert p.size == int(cfsim.load().cf_mlp_nparam())
    return p.astype(np.float32)


def collect(model, q, v, steps, margin, every=1, tau=None):
    """Run `steps` plain steps from (q, v) (device tensors, updated in place)
    and gather the training rows of every contact of every `every`-th step,
    the targets for the fallback margin `margin` (m; the learned gains are
    switched off).  Returns (features [n][8], targets [n][16], q, v)."""
    import torch
    model.set_learned_impedance(None, margin=margin)
    feats, tgts = [], []
    for t in range(steps):
        con = model.alloc_contacts(training=True) if t % every == 0 else None
        q, v = model.step(q, v, tau=tau, contacts=con)
        if con is not None:
            nc = con["ncon"].long()
            keep = torch.arange(model.ncon_max, device=q.device)[None, :] < nc[:, None]
            feats.append(con["features"][keep])
            tgts.append(con["target"][keep])
    return torch.cat(feats).contiguous(), torch.cat(tgts).contiguous(), q, v


def train(feats, targets, nout, steps=400, batch=65536, lr=3e-3, seed=0):
    """Adam on minibatches drawn from the rows; returns (net, losses)."""
    import torch
    if feats.shape[0] == 0:
        raise ValueError("no training rows: the step that was sampled had no contacts "
                         "(let the scene settle into contact before collecting)")
    net = cfsim.ImpedanceNet(init_params(feats, seed))
    g = torch.Generator(device=feats.device)
    g.manual_seed(seed)
    n = feats.shape[0]
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), device=feats.device, generator=g)
        loss = net.train_step(feats[idx].contiguous(), targets[idx].contiguous(), nout, lr)
        if it % 50 == 0 or it == steps - 1:
            losses.append(float(loss.item()))
    return net, losses


def penetration_stats(model, q, v, steps, tau=None):
    """Steps from (q, v) recording every contact's gap; returns the mean and the
    maximum penetration (m) over all contacts and steps, the final state, the
    final velocities (for jitter checks) and, with the learned gains on, the
    fraction of contacts that fell back to the heuristic (else None)."""
    import torch
    tot, cnt, mx, nfb = 0.0, 0, 0.0, 0
    for _ in range(steps):
        con = {"ncon": torch.zeros(model.nworld, dtype=torch.int32, device=q.device),
               "dist": torch.zeros((model.nworld, model.ncon_max), dtype=torch.float32, device=q.device),
               "fallback": torch.zeros((model.nworld, model.ncon_max), dtype=torch.int32, device=q.device)}
        q, v = model.step(q, v, tau=tau, contacts=con)
        keep = torch.arange(model.ncon_max, device=q.device)[None, :] < con["ncon"].long()[:, None]
        pen = torch.clamp(-con["dist"][keep], min=0.0)
        tot += float(pen.sum())
        cnt += int(pen.numel())
        nfb += int(con["fallback"][keep].sum())
        if pen.numel():
            mx = max(mx, float(pen.max()))
    fb = nfb / max(cnt, 1) if getattr(model, "_net", None) is not None else None
    return tot / max(cnt, 1), mx, q, v, fb
