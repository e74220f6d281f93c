"""Central differences of the FP64 oracle for the adjoint tests.

The oracle steps in float64; a vector-Jacobian product of the step is checked
against central differences of L = <gq_out, q+> + <gv_out, v+> (or of a
rollout cost), evaluated with every perturbation as a world of its own in one
oracle call.  The step is piecewise smooth, so a component whose stencil
crosses a branch (contact set, facet activity, the impedance clamp, the
tangent helper) is reported and left out of the comparison.
"""
from __future__ import annotations

import numpy as np

from oracle.cfo import Oracle
from paper_2603_12185_amd import scenes


def branch_key(out, w, width):
    """Everything discrete the oracle's step decided for world w (with learned
    gains also each contact's fallback decision and which outputs are clamped)."""
    n = int(out["ncon"][w])
    key = (n, out["geom"][w, :n].tobytes(), out["sub"][w, :n].tobytes(),
           (out["impulse"][w, :n] > 0).tobytes(),
           (np.abs(out["dist"][w, :n]) >= width).tobytes(),
           (np.abs(out["frame"][w, :n, 0]) <= 0.5).tobytes())
    if "learned_y" in out:
        nf = out["impulse"].shape[-1]
        key += (out["fallback"][w, :n].tobytes(),
                (np.abs(out["learned_y"][w, :n, :nf]) >= np.log(256.0)).tobytes())
    return key


def step_grad_fd(scene, w, q, v, tau, gq_out, gv_out, eps=1e-6, learned=None):
    """FD gradient of <gq_out[w], q+> + <gv_out[w], v+> of world w with respect to
    (q[w], v[w], tau[w]) in float64 (the oracle's learned-gain step when
    learned = (params, margin)).  Returns (g, ok): g = concatenated
    (dq, dv, dtau), ok = stencil stayed on the base point's branch."""
    nq, nv = q.shape[-1], v.shape[-1]
    n_in = nq + 2 * nv
    m = 2 * n_in + 1
    o = Oracle(scenes.select_worlds(scene, [w] * m))
    t = np.zeros(nv) if tau is None else np.asarray(tau[w], np.float64)
    x0 = np.concatenate([np.asarray(q[w], np.float64), np.asarray(v[w], np.float64), t])
    X = np.tile(x0, (m, 1))
    idx = np.arange(n_in)
    X[1 + 2 * idx, idx] += eps
    X[2 + 2 * idx, idx] -= eps
    qo, vo, out = o.step(X[:, :nq], X[:, nq:nq + nv], X[:, nq + nv:], learned=learned)
    L = qo @ np.asarray(gq_out[w], np.float64) + vo @ np.asarray(gv_out[w], np.float64)
    g = (L[1::2] - L[2::2]) / (2 * eps)
    width = float(scene["solimp"][2])
    k0 = branch_key(out, 0, width)
    ok = np.array([branch_key(out, 1 + 2 * i, width) == k0 and branch_key(out, 2 + 2 * i, width) == k0
                   for i in range(n_in)])
    return g, ok, out


def rollout_cost_fd(scene, worlds, q0, v0, tau_seq, cost, comps, eps=1e-6, learned=None):
    """FD gradient of cost(w, q_T, v_T) (world w's cost of each row, float64) with respect to the
    components `comps` (list of (t, dof)) of tau_seq [T][nw][nv], for each world
    in `worlds`.  Returns (g [len(worlds)][len(comps)], ok) with ok marking
    stencils whose every step stayed on the base trajectory's branches."""
    T = tau_seq.shape[0]
    nc = len(comps)
    m = 2 * nc + 1
    width = float(scene["solimp"][2])
    g = np.zeros((len(worlds), nc))
    ok = np.zeros((len(worlds), nc), bool)
    for wi, w in enumerate(worlds):
        o = Oracle(scenes.select_worlds(scene, [w] * m))
        q = np.tile(np.asarray(q0[w], np.float64), (m, 1))
        v = np.tile(np.asarray(v0[w], np.float64), (m, 1))
        tau = np.tile(np.asarray(tau_seq[:, w], np.float64)[:, None, :], (1, m, 1))
        for i, (t, d) in enumerate(comps):
            tau[t, 1 + 2 * i, d] += eps
            tau[t, 2 + 2 * i, d] -= eps
        same = np.ones(nc, bool)
        for t in range(T):
            q, v, out = o.step(q, v, tau[t], learned=learned)
            k0 = branch_key(out, 0, width)
            for i in range(nc):
                if same[i] and (branch_key(out, 1 + 2 * i, width) != k0 or
                                branch_key(out, 2 + 2 * i, width) != k0):
                    same[i] = False
        c = cost(w, q, v)
        g[wi] = (c[1::2] - c[2::2]) / (2 * eps)
        ok[wi] = same
    return g, ok
