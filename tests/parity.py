"""Helpers for GPU-vs-oracle parity tests (imported by the gpu-marked tests).

Tolerances (float32 GPU path against the float64 oracle fed the same float32
input state):
  velocities  relative error of the velocity state <= 1e-5 per world, where a
              free body's velocity state is its COM velocity and its angular
              velocity times its bounding radius r_b (the surface speed, so that
              every component is in m/s):
                max_b max(|dv_b|, r_b |dw_b|) <= 1e-5 * max(max_b max(|v_b|, r_b |w_b|), g h)
              with the maximum taken over the oracle's output and the input state
  positions   max|x_gpu - x_ora| <= 1e-5 * h * (same scale) + 1e-6 m
  quaternions max abs difference <= 1e-6 + h * 1e-5 * scale / r_b per body (the
              orientation change allowed by the angular-velocity tolerance)
  contact set count, geom pairs, sub-contact indices and order: bit-exact
  contact data phi, point: 1e-6 m; frame rows: 2e-5
  facet impulses <= 1e-4 * max facet impulse of the world + 1e-12
A world-step is "guarded" (excluded from the bit-exact and tolerance checks,
and counted) when some evaluated candidate has |phi - margin| < 1e-6 m or
some contact has ||n_x| - 0.5| < 1e-6: there float32 and float64 may take
different discrete decisions (contact exists, tangent-basis branch).
"""
from __future__ import annotations

import numpy as np

GUARD = 1e-6
VREL = 1e-5


def tdev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def to_np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def body_radius(scene):
    """[nw][nb] bounding radius of each body's geoms about its origin (0.05 m if none)."""
    nw, nb = scene["nworld"], scene["nbody"]
    r = np.zeros((nw, nb))
    for g in range(scene["ngeom"]):
        b = scene["geom_body"][g]
        if b < 0:
            continue
        sz = scene["geom_size"][:, g]
        t = scene["geom_type"][g]
        ext = sz[:, 0] if t == 1 else (sz[:, 0] + sz[:, 1]) if t == 2 else np.linalg.norm(sz, axis=1)
        r[:, b] = np.maximum(r[:, b], np.linalg.norm(scene["geom_pos"][:, g], axis=1) + ext)
    r[r == 0] = 0.05
    return r


def vel_state(v, radius):
    """[nb][6] -> [nb][2] per-body (|v|_inf, r |w|_inf) in m/s."""
    vb = v.reshape(-1, 6)
    return np.stack([np.abs(vb[:, :3]).max(1), radius * np.abs(vb[:, 3:]).max(1)], 1)


def _explain(w, v_gpu, vo, v_in, rad, scale, out):
    d = (v_gpu.astype(np.float64) - vo).reshape(-1, 6)
    e = np.stack([np.abs(d[:, :3]).max(1), rad * np.abs(d[:, 3:]).max(1)], 1)
    b, c = np.unravel_index(np.argmax(e), e.shape)
    part = "linear" if c == 0 else "angular*r"
    return (f"world {w}: body {b} {part} err {e[b, c]:.3e} (scale {scale:.3e}); "
            f"gpu {v_gpu.reshape(-1, 6)[b]} oracle {vo.reshape(-1, 6)[b]} in {v_in.reshape(-1, 6)[b]}; "
            f"ncon {out['ncon'][w]}")


def compare_step(scene, oracle, q_in, v_in, tau, q_gpu, v_gpu, con, worlds=None, stats=None):
    """Check one GPU step of `worlds` against the oracle run from the same float32 input.

    q_in, v_in, tau, q_gpu, v_gpu: numpy float32 [nw][..]; con: numpy contact dict of the
    GPU step (from Model.alloc_contacts) or None.  Returns a stats dict."""
    nw = q_in.shape[0]
    worlds = range(nw) if worlds is None else worlds
    stats = stats if stats is not None else dict(checked=0, guarded=0, max_vrel=0.0,
                                                 contacts=0, max_imp_rel=0.0)
    qo, vo, out = oracle.step(q_in.astype(np.float64), v_in.astype(np.float64),
                              None if tau is None else tau.astype(np.float64), worlds=list(worlds))
    h = scene["h"]
    g = float(np.linalg.norm(scene["gravity"]))
    nb = scene["nbody"]
    rad = body_radius(scene)
    for w in worlds:
        if out["guard_phi"][w] < GUARD or out["guard_frame"][w] < GUARD:
            stats["guarded"] += 1
            continue
        stats["checked"] += 1
        scale = max(vel_state(vo[w], rad[w]).max(initial=0.0),
                    vel_state(v_in[w].astype(np.float64), rad[w]).max(initial=0.0), g * h)
        vrel = vel_state(v_gpu[w].astype(np.float64) - vo[w], rad[w]).max(initial=0.0) / scale
        stats["max_vrel"] = max(stats["max_vrel"], vrel)
        assert vrel <= VREL, (f"velocity rel err {vrel:.3e} > {VREL}: "
                              + _explain(w, v_gpu[w], vo[w], v_in[w], rad[w], scale, out))
        qg = q_gpu[w].astype(np.float64).reshape(nb, 7)
        qr = qo[w].reshape(nb, 7)
        perr = np.abs(qg[:, :3] - qr[:, :3]).max(initial=0.0)
        assert perr <= VREL * h * scale + 1e-6, f"world {w}: position err {perr:.3e}"
        qerr = np.abs(qg[:, 3:] - qr[:, 3:]).max(1)
        qtol = 1e-6 + h * VREL * scale / rad[w]
        assert (qerr <= qtol).all(), f"world {w}: quaternion err {qerr.max():.3e}"
        if con is None:
            continue
        n = int(out["ncon"][w])
        assert int(con["ncon"][w]) == n, f"world {w}: ncon {con['ncon'][w]} vs {n}"
        assert int(con["overflow"][w]) == int(out["overflow"][w]), f"world {w}: overflow"
        stats["contacts"] += n
        if n == 0:
            continue
        np.testing.assert_array_equal(con["geom"][w, :n], out["geom"][w, :n], err_msg=f"world {w}")
        np.testing.assert_array_equal(con["sub"][w, :n], out["sub"][w, :n], err_msg=f"world {w}")
        np.testing.assert_allclose(con["dist"][w, :n], out["dist"][w, :n], atol=1e-6, rtol=0)
        np.testing.assert_allclose(con["pos"][w, :n], out["pos"][w, :n], atol=1e-6, rtol=0)
        np.testing.assert_allclose(con["frame"][w, :n], out["frame"][w, :n], atol=2e-5, rtol=0)
        li, lo = con["impulse"][w, :n].astype(np.float64), out["impulse"][w, :n]
        lmax = max(np.abs(lo).max(initial=0.0), 1e-300)
        irel = np.abs(li - lo).max(initial=0.0) / lmax
        stats["max_imp_rel"] = max(stats["max_imp_rel"], irel)
        assert np.abs(li - lo).max() <= 1e-4 * lmax + 1e-12, f"world {w}: impulse rel err {irel:.3e}"
    return stats
