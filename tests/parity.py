"""Helpers for GPU-vs-oracle parity tests (imported by the gpu-marked tests).

Tolerances (float32 GPU path against the float64 oracle fed the same float32
input state):
  velocities  relative error of the velocity state <= 1e-5 per world, where each
              component is turned into a speed (m/s): free-joint linear and
              slide rates as they are, free-joint angular velocities times the
              body's bounding radius r_b, hinge rates times r_b + |COM offset|:
                max_i L_i |dv_i| <= 1e-5 * max(max_i L_i |v_i|, g h)
              with the maximum taken over the oracle's output and the input state
  positions   free-body positions <= 1e-5 * h * (same scale) + 1e-6 m; joint
              positions and quaternions <= 1e-6 + h * 1e-5 * scale / L (the change
              allowed by the velocity tolerance)
  contact set count, geom pairs, sub-contact indices and order: bit-exact
  contact data phi, point: 1e-6 m; frame rows: 2e-5
  facet impulses <= 1e-4 * max facet impulse of the world + A_f (k h + d) 1e-5 * scale
              + 1e-12, A_f the facet's impulse gain (lambda_f h = A_f max(arg_f, 0)):
              the second term is the impulse a velocity error within the velocity
              tolerance makes on that facet
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


def dof_lengths(scene):
    """[nw][nv] length that turns each velocity component into a speed: 1 for
    free-joint linear and slide dofs, the body's bounding radius for free-joint
    angular dofs, and bounding radius + |COM offset| for hinges."""
    from paper_2603_12185_amd import scenes
    rad = body_radius(scene)
    nw = scene["nworld"]
    cols = []
    for b, jt in enumerate(scene["body_jnt"]):
        if jt == scenes.JNT_FREE:
            cols += [np.ones(nw)] * 3 + [rad[:, b]] * 3
        elif jt == scenes.JNT_HINGE:
            cols.append(rad[:, b] + np.linalg.norm(scene["body_ipos"][b]))
        else:
            cols.append(np.ones(nw))
    return np.stack(cols, 1) if cols else np.zeros((nw, 0))


def vel_state(v, lengths):
    """Velocity components as speeds (m/s)."""
    return np.abs(v) * lengths


def _explain(w, v_gpu, vo, v_in, lengths, scale, out):
    e = vel_state(v_gpu.astype(np.float64) - vo, lengths)
    i = int(np.argmax(e))
    return (f"world {w}: dof {i} err {e[i]:.3e} (scale {scale:.3e}); "
            f"gpu {v_gpu[i]} oracle {vo[i]} in {v_in[i]}; ncon {out['ncon'][w]}")


def compare_step(scene, oracle, q_in, v_in, tau, q_gpu, v_gpu, con, worlds=None, stats=None,
                 learned=None, vtol_extra=None, imp_tol_extra=None):
    """Check one GPU step of `worlds` against the oracle run from the same float32 input.

    q_in, v_in, tau, q_gpu, v_gpu: numpy float32 [nw][..]; con: numpy contact dict of the
    GPU step (from Model.alloc_contacts) or None.  learned = (params, margin): the
    oracle takes the learned-gain step of that network (and, where `con` holds
    the GPU's fallback decisions, they must equal the oracle's).  vtol_extra [nw]
    (m/s) and imp_tol_extra [nw][ncon_max][nfacet] widen the velocity and impulse
    tolerances by error bounds the caller derives (a bf16 network's).  Returns a
    stats dict."""
    nw = q_in.shape[0]
    worlds = range(nw) if worlds is None else worlds
    stats = stats if stats is not None else dict(checked=0, guarded=0, max_vrel=0.0,
                                                 contacts=0, max_imp_rel=0.0)
    qo, vo, out = oracle.step(q_in.astype(np.float64), v_in.astype(np.float64),
                              None if tau is None else tau.astype(np.float64), worlds=list(worlds),
                              learned=learned)
    from paper_2603_12185_amd import scenes
    h = scene["h"]
    g = float(np.linalg.norm(scene["gravity"]))
    rad = body_radius(scene)
    lens = dof_lengths(scene)
    qa, da = scenes.qadr(scene), scenes.dadr(scene)
    for w in worlds:
        if out["guard_phi"][w] < GUARD or out["guard_frame"][w] < GUARD:
            stats["guarded"] += 1
            continue
        stats["checked"] += 1
        scale = max(vel_state(vo[w], lens[w]).max(initial=0.0),
                    vel_state(v_in[w].astype(np.float64), lens[w]).max(initial=0.0), g * h)
        vrel = vel_state(v_gpu[w].astype(np.float64) - vo[w], lens[w]).max(initial=0.0) / scale
        stats["max_vrel"] = max(stats["max_vrel"], vrel)
        vlim = VREL + (0.0 if vtol_extra is None else vtol_extra[w] / scale)
        assert vrel <= vlim, (f"velocity rel err {vrel:.3e} > {vlim:.3e}: "
                              + _explain(w, v_gpu[w], vo[w], v_in[w], lens[w], scale, out))
        qg, qr = q_gpu[w].astype(np.float64), qo[w]
        for b, jt in enumerate(scene["body_jnt"]):
            a0, d0 = qa[b], da[b]
            if jt == scenes.JNT_FREE:
                perr = np.abs(qg[a0:a0 + 3] - qr[a0:a0 + 3]).max()
                assert perr <= vlim * h * scale + 1e-6, f"world {w} body {b}: position err {perr:.3e}"
                qerr = np.abs(qg[a0 + 3:a0 + 7] - qr[a0 + 3:a0 + 7]).max()
                assert qerr <= 1e-6 + h * vlim * scale / rad[w, b], \
                    f"world {w} body {b}: quaternion err {qerr:.3e}"
            else:
                jerr = abs(qg[a0] - qr[a0])
                assert jerr <= 1e-6 + h * vlim * scale / lens[w, d0], \
                    f"world {w} body {b}: joint position err {jerr:.3e}"
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
        # a facet's impulse is A_f max(arg_f, 0) with arg_f = -(k h + d) s_f - k phi:
        # besides 1e-4 of the world's largest impulse, allow the impulse that a
        # velocity error within the velocity tolerance would make on that facet
        # (arg_f can be a small difference of large terms on a sliding contact)
        aa = scene["k_user"] * h + scene["d_user"]
        tol = 1e-4 * lmax + out["facet_gain"][w, :n] * aa * vlim * scale + 1e-12
        if imp_tol_extra is not None:
            tol = tol + imp_tol_extra[w, :n]
        if learned is not None and "fallback" in con:
            np.testing.assert_array_equal(con["fallback"][w, :n], out["fallback"][w, :n],
                                          err_msg=f"world {w}: fallback decisions")
        if (np.abs(li - lo) > tol).any():
            k, f = np.unravel_index(int(np.argmax(np.abs(li - lo))), li.shape)
            raise AssertionError(f"world {w}: impulse rel err {irel:.3e} at contact {k} facet {f}: gpu "
                                 f"{li[k, f]:.9e} oracle {lo[k, f]:.9e} (largest {lmax:.3e}); contact "
                                 f"geoms {out['geom'][w, k].tolist()} phi {out['dist'][w, k]:.3e} "
                                 f"gpu facets {li[k].tolist()} oracle facets {lo[k].tolist()}")
    return stats
