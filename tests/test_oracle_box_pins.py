"""Pins of the oracle's box-sphere and box-capsule contacts and of position
actuators, against results obtained another way.

Box contacts (the narrow phase that feeds Eq. cf_wrench): the gap of a sphere
outside a box is checked against a bounded minimisation of the centre-to-box
distance (scipy), inside against a brute-force scan over the six face planes;
invariance under a rigid motion of the whole scene; a capsule is checked
against two spheres at its end centres; a sphere resting on a static box top
follows the same trajectory as on a plane at that height.

Actuators (the applied force tau of Eq. smooth_vel in the hand of the paper's
application section): one step of an actuated slide dof against the hand
derivation of the discrete update, and the static balance of an actuated
pendulum against the textbook gravity torque.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle.cfo import Oracle, OracleError
from paper_2603_12185_amd import scenes

# float32-representable sizes: the scene stores sizes in float32
HALF = np.array([0.05, 0.04, 0.03], np.float32).astype(float)
R_SPH = float(np.float32(0.02))


def _rot(q):
    q = np.asarray(q, float) / np.linalg.norm(q)
    return scenes._quat_to_mat(q)


def _box_sphere_scene(box_first=True, capsule=False, margin=0.2):
    b = scenes._Builder(1)
    bx = b.body(scenes.JNT_FREE, mass=1.0, inertia=(1e-3,) * 3)
    ob = b.body(scenes.JNT_FREE, mass=0.5, inertia=(1e-4,) * 3)
    gshape = (scenes.CAPSULE, (R_SPH, 0.03, 0)) if capsule else (scenes.SPHERE, (R_SPH, 0, 0))
    if box_first:
        b.geom(scenes.BOX, bx, size=tuple(HALF), friction=(0.5, 0, 0))
        b.geom(gshape[0], ob, size=gshape[1], friction=(0.5, 0, 0))
    else:
        b.geom(gshape[0], ob, size=gshape[1], friction=(0.5, 0, 0))
        b.geom(scenes.BOX, bx, size=tuple(HALF), friction=(0.5, 0, 0))
    return b.build(gravity=(0, 0, 0), margin=margin, ncon_max=8)


def _place(s, box_pos, box_quat, local):
    """Box at (box_pos, box_quat), other body at the box-frame point `local`."""
    R = _rot(box_quat)
    q = s["q0"].astype(float).copy()
    q[0, 0:3] = box_pos
    q[0, 3:7] = np.asarray(box_quat) / np.linalg.norm(box_quat)
    q[0, 7:10] = np.asarray(box_pos) + R @ np.asarray(local)
    q[0, 10:14] = (1, 0, 0, 0)
    return q


def _dist_outside(local):
    """Distance from a box-frame point to the box by bounded minimisation."""
    res = minimize(lambda x: np.sum((x - local) ** 2), np.zeros(3), jac=lambda x: 2 * (x - local),
                   bounds=[(-h, h) for h in HALF], method="L-BFGS-B",
                   options=dict(ftol=1e-300, gtol=1e-14, maxiter=1000))
    return math.sqrt(res.fun), res.x


def _depth_inside(local):
    """Penetration depth of an interior point: distance to the nearest face plane,
    scanned over the six faces, and that face's outward normal (box frame)."""
    best = (np.inf, None)
    for k in range(3):
        for sgn in (1.0, -1.0):
            d = HALF[k] - sgn * local[k]
            if d < best[0] - 1e-15:
                nl = np.zeros(3)
                nl[k] = sgn
                best = (d, nl)
    return best


LOCALS_OUT = [(0.01, -0.012, HALF[2] + 0.015),          # above the +z face
              (-HALF[0] - 0.01, 0.005, -0.02),          # beside the -x face
              (HALF[0] + 0.008, 0.01, HALF[2] + 0.011),  # +x +z edge region
              (-HALF[0] - 0.006, HALF[1] + 0.007, -HALF[2] - 0.009)]  # corner region
LOCALS_IN = [(0.01, -0.005, 0.02), (0.0, 0.002, -0.025), (-0.045, 0.0, 0.0), (0.001, 0.037, 0.0)]


@pytest.mark.parametrize("box_first", [True, False])
def test_box_sphere_gap_normal_point(box_first):
    s = _box_sphere_scene(box_first)
    o = Oracle(s)
    bq = (0.9, 0.2, -0.3, 0.25)
    R = _rot(bq)
    bp = np.array([0.1, -0.2, 0.3])
    for local in LOCALS_OUT + LOCALS_IN:
        local = np.array(local, float)
        q = _place(s, bp, bq, local)
        _, _, out = o.step(q, s["v0"])
        assert out["ncon"][0] == 1
        g = out["geom"][0, 0]
        assert s["geom_type"][g[0]] == scenes.BOX and s["geom_type"][g[1]] == scenes.SPHERE
        outside = np.any(np.abs(local) > HALF)
        if outside:
            d, x = _dist_outside(local)
            phi = d - R_SPH
            nl = (local - x) / d
        else:
            depth, nl = _depth_inside(local)
            phi = -depth - R_SPH
        c = bp + R @ local
        n = R @ nl
        np.testing.assert_allclose(out["dist"][0, 0], phi, atol=1e-10)
        np.testing.assert_allclose(out["frame"][0, 0, :3], n, atol=1e-8)
        np.testing.assert_allclose(out["pos"][0, 0], c - n * (R_SPH + 0.5 * phi), atol=1e-9)


def test_box_sphere_rigid_motion_invariance():
    s = _box_sphere_scene()
    o = Oracle(s)
    rng = np.random.default_rng(3)
    for local in LOCALS_OUT + LOCALS_IN:
        base = None
        for _ in range(3):
            bq = rng.normal(size=4)
            bp = rng.normal(size=3)
            _, _, out = o.step(_place(s, bp, bq, np.array(local, float)), s["v0"])
            R = _rot(bq)
            nl = R.T @ out["frame"][0, 0, :3]
            cur = (out["dist"][0, 0], nl)
            if base is None:
                base = cur
            else:
                np.testing.assert_allclose(cur[0], base[0], atol=1e-13)
                np.testing.assert_allclose(cur[1], base[1], atol=1e-12)


def test_box_capsule_is_two_end_spheres():
    cap = _box_sphere_scene(capsule=True)
    # reference: two spheres of the capsule's radius at its end centres
    b = scenes._Builder(1)
    bx = b.body(scenes.JNT_FREE, mass=1.0, inertia=(1e-3,) * 3)
    b.geom(scenes.BOX, bx, size=tuple(HALF), friction=(0.5, 0, 0))
    ends = [b.body(scenes.JNT_FREE, mass=0.5, inertia=(1e-4,) * 3) for _ in range(2)]
    for e in ends:
        b.geom(scenes.SPHERE, e, size=(R_SPH, 0, 0), friction=(0.5, 0, 0))
    two = b.build(gravity=(0, 0, 0), margin=0.2, ncon_max=8)
    bq = np.array([0.8, -0.1, 0.4, 0.3])
    bq /= np.linalg.norm(bq)
    cq = np.array([0.7, 0.5, 0.2, -0.4])
    cq /= np.linalg.norm(cq)
    axis = _rot(cq)[:, 2]
    for local in ((0.0, 0.0, HALF[2] + 0.03), (0.02, -0.01, 0.01), (HALF[0] + 0.01, 0.0, 0.0)):
        q = _place(cap, (0.0, 0.1, 0.2), bq, np.array(local, float))
        q[0, 10:14] = cq
        _, _, a = Oracle(cap).step(q, cap["v0"])
        c = q[0, 7:10]
        q2 = np.zeros((1, 21))
        q2[0, :7] = q[0, :7]
        q2[0, 7:10] = c - 0.03 * axis
        q2[0, 10:14] = cq
        q2[0, 14:17] = c + 0.03 * axis
        q2[0, 17:21] = cq
        _, _, r = Oracle(two).step(q2, np.zeros((1, 18)))
        # the reference's box contacts (its two spheres also meet each other)
        keep = [k for k in range(r["ncon"][0]) if r["geom"][0, k, 0] == 0]
        assert a["ncon"][0] == len(keep) == 2
        assert list(a["sub"][0, :2]) == [0, 1]
        np.testing.assert_allclose(a["dist"][0, :2], r["dist"][0, keep], atol=1e-13)
        np.testing.assert_allclose(a["frame"][0, :2], r["frame"][0, keep], atol=1e-12)
        np.testing.assert_allclose(a["pos"][0, :2], r["pos"][0, keep], atol=1e-13)


def test_sphere_on_static_box_top_matches_plane():
    """A sphere dropped onto the top face of a static box moves exactly as on a
    plane at the face height (same contact frame, gap and impulses)."""
    top = 0.1
    b = scenes._Builder(1)
    b.geom(scenes.BOX, -1, size=(0.5, 0.5, top / 2), pos=(0, 0, top / 2), friction=(0.6, 0, 0))
    bi = b.body(scenes.JNT_FREE, mass=1.0, inertia=(4e-4,) * 3)
    b.geom(scenes.SPHERE, bi, size=(0.05, 0, 0), friction=(0.6, 0, 0))
    box = b.build(condim=6)
    b = scenes._Builder(1)
    b.geom(scenes.PLANE, -1, pos=(0, 0, top), friction=(0.6, 0, 0))
    bi = b.body(scenes.JNT_FREE, mass=1.0, inertia=(4e-4,) * 3)
    b.geom(scenes.SPHERE, bi, size=(0.05, 0, 0), friction=(0.6, 0, 0))
    pln = b.build(condim=6)
    q = np.array([[0.01, -0.02, top + 0.06, 1, 0, 0, 0]], float)
    v = np.array([[0.3, -0.1, -0.5, 2.0, 1.0, -3.0]], float)
    qa, va, qb, vb = q.copy(), v.copy(), q.copy(), v.copy()
    oa, ob = Oracle(box), Oracle(pln)
    touched = 0
    for _ in range(150):
        qa, va, a = oa.step(qa, va)
        qb, vb, r = ob.step(qb, vb)
        assert a["ncon"][0] == r["ncon"][0]
        touched += int(a["ncon"][0])
        np.testing.assert_allclose(qa, qb, atol=1e-12)
        np.testing.assert_allclose(va, vb, atol=1e-10)
    assert touched > 50


def test_actuated_slide_one_step():
    """Slide dof of mass m, no gravity or contact: v+ = v + h (kp (u - x) - kd v) / m,
    x+ = x + h v+ (the discrete update written out by hand)."""
    b = scenes._Builder(1)
    b.body(scenes.JNT_SLIDE, -1, axis=(1, 0, 0), mass=2.0, inertia=(1e-3,) * 3)
    s = b.build(gravity=(0, 0, 0))
    s["dof_kp"], s["dof_kd"] = np.array([30.0]), np.array([0.7])
    o = Oracle(s)
    x, v, u, h = 0.12, -0.4, 0.5, s["h"]
    q1, v1, _ = o.step(np.array([[x]]), np.array([[v]]), tau=np.array([[u]]))
    vp = v + h * (30.0 * (u - x) - 0.7 * v) / 2.0
    np.testing.assert_allclose(v1[0, 0], vp, rtol=1e-14)
    np.testing.assert_allclose(q1[0, 0], x + h * vp, rtol=1e-14)
    # an unactuated scene takes the same input as a force
    del s["dof_kp"], s["dof_kd"]
    _, v2, _ = Oracle(s).step(np.array([[x]]), np.array([[v]]), tau=np.array([[u]]))
    np.testing.assert_allclose(v2[0, 0], v + h * u / 2.0, rtol=1e-14)


def test_actuated_pendulum_static_balance():
    """Pendulum (hinge about y, bob at distance L): the actuator holds theta* when
    kp (u - theta*) equals the gravity torque m g L sin(theta*)."""
    L, m, kp, th = float(np.float32(0.5)), 1.0, 40.0, 0.3
    s = scenes.pendulum(length=L, mass=m)
    s["dof_kp"], s["dof_kd"] = np.array([kp]), np.array([0.5])
    g = -float(s["gravity"][2])  # float32 value the scene holds
    u = th + m * g * L * math.sin(th) / kp
    q1, v1, _ = Oracle(s).step(np.array([[th]]), np.array([[0.0]]), tau=np.array([[u]]))
    assert abs(v1[0, 0]) < 1e-12 and abs(q1[0, 0] - th) < 1e-14
    # off balance the bob accelerates toward the balance angle
    _, v2, _ = Oracle(s).step(np.array([[th + 0.05]]), np.array([[0.0]]), tau=np.array([[u]]))
    assert v2[0, 0] < 0


def test_actuators_on_free_dofs_rejected():
    s = scenes.sphere_on_plane()
    s["dof_kp"] = np.ones(6)
    with pytest.raises(OracleError):
        Oracle(s)
