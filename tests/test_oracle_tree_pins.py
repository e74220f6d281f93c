"""Pins of the oracle's articulated dynamics for trees whose root is a free
joint (a floating base with hinge and slide descendants), Sec. III.A, the mass
matrix M(q) and bias c(q, v) of the system dynamics.

Nothing here uses the oracle's Jacobian or bias formulas.  The test carries its
own forward kinematics, written from the model conventions of the C ABI (body
frame in its parent frame at q = 0, hinge and slide axes in the body frame,
free joint q = (origin, quaternion), v = (origin velocity, world angular
velocity)).  From it:

* the Jacobians, by central differences of body COM positions and rotations;
* M, from the kinetic energy sum_b 1/2 (m |v_c|^2 + w^T I_w w) over those
  Jacobians, and the composite-rigid-body closed forms of the free root's 6x6
  block (total mass, first moment about the root origin, composite inertia);
* c, from Lagrange's equations in a chart xi = (x, phi, joints) with the root
  orientation exp([phi]x) R0.  At phi = 0 the chart velocities equal the
  quasi-velocities v and the chart's Coriolis terms equal the oracle's, since
  the left Jacobian of SO(3) is I + [phi]x / 2 + O(|phi|^2) and w x w = 0.
"""
import math

import numpy as np
import pytest

from oracle.cfo import Oracle
from paper_2603_12185_amd import scenes


def _quat_mat(qt):
    w, x, y, z = np.asarray(qt, float) / np.linalg.norm(qt)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _skew(a):
    return np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])


def _expm_so3(phi):
    th = np.linalg.norm(phi)
    K = _skew(phi)
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


def _fk(s, root_pos, root_R, joints):
    """World COM positions [nb][3] and rotations [nb][3][3]: root free joint
    (origin = COM) at (root_pos, root_R); every other body a hinge or slide
    with its joint value in `joints` (body order)."""
    nb = s["nbody"]
    org, rot, com = np.zeros((nb, 3)), np.zeros((nb, 3, 3)), np.zeros((nb, 3))
    ji = 0
    for b in range(nb):
        jt, p = int(s["body_jnt"][b]), int(s["body_parent"][b])
        if jt == scenes.JNT_FREE:
            org[b], rot[b] = root_pos, root_R
        else:
            po, pR = (org[p], rot[p]) if p >= 0 else (np.zeros(3), np.eye(3))
            R0 = pR @ _quat_mat(s["body_quat"][b])
            o = po + pR @ s["body_pos"][b]
            ax = s["jnt_axis"][b] / np.linalg.norm(s["jnt_axis"][b])
            th = joints[ji]
            ji += 1
            if jt == scenes.JNT_HINGE:
                R = R0 @ _expm_so3(th * ax)
            else:
                R = R0
                o = o + R0 @ ax * th
            org[b], rot[b] = o, R
        com[b] = org[b] + rot[b] @ s["body_ipos"][b]
    return com, rot


def _tree_with_free_root(seed, nchild=5):
    rng = np.random.default_rng([seed, 77])
    b = scenes._Builder(1)
    b.body(scenes.JNT_FREE, -1, mass=rng.uniform(0.5, 2.0), inertia=rng.uniform(0.02, 0.1, 3))
    for i in range(1, nchild + 1):
        jt = scenes.JNT_HINGE if rng.random() < 0.65 else scenes.JNT_SLIDE
        ax = rng.normal(size=3)
        b.body(jt, int(rng.integers(0, i)), pos=rng.uniform(-0.3, 0.3, 3), quat=rng.normal(size=4),
               ipos=rng.uniform(-0.2, 0.2, 3), axis=ax / np.linalg.norm(ax),
               mass=rng.uniform(0.2, 2.0), inertia=rng.uniform(0.01, 0.1, 3))
    s = b.build(gravity=(0.3, -0.2, -9.81))
    q = s["q0"][0].astype(float)
    q[0:3] = rng.uniform(-0.5, 0.5, 3)
    q[3:7] = rng.normal(size=4)
    q[3:7] /= np.linalg.norm(q[3:7])
    q[7:] = rng.uniform(-1.0, 1.0, nchild)
    v = rng.uniform(-1.0, 1.0, 6 + nchild)
    return s, q, v


class _Chart:
    """Chart xi = (x, phi, joints) around the state q: root orientation
    exp([phi]x) R0, root origin x, joint values as they are."""

    def __init__(self, s, q):
        self.s, self.q = s, q
        self.R0 = _quat_mat(q[3:7])
        self.nv = 6 + s["nbody"] - 1
        self.m = s["body_mass"][0]
        self.I = s["body_inertia"][0]

    def fk(self, xi):
        return _fk(self.s, xi[0:3], _expm_so3(xi[3:6]) @ self.R0, xi[6:])

    def xi0(self):
        return np.r_[self.q[0:3], 0.0, 0.0, 0.0, self.q[7:]]

    def jacobians(self, xi, eps=1e-5):
        """Per body: linear (COM) and angular Jacobians [3][nv] by central differences."""
        nb = self.s["nbody"]
        Jc, Jw = np.zeros((nb, 3, self.nv)), np.zeros((nb, 3, self.nv))
        for k in range(self.nv):
            e = np.zeros(self.nv)
            e[k] = eps
            cp, rp = self.fk(xi + e)
            cm, rm = self.fk(xi - e)
            Jc[:, :, k] = (cp - cm) / (2 * eps)
            for b in range(nb):
                A = rp[b] @ rm[b].T  # exp(2 eps [w_k]x) + O(eps^3)
                W = 0.5 * (A - A.T)
                Jw[b, :, k] = np.array([W[2, 1], W[0, 2], W[1, 0]]) / (2 * eps)
        return Jc, Jw

    def mass_matrix(self, xi):
        """M from the kinetic energy of the bodies over the difference Jacobians."""
        Jc, Jw = self.jacobians(xi)
        _, rot = self.fk(xi)
        M = np.zeros((self.nv, self.nv))
        for b in range(self.s["nbody"]):
            Iw = rot[b] @ np.diag(self.I[b]) @ rot[b].T
            M += self.m[b] * Jc[b].T @ Jc[b] + Jw[b].T @ Iw @ Jw[b]
        return M

    def potential(self, xi):
        com, _ = self.fk(xi)
        return -sum(self.m[b] * (self.s["gravity"] @ com[b]) for b in range(self.s["nbody"]))

    def bias(self, xi, xid, d=2e-3):
        """c = Mdot xid - dT/dxi + dU/dxi from Lagrange's equations, fourth-order
        central differences in xi."""
        def d4(f, dirn):
            return (-f(xi + 2 * d * dirn) + 8 * f(xi + d * dirn) - 8 * f(xi - d * dirn)
                    + f(xi - 2 * d * dirn)) / (12 * d)
        Mdot = d4(self.mass_matrix, xid)
        dT = np.zeros(self.nv)
        dU = np.zeros(self.nv)
        for i in range(self.nv):
            e = np.zeros(self.nv)
            e[i] = 1.0
            dT[i] = 0.5 * xid @ d4(self.mass_matrix, e) @ xid
            dU[i] = d4(self.potential, e)
        return Mdot @ xid - dT + dU


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_free_root_tree_jacobians_match_differences(seed):
    """Body Jacobians of a floating-base tree, including the free root's
    angular columns e_k x (com_b - root origin) on every descendant, against
    central differences of the test's own forward kinematics."""
    s, q, _ = _tree_with_free_root(seed)
    o = Oracle(s)
    ch = _Chart(s, q)
    com_o, rot_o = o.frames(0, q)
    com_t, rot_t = ch.fk(ch.xi0())
    np.testing.assert_allclose(com_o, com_t, atol=1e-13)
    np.testing.assert_allclose(rot_o, rot_t, atol=1e-13)
    Jc, Jw = ch.jacobians(ch.xi0())
    for b in range(s["nbody"]):
        J = o.jacobian(0, q, b)
        np.testing.assert_allclose(J[:3], Jc[b], atol=1e-8)
        np.testing.assert_allclose(J[3:], Jw[b], atol=1e-8)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_free_root_tree_mass_matrix(seed):
    """M of a floating-base tree against the kinetic energy of its bodies, and
    the free root's block against the composite-rigid-body closed forms:
    (sum m) I3, -(sum m)[c - x]x and sum_b (I_w,b + m_b [r_b]x^T [r_b]x),
    r_b = com_b - x."""
    s, q, _ = _tree_with_free_root(seed)
    o = Oracle(s)
    ch = _Chart(s, q)
    M = o.mass_matrix(0, q)
    np.testing.assert_allclose(M, ch.mass_matrix(ch.xi0()), rtol=1e-8, atol=1e-9)
    m, I = s["body_mass"][0], s["body_inertia"][0]
    com, rot = ch.fk(ch.xi0())
    mt = m.sum()
    ctot = (m[:, None] * com).sum(0) / mt
    x = q[0:3]
    np.testing.assert_allclose(M[0:3, 0:3], mt * np.eye(3), rtol=1e-13)
    np.testing.assert_allclose(M[0:3, 3:6], -mt * _skew(ctot - x), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(M[3:6, 0:3], M[0:3, 3:6].T, rtol=1e-12, atol=1e-13)
    Ic = sum(rot[b] @ np.diag(I[b]) @ rot[b].T + m[b] * _skew(com[b] - x).T @ _skew(com[b] - x)
             for b in range(s["nbody"]))
    np.testing.assert_allclose(M[3:6, 3:6], Ic, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_free_root_tree_bias_from_lagrange(seed):
    """c(q, v) of a floating-base tree (Coriolis, centrifugal, gyroscopic and
    gravity terms) against Lagrange's equations of the test's own kinetic and
    potential energy in the chart at phi = 0, and the power balance
    v^T c_v = 1/2 v^T Mdot v."""
    s, q, v = _tree_with_free_root(seed)
    o = Oracle(s)
    ch = _Chart(s, q)
    c_ref = ch.bias(ch.xi0(), v)
    c = o.bias(0, q, v)
    np.testing.assert_allclose(c, c_ref, rtol=1e-6, atol=1e-6 * np.abs(c_ref).max())
    # gravity part alone, and the power balance of the velocity part
    g0 = o.bias(0, q, np.zeros_like(v))
    np.testing.assert_allclose(g0, ch.bias(ch.xi0(), np.zeros_like(v)), rtol=1e-7,
                               atol=1e-7 * np.abs(g0).max())
    cv = c - g0
    d = 2e-3
    Md = (-ch.mass_matrix(ch.xi0() + 2 * d * v) + 8 * ch.mass_matrix(ch.xi0() + d * v)
          - 8 * ch.mass_matrix(ch.xi0() - d * v) + ch.mass_matrix(ch.xi0() - 2 * d * v)) / (12 * d)
    np.testing.assert_allclose(v @ cv, 0.5 * v @ Md @ v, rtol=1e-6, atol=1e-8)


def test_free_root_tree_momentum_rate():
    """Gravity off, no contacts: the step's prediction v_s = v - h M^-1 c keeps
    the tree's linear momentum sum m_b v_c,b to first order in h (the exact
    rate d/dt P = 0 of a free system), checked through the composite forms:
    P = (sum m)(v_x + w x (c - x)) + sum over joint columns."""
    s, q, v = _tree_with_free_root(3)
    s = dict(s)
    s["gravity"] = np.zeros(3)
    o = Oracle(s)
    ch = _Chart(s, q)
    M = o.mass_matrix(0, q)
    c = o.bias(0, q, v)
    vdot = -np.linalg.solve(M, c)
    # linear momentum P(q, v) = M[0:3] v; its rate along the motion must vanish
    h = 1e-4

    def P(qq_xi, vv):
        return ch.mass_matrix(qq_xi)[0:3] @ vv

    xi = ch.xi0()
    rate = (P(xi + h * v, v + h * vdot) - P(xi - h * v, v - h * vdot)) / (2 * h)
    assert np.abs(rate).max() < 1e-5 * max(1.0, np.abs(M[0:3] @ v).max())
