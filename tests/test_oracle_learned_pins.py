"""Pins of the oracle's learned-gain step (Sec. III.B allows K and D to be
learned; the network and the fallback rule are this build's design, stated in
the oracle's header): hand-derived values of single contacts and the
positive homogeneity of the facet law.

  * the exported features of a sphere on a plane equal the hand-computed gap,
    relative velocities at v_s, effective mass, friction and step;
  * a network whose outputs are constant biases b3_f scales facet f's impulse
    by exp(b3_f) exactly: for a sphere resting on the plane every facet's
    argument is a g h + k delta, so lambda_f = exp(b3_f) A (a g h + k delta)
    (facet order and output order pinned together);
  * with one constant c on every facet and the fallback off the step equals
    the plain step with k_user and d_user times exp(c) (max(., 0) is
    positively homogeneous);
  * the fallback rule on one normal facet, with the predicted penetration and
    normal energy worked out by hand, on both sides of each threshold.
"""
import math

import numpy as np
import pytest

from oracle import mlp
from oracle.cfo import Oracle
from paper_2603_12185_amd import scenes

def _bias_net(b3):
    """Zero weights, unit std: y = b3 for every contact."""
    p = np.zeros(mlp.NPARAM)
    p[mlp.OFF_STD:mlp.OFF_W1] = 1.0
    p[mlp.OFF_B3:mlp.OFF_B3 + len(b3)] = b3
    return p


def _rho(s, phi):
    """r/(1-r) of Eq. r_scaling at |phi| (x clamped to [0, 1]), written out."""
    rmin, rmax, w, mid, pw = s["solimp"]
    x = min(abs(phi) / w, 1.0)
    gam = mid * (x / mid) ** pw if x < mid else 1 - (1 - mid) * ((1 - x) / (1 - mid)) ** pw
    r = rmin + (rmax - rmin) * gam
    return r / (1 - r)


def test_features_of_a_sliding_spinning_sphere():
    """phi, v_n, u_1, u_2 at the smooth velocity (gravity applied), m_eff = m/3
    (one free body, trace 3/m), mu_t and h."""
    R, m = 0.05, 0.7
    s = scenes.sphere_on_plane(radius=R, mass=m, mu=(0.4, 0.0, 0.0), condim=3)
    R, m = s["geom_size"][0, 1, 0], s["body_mass"][0, 0]
    s["q0"][0, 2] = R - 0.003
    depth = R - float(s["q0"][0, 2])  # the float32 state's depth
    s["v0"][0] = (0.2, -0.1, -0.05, 1.5, 2.0, -3.0)
    o = Oracle(s)
    _, _, out = o.step(s["q0"], s["v0"])
    v = s["v0"][0].astype(float)
    h = s["h"]
    vs_lin = v[0:3] + h * s["gravity"]
    w = v[3:6]
    r = np.array([0.0, 0.0, -(R - depth / 2)])  # COM -> contact point (middle of the overlap)
    vp = vs_lin + np.cross(w, r)                  # sphere is body b, the plane static
    f = out["features"][0, 0]
    np.testing.assert_allclose(f[0], -depth, rtol=1e-12)
    np.testing.assert_allclose(f[1:4], [vp[2], vp[0], vp[1]], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(f[4:8], [m / 3, s["geom_friction"][0, 1, 0], h, 0.0], rtol=1e-12)


@pytest.mark.parametrize("condim", [3, 6])
def test_bias_network_scales_each_facet(condim):
    """Sphere resting at depth delta (v = 0, v_s = -g h along n): every facet's
    argument is a g h + k delta; the learned impulse of facet f is
    exp(b3_f) A (a g h + k delta) with A = rho(delta) m / 3; the fallback is off
    (a margin of 1 km)."""
    nf = scenes.nfacet(condim)
    s = scenes.sphere_on_plane(radius=0.05, mass=0.5, mu=(0.5, 0.02, 0.01), condim=condim)
    R, m = s["geom_size"][0, 1, 0], s["body_mass"][0, 0]
    s["q0"][0, 2] = R - 0.004
    delta = R - float(s["q0"][0, 2])
    b3 = np.array([0.5, -0.25, 1.0, -1.5, 0.125, -0.75, 2.0, -2.0, 0.25, 0.0])[:nf]
    o = Oracle(s)
    _, _, out = o.step(s["q0"], s["v0"], learned=(_bias_net(b3), 1e3))
    a = s["k_user"] * s["h"] + s["d_user"]
    A = _rho(s, delta) * m / 3
    arg = a * (-s["gravity"][2]) * s["h"] + s["k_user"] * delta
    np.testing.assert_allclose(out["impulse"][0, 0, :nf], np.exp(b3) * A * arg, rtol=1e-12)
    assert out["fallback"][0, 0] == 0


@pytest.mark.parametrize("c", [-0.7, 0.4])
def test_constant_network_equals_scaled_gains(c):
    """Same constant output on every facet, fallback off: the learned step of a
    mixed scene equals the plain step with k_user, d_user times exp(c)."""
    s = scenes.mixed_shapes(nworld=2, seed=17, condim=4)
    o = Oracle(s)
    q, v = s["q0"].astype(float), s["v0"].astype(float)
    for _ in range(40):
        q, v, _ = o.step(q, v, outputs=False)
    ql, vl, outl = o.step(q, v, learned=(_bias_net(np.full(mlp.NOUT, c)), 1e3))
    s2 = scenes.with_params(s, k_user=s["k_user"] * math.exp(c), d_user=s["d_user"] * math.exp(c))
    s2["k_user"], s2["d_user"] = s["k_user"] * math.exp(c), s["d_user"] * math.exp(c)
    qp, vp, outp = Oracle(s2).step(q, v)
    assert outl["ncon"].sum() > 5
    np.testing.assert_allclose(vl, vp, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(ql, qp, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(outl["impulse"], outp["impulse"], rtol=1e-11, atol=1e-16)


def test_fallback_rule_worked_by_hand():
    """One normal facet (condim 1), sphere of mass m approaching the plane at
    depth delta with normal speed u: heuristic impulse L_h = A (a (u + g h) +
    k delta), learned L_l = 200 L_h (b3 = ln 200); with w = 1/m the normal speeds
    after them v_x = -(u + g h) + w L_x, penetrations max(delta - h v_x, 0),
    energies v_x^2 / (2 w).  The decision and both slacks equal the hand values
    at margins on either side of the binding threshold."""
    R, m = 0.04, 0.3
    s = scenes.sphere_on_plane(radius=R, mass=m, mu=(0.0, 0.0, 0.0), condim=1)
    R, m = s["geom_size"][0, 1, 0], s["body_mass"][0, 0]
    s["q0"][0, 2] = R - 0.002
    s["v0"][0, 2] = -0.15
    delta, u = R - float(s["q0"][0, 2]), -float(s["v0"][0, 2])
    h, k, d = s["h"], s["k_user"], s["d_user"]
    a = k * h + d
    A = _rho(s, delta) * m / 3
    vn = -(u - s["gravity"][2] * h)
    Lh = A * (-a * vn + k * delta)
    Ll = 200 * Lh
    wi = 1 / m
    vh, vl = vn + wi * Lh, vn + wi * Ll
    ph, pl = max(delta - h * vh, 0), max(delta - h * vl, 0)
    eh, el = 0.5 * vh * vh / wi, 0.5 * vl * vl / wi
    o = Oracle(s)
    # the learned impulse reverses the approach: less penetration, more energy; the energy
    # test binds at delta* with (delta*/h)^2 / (2 w) = el - eh
    assert pl <= ph and el > eh
    dstar = h * math.sqrt(2 * wi * (el - eh))
    for margin, keep in ((0.5 * dstar, False), (2.0 * dstar, True)):
        _, v1, out = o.step(s["q0"], s["v0"], learned=(_bias_net([math.log(200.0)]), margin))
        em = 0.5 * (margin / h) ** 2 / wi
        np.testing.assert_allclose(out["fallback_slack"][0, 0], [ph + margin - pl, eh + em - el],
                                   rtol=1e-10, atol=1e-15)
        assert out["fallback"][0, 0] == (0 if keep else 1)
        np.testing.assert_allclose(out["impulse"][0, 0, 0], Ll if keep else Lh, rtol=1e-12)
        np.testing.assert_allclose(v1[0, 2], vl if keep else vh, rtol=1e-12)
    # a gain 1/16 of the heuristic's penetrates more: the penetration test binds
    _, _, out = o.step(s["q0"], s["v0"], learned=(_bias_net([math.log(1 / 16)]), 1e-6))
    vq = vn + wi * Lh / 16
    pq = max(delta - h * vq, 0)
    assert pq > ph + 1e-6
    assert out["fallback"][0, 0] == 1
    np.testing.assert_allclose(out["fallback_slack"][0, 0, 0], ph + 1e-6 - pq, rtol=1e-10)
