"""Pins of the FP64 oracle against closed forms, invariants and textbook results.

Each test names the part of the method it pins and the passage of the paper it
follows.  None of them re-types the oracle's own formulas: expected values come
from hand-derived closed forms of the discrete update, textbook mechanics,
finite differences or conservation laws.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle.cfo import Oracle, OracleError
from paper_2603_12185_amd import scenes

G = 9.81
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def rho_star(s):
    r = s["solimp"][1]
    return r / (1 - r)


def steady_depth(s, nfacet):
    """Resting depth of a point-like body under the impulse law (all facets active, |phi| >= w).

    Derivation: at rest v_s,n = -g h; every facet carries A(a g h + k delta) with
    A = rho* m / 3 (COM trace 3/m); the facets' normal parts sum to m g h.
    """
    g = -s["gravity"][2]
    a = s["k_user"] * s["h"] + s["d_user"]
    return (g * s["h"] / s["k_user"]) * (3.0 / (nfacet * rho_star(s)) - a)


# ---------------------------------------------------------------- golden
def test_paper_constants_match_defaults():
    gold = json.load(open(GOLD))
    assert list(scenes.SOLIMP_DEFAULT) == gold["solimp_default"]["value"]
    s = scenes.sphere_on_plane()
    np.testing.assert_allclose(s["h"], gold["timestep"]["value"], rtol=1e-7)


# ---------------------------------------------------------------- P-ff, P-rot
def test_free_fall_closed_form():
    """No contacts: v_n = v0 + n h g, x_n = x0 + n h v0 + h^2 g n(n+1)/2 (semi-implicit Euler)."""
    s = scenes.sphere_on_plane(z0=50.0)
    s["v0"][0, :] = [0.3, -0.2, 1.5, 2.0, -1.0, 0.5]
    o = Oracle(s)
    n = 200
    q, v = o.rollout(n)
    h, g = s["h"], s["gravity"]
    x0, v0 = s["q0"][0, :3].astype(float), s["v0"][0, :3].astype(float)
    np.testing.assert_allclose(v[0, :3], v0 + n * h * g, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(q[0, :3], x0 + n * h * v0 + h * h * g * n * (n + 1) / 2,
                               rtol=1e-12, atol=1e-12)


def test_torque_free_isotropic_rotation():
    """Isotropic body: omega constant, quat_n = exp(n h omega) (x) quat_0."""
    s = scenes.sphere_on_plane(z0=50.0)
    q0 = np.array([0.8, 0.1, -0.3, 0.5])
    q0 /= np.linalg.norm(q0)
    s["q0"][0, 3:7] = q0
    om = np.array([2.0, -1.0, 0.5])
    s["v0"][0, 3:6] = om
    s["q0"][0, 3:7] = s["q0"][0, 3:7]  # float32 storage
    q0 = s["q0"][0, 3:7].astype(float)
    om = s["v0"][0, 3:6].astype(float)
    o = Oracle(s)
    n = 300
    q, v = o.rollout(n)
    np.testing.assert_allclose(v[0, 3:6], om, rtol=1e-13)
    th = n * s["h"] * om
    ang = np.linalg.norm(th)
    e = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * th / ang)])
    want = qmul(e, q0)
    want /= np.linalg.norm(want)
    np.testing.assert_allclose(q[0, 3:7], want, atol=1e-12)


# ---------------------------------------------------------------- P-rest
@pytest.mark.parametrize("k,d,condim", [(0.1, 0.001, 3), (0.5, 0.005, 3), (0.3, 0.001, 3),
                                        (0.1, 0.001, 6), (0.1, 0.001, 4), (0.1, 0.001, 1)])
def test_resting_depth_sphere(k, d, condim):
    s = scenes.sphere_on_plane(k_user=k, d_user=d, condim=condim, z0=0.05)
    nf = scenes.nfacet(condim)
    want = steady_depth(s, nf)
    assert want >= s["solimp"][2]  # closed form valid in the saturated branch
    q, v = Oracle(s).rollout(3000 if nf > 1 else 12000)
    R = s["geom_size"][0, 1, 0]
    np.testing.assert_allclose(R - q[0, 2], want, rtol=1e-10)
    assert abs(v[0, 2]) < 1e-12


def test_resting_depth_values_quoted():
    """Numerical values of the closed form at the printed gains (h = 2 ms)."""
    for (k, d, nf), mm in [((0.1, 0.001, 4), 7.5093), ((0.5, 0.005, 4), 1.3135),
                           ((0.3, 0.001, 4), 2.4769), ((0.1, 0.001, 10), 2.8625)]:
        s = scenes.sphere_on_plane(k_user=k, d_user=d)
        assert abs(steady_depth(s, nf) * 1e3 - mm) < 1e-3


def test_resting_depth_flat_cube():
    """Flat cube: 4 corner contacts x 4 facets share the load; each contact's
    impedance uses the cube's COM trace 3/m."""
    s = scenes.boxes_drop()
    s = scenes.select_worlds(s, [0])
    # keep only the first box, flat, touching the ground
    s2 = scenes._Builder(1)
    s2.geom(scenes.PLANE)
    b = s2.body(scenes.JNT_FREE, pos=(0, 0, 0.05), mass=1.0, inertia=(1 / 600,) * 3)
    s2.geom(scenes.BOX, b, size=(0.05, 0.05, 0.05), friction=(0.5, 0, 0))
    s2 = s2.build()
    q, v, traj, outs = Oracle(s2).rollout(800, record=True)
    assert outs[-1]["ncon"][0] == 4
    assert list(outs[-1]["sub"][0, :4]) == [0, 1, 2, 3]
    want = steady_depth(s2, 16)
    np.testing.assert_allclose(s2["geom_size"][0, 1, 2] - q[0, 2], want, rtol=1e-9)
    np.testing.assert_allclose(-outs[-1]["dist"][0, :4], want, rtol=1e-9)


def test_penetration_monotone_in_gains():
    """Resting depth falls with k_user and with d_user, the ordering of the
    paper's penetration table (Sec. IV.A)."""
    gold = json.load(open(GOLD))["penetration_table_mm"]["rows"]
    depth = {}
    for r in gold:
        s = scenes.sphere_on_plane(k_user=r["k_user"], d_user=r["d_user"], z0=0.05)
        q, _ = Oracle(s).rollout(2500)
        depth[(r["k_user"], r["d_user"])] = s["geom_size"][0, 1, 0] - q[0, 2]
    for d in (0.001, 0.005):
        assert depth[(0.1, d)] > depth[(0.3, d)] > depth[(0.5, d)]
    for k in (0.1, 0.3, 0.5):
        assert depth[(k, 0.001)] > depth[(k, 0.005)]
    # same ordering as the table's means
    order_model = sorted(depth, key=depth.get)
    order_table = sorted(depth, key=lambda kd: next(r["mean"] for r in gold
                                                    if (r["k_user"], r["d_user"]) == kd))
    assert order_model == order_table


# ---------------------------------------------------------------- P-slide
def _settled_point_mass(mu, k=0.1, d=0.001):
    """Point mass at its resting depth; returns the scene and the float64 state."""
    s = scenes.point_mass(mu=mu, k_user=k, d_user=d)
    delta = steady_depth(s, 4)
    q = s["q0"].astype(float)
    q[0, 2] = s["geom_size"][0, 1, 0] - delta
    return s, q


def test_slide_stick_regime_geometric_decay():
    """All four facets active: u_{n+1} = (1 - 2 rho* a mu^2 / 3) u_n in every
    tangential direction; the normal state stays at rest."""
    mu = 0.5
    for ang in (0.0, math.pi / 4, 1.1):
        s, q = _settled_point_mass(mu)
        a = s["k_user"] * s["h"] + s["d_user"]
        u1 = 3 * G * s["h"] / (4 * rho_star(s) * a * mu)
        u0 = 0.6 * u1
        s["v0"][0, 0:2] = (u0 * math.cos(ang), u0 * math.sin(ang))
        v = s["v0"].astype(float)
        o = Oracle(s)
        fac = 1 - 2 * rho_star(s) * a * mu * mu / 3
        for n in range(1, 60):
            q, v, _ = o.step(q, v, outputs=False)
            np.testing.assert_allclose(v[0, 0:2], fac ** n * np.array(s["v0"][0, 0:2], float),
                                       rtol=1e-11, atol=1e-15)
            assert abs(v[0, 2]) < 1e-12


def test_slide_diagonal_identity_and_deceleration():
    """Diagonal sliding with only the two front facets active: the per-step
    tangential change equals mu/sqrt(2) times the normal change, and the
    steady deceleration is mu g / sqrt(2)."""
    mu = 0.1
    s, q = _settled_point_mass(mu)
    u0 = 15.0
    s["v0"][0, 0:2] = (u0 / math.sqrt(2), u0 / math.sqrt(2))
    o = Oracle(s)
    v = s["v0"].astype(float)
    g = -s["gravity"][2]
    mu = s["geom_friction"][0, 1, 0]
    speeds = []
    for n in range(1100):
        q1, v1, out = o.step(q, v)
        if out["ncon"][0] == 1:
            lam = out["impulse"][0, 0]
            assert lam[2] == 0.0 and lam[3] == 0.0 and lam[0] > 0 and lam[1] > 0
            dw_contact = (v1[0, 2] - out["v_smooth"][0, 2])
            du = np.linalg.norm(v1[0, 0:2] - out["v_smooth"][0, 0:2])
            np.testing.assert_allclose(du, mu / math.sqrt(2) * dw_contact, rtol=1e-10)
        speeds.append(np.linalg.norm(v1[0, 0:2]))
        q, v = q1, v1
    decel = (speeds[1000] - speeds[1099]) / (99 * s["h"])
    # the normal load lags the slowly falling speed by a few 1e-5 (quasi-steady)
    np.testing.assert_allclose(decel, mu * g / math.sqrt(2), rtol=5e-5)


def test_slide_aligned_deceleration():
    """Aligned sliding, three facets active (u1 <= u < u2 = 4 u1): deceleration
    mu g (1 + 2 u / u2) / 3 at quasi-steady normal load."""
    mu = 0.5
    s, q = _settled_point_mass(mu)
    a = s["k_user"] * s["h"] + s["d_user"]
    u1 = 3 * G * s["h"] / (4 * rho_star(s) * a * mu)
    u2 = 4 * u1
    s["v0"][0, 0] = 0.8 * u2
    o = Oracle(s)
    v = s["v0"].astype(float)
    g = -s["gravity"][2]
    mu = s["geom_friction"][0, 1, 0]
    us = []
    for n in range(400):
        q1, v1, out = o.step(q, v)
        lam = out["impulse"][0, 0]
        us.append(v1[0, 0])
        if n > 100:
            assert lam[0] > 0 and lam[1] > 0 and lam[3] > 0 and lam[2] == 0.0
            # per-step identity of the 3-active pattern:
            # du_t = -(mu/3) (dw_contact + (2 rho* a mu / 3) u_s)
            us_ = out["v_smooth"][0, 0]
            dw = v1[0, 2] - out["v_smooth"][0, 2]
            np.testing.assert_allclose(v1[0, 0] - us_,
                                       -(mu / 3) * (dw + 2 * rho_star(s) * a * mu * us_ / 3),
                                       rtol=1e-11)
        q, v = q1, v1
    for n in (200, 300):
        u = us[n]
        dec = (us[n - 1] - us[n + 1]) / (2 * s["h"])
        # quasi-steady normal load: the normal state lags the slowly falling speed
        np.testing.assert_allclose(dec, mu * g * (1 + 2 * u / u2) / 3, rtol=2e-2)


def test_stick_threshold_separates_regimes():
    """Below u1 the back facet stays active (stick); above it the back facet
    switches off (slide)."""
    mu = 0.5
    for frac, back_active in ((0.95, True), (1.05, False)):
        s, q = _settled_point_mass(mu)
        a = s["k_user"] * s["h"] + s["d_user"]
        u1 = 3 * G * s["h"] / (4 * rho_star(s) * a * mu)
        v = s["v0"].astype(float)
        v[0, 0] = frac * u1
        _, _, out = Oracle(s).step(q, v)
        assert (out["impulse"][0, 0, 2] > 0) == back_active


# ---------------------------------------------------------------- P-cone, P-sep
def _cone_check(out, scene, nf):
    mu_all = np.maximum(scene["geom_friction"][:, out["geom"][..., 0].clip(0)],
                        scene["geom_friction"][:, out["geom"][..., 1].clip(0)])
    dirs = np.array([[1, 0], [0, 1], [-1, 0], [0, -1]], float)
    for w in range(out["ncon"].shape[0]):
        for k in range(out["ncon"][w]):
            lam = out["impulse"][w, k]
            assert (lam >= 0).all()
            N = lam.sum()
            mu = np.maximum(scene["geom_friction"][w, out["geom"][w, k, 0]],
                            scene["geom_friction"][w, out["geom"][w, k, 1]])
            if nf >= 4:
                ft = mu[0] * (lam[0:4, None] * dirs).sum(0)
                assert np.linalg.norm(ft) <= mu[0] * lam[0:4].sum() * (1 + 1e-12) + 1e-300
                assert mu[0] * lam[0:4].sum() <= mu[0] * N * (1 + 1e-12)
            if nf >= 6:
                mt = mu[1] * (lam[4] - lam[5])
                assert abs(mt) <= mu[1] * N * (1 + 1e-12)
            if nf == 10:
                mr = mu[2] * (lam[6:10, None] * dirs).sum(0)
                assert np.linalg.norm(mr) <= mu[2] * lam[6:10].sum() * (1 + 1e-12) + 1e-300
    del mu_all


@pytest.mark.parametrize("condim", [3, 4, 6])
def test_primal_cone_by_construction(condim):
    s = scenes.mixed_shapes(nworld=3, condim=condim)
    o = Oracle(s)
    q, v = s["q0"].astype(float), s["v0"].astype(float)
    total = 0
    for _ in range(30):
        q, v, out = o.step(q, v)
        _cone_check(out, s, o.nf)
        total += out["ncon"].sum()
    assert total > 0


def test_coulomb_bound_per_step():
    """Single contact point mass: |du_t| <= mu * dw_contact every step."""
    mu = 0.4
    s, q = _settled_point_mass(mu)
    s["v0"][0, 0:3] = (3.0, -1.0, -0.5)
    o = Oracle(s)
    v = s["v0"].astype(float)
    for _ in range(300):
        q1, v1, out = o.step(q, v)
        du = np.linalg.norm(v1[0, :2] - out["v_smooth"][0, :2])
        dw = v1[0, 2] - out["v_smooth"][0, 2]
        assert du <= mu * dw * (1 + 1e-12) + 1e-15
        q, v = q1, v1


def test_separating_contact_has_zero_impulse():
    """If every facet argument -(k h + d) s - k phi is <= 0 the impulse is exactly zero."""
    s = scenes.sphere_on_plane(z0=0.0499, mu=(0.5, 0, 0))
    s["v0"][0, 2] = 2.0  # leaving fast
    q1, v1, out = Oracle(s).step(s["q0"], s["v0"])
    assert out["ncon"][0] == 1
    assert (out["impulse"][0, 0] == 0).all()
    np.testing.assert_array_equal(v1[0], out["v_smooth"][0])


# ---------------------------------------------------------------- P-mom
@pytest.mark.parametrize("condim", [3, 4, 6])
def test_momentum_conserved_in_free_collisions(condim):
    """Gravity off, no static geometry: total linear and angular momentum are
    conserved by every step (equal and opposite impulses at a shared point)."""
    for sc in (scenes.two_spheres(condim=condim), scenes.sphere_cluster(nsphere=6, condim=condim)):
        o = Oracle(sc)
        nb = sc["nbody"]
        m = sc["body_mass"][0]
        I = sc["body_inertia"][0]

        def momenta(q, v):
            qb, vb = q.reshape(nb, 7), v.reshape(nb, 6)
            P = (m[:, None] * vb[:, :3]).sum(0)
            L = (np.cross(qb[:, :3], m[:, None] * vb[:, :3]) + I * vb[:, 3:]).sum(0)
            return P, L

        q, v = sc["q0"][0].astype(float), sc["v0"][0].astype(float)
        P0, L0 = momenta(q, v)
        sawcontact = False
        for _ in range(200):
            q2, v2, out = o.step(q[None], v[None])
            sawcontact |= out["ncon"][0] > 0
            q, v = q2[0], v2[0]
            P, L = momenta(q, v)
            np.testing.assert_allclose(P, P0, atol=1e-12 * (1 + np.abs(P0).max()))
            np.testing.assert_allclose(L, L0, atol=1e-12 * (1 + np.abs(L0).max()))
        assert sawcontact


# ---------------------------------------------------------------- P-imp
def test_impedance_shape_values():
    s = scenes.sphere_on_plane()
    o = Oracle(s)
    si = s["solimp"]
    rmin, rmax, w, mid = si[0], si[1], si[2], si[3]
    np.testing.assert_allclose(o.impedance_ratio(0.0), rmin / (1 - rmin), rtol=1e-15)
    r_mid = rmin + (rmax - rmin) * mid
    np.testing.assert_allclose(o.impedance_ratio(mid * w), r_mid / (1 - r_mid), rtol=1e-14)
    np.testing.assert_allclose(o.impedance_ratio(-mid * w), r_mid / (1 - r_mid), rtol=1e-14)
    for phi in (w, 2 * w, -0.05):
        np.testing.assert_allclose(o.impedance_ratio(phi), rmax / (1 - rmax), rtol=1e-15)
    assert abs(o.impedance_ratio(0.0) - 9.0) < 1e-5 and abs(o.impedance_ratio(0.01) - 19.0) < 1e-4
    # gamma: 0 at 0, 1 at 1, continuous and C1 at the midpoint, monotone
    assert o.gamma(0.0) == 0.0 and abs(o.gamma(1.0) - 1.0) < 1e-15
    e = 1e-7
    gl, gr = o.gamma(mid - e), o.gamma(mid + e)
    assert abs(gl - gr) < 1e-6
    dl = (o.gamma(mid) - o.gamma(mid - e)) / e
    dr = (o.gamma(mid + e) - o.gamma(mid)) / e
    assert abs(dl - dr) < 1e-5
    xs = np.linspace(0, 1.5, 301)
    gs = [o.gamma(x) for x in xs]
    assert all(b >= a for a, b in zip(gs, gs[1:]))


# ---------------------------------------------------------------- P-6D
@pytest.mark.parametrize("condim", [4, 6])
def test_torsional_stick_decay(condim):
    """Spin about the normal, both torsional facets active:
    omega_{n+1} = (1 - 5 rho* a mu_tor^2 / (3 R^2)) omega_n."""
    R, mu_tor = 0.05, 0.02
    s = scenes.sphere_on_plane(radius=R, mu=(0.5, mu_tor, 0.001), condim=condim)
    nf = scenes.nfacet(condim)
    R = s["geom_size"][0, 1, 0]
    s["q0"][0, 2] = R - steady_depth(s, nf)
    s["v0"][0, 5] = 0.5
    o = Oracle(s)
    a = s["k_user"] * s["h"] + s["d_user"]
    mu_tor = s["geom_friction"][0, 1, 1]
    m, I = s["body_mass"][0, 0], s["body_inertia"][0, 0, 2]
    # 1 - 2 A a mu_tor^2 / I with A = rho* m / 3; equals 1 - 5 rho* a mu_tor^2 / (3 R^2) for I = 0.4 m R^2
    fac = 1 - 2 * (rho_star(s) * m / 3) * a * mu_tor ** 2 / I
    assert abs(fac - (1 - 5 * rho_star(s) * a * mu_tor ** 2 / (3 * R * R))) < 1e-9
    q, v = s["q0"].astype(float), s["v0"].astype(float)
    w0 = v[0, 5]
    for n in range(1, 50):
        w_before = v[0, 5]
        q, v, out = o.step(q, v)
        assert out["impulse"][0, 0, 4] > 0 and out["impulse"][0, 0, 5] > 0
        # facet order and sign: sigma = +1 first, lambda(+) - lambda(-) = 2 A a mu_tor (n . w)
        np.testing.assert_allclose(out["impulse"][0, 0, 4] - out["impulse"][0, 0, 5],
                                   2 * (rho_star(s) * m / 3) * a * mu_tor * w_before, rtol=1e-9)
        np.testing.assert_allclose(v[0, 5], fac ** n * w0, rtol=1e-11)
        np.testing.assert_allclose(v[0, 3:5], 0, atol=1e-14)


@pytest.mark.parametrize("direction", [(1.0, 0.0), (0.6, -0.8)])
def test_rolling_stick_decay(direction):
    """Rolling facets alone (condim 6, mu_t = mu_tor = 0): a sphere resting on
    the plane with angular velocity w in the tangent plane.  With mu_t = 0 the
    tangential and torsional facets are plain normal rows, so no tangential
    force acts and nothing but the rolling couple -mu_rol sum_f lambda_f d_f
    turns the sphere (its torque about the COM from forces along n vanishes).
    While all four rolling facets are active, lambda_(+d) - lambda_(-d) =
    2 A a mu_rol (d . w) for d = t1, t2 (Eq. cf_wrench), so every tangential
    direction decays by the same factor per step:
    w_{n+1} = (1 - 2 A a mu_rol^2 / I) w_n, A = rho* m / 3, while the normal
    spin, the linear velocity and the normal state are untouched by w."""
    R, mu_rol = 0.05, 0.01
    s = scenes.sphere_on_plane(radius=R, mu=(0.0, 0.0, mu_rol), condim=6)
    R = s["geom_size"][0, 1, 0]
    mu_rol = s["geom_friction"][0, 1, 2]
    s["q0"][0, 2] = R - steady_depth(s, 10)
    w0 = 8.0 * np.array(direction)
    s["v0"][0, 3:5] = w0
    s["v0"][0, 0:2] = (0.3, -0.2)  # free tangential slip (mu_t = 0)
    o = Oracle(s)
    a = s["k_user"] * s["h"] + s["d_user"]
    m, I = s["body_mass"][0, 0], s["body_inertia"][0, 0, 0]
    fac = 1 - 2 * (rho_star(s) * m / 3) * a * mu_rol ** 2 / I
    assert 0.99 < fac < 1
    q, v = s["q0"].astype(float), s["v0"].astype(float)
    w_start = v[0, 3:5].copy()
    vt = v[0, 0:2].copy()
    A = rho_star(s) * m / 3
    for n in range(1, 60):
        w_before = v[0, 3:5].copy()
        q, v, out = o.step(q, v)
        assert out["ncon"][0] == 1 and (out["impulse"][0, 0, 6:10] > 0).all()
        # facet order and sign (t1 = +x, t2 = +y here): lambda(+d) - lambda(-d) = 2 A a mu_rol (d . w)
        lam = out["impulse"][0, 0]
        np.testing.assert_allclose(out["frame"][0, 0, 3:9], [1, 0, 0, 0, 1, 0], atol=1e-15)
        np.testing.assert_allclose([lam[6] - lam[8], lam[7] - lam[9]], 2 * A * a * mu_rol * w_before,
                                   rtol=1e-9, atol=1e-18)
        assert -out["dist"][0, 0] >= s["solimp"][2]  # |phi| >= w: rho = rho*
        np.testing.assert_allclose(v[0, 3:5], fac ** n * w_start, rtol=1e-11, atol=1e-15)
        assert abs(v[0, 5]) < 1e-15
        np.testing.assert_allclose(v[0, 0:2], vt, rtol=1e-13, atol=1e-15)


def test_rolling_friction_decays_monotonically():
    """Rolling sphere (condim 6) with tangential friction: speed decays
    monotonically and faster with larger mu_rol (the exact stick-regime decay
    of the rolling facets alone is pinned by test_rolling_stick_decay)."""
    finals = []
    for mu_rol in (0.0, 0.002, 0.005):
        R = 0.05
        s = scenes.sphere_on_plane(radius=R, mu=(1.0, 0.0, mu_rol), condim=6)
        s["q0"][0, 2] = R - steady_depth(s, 10)
        s["v0"][0, 0] = 0.5
        s["v0"][0, 4] = 0.5 / R  # rolling without slip about +y
        o = Oracle(s)
        q, v = s["q0"].astype(float), s["v0"].astype(float)
        prev = np.inf
        for _ in range(400):
            q, v, out = o.step(q, v)
            sp = abs(v[0, 0])
            assert sp <= prev + 1e-12
            prev = sp
            _cone_check(out, s, 10)
        finals.append(prev)
    assert finals[0] > finals[1] > finals[2]


# ---------------------------------------------------------------- P-tree
def test_free_body_mass_and_bias():
    s = scenes.mixed_shapes(nworld=1)
    o = Oracle(s)
    q, v = s["q0"][0].astype(float), s["v0"][0].astype(float)
    M = o.mass_matrix(0, q)
    c = o.bias(0, q, v)
    com, rot = o.frames(0, q)
    for b in range(s["nbody"]):
        m = s["body_mass"][0, b]
        Iw = rot[b] @ np.diag(s["body_inertia"][0, b]) @ rot[b].T
        blk = M[6 * b:6 * b + 6, 6 * b:6 * b + 6]
        np.testing.assert_allclose(blk[:3, :3], m * np.eye(3), atol=1e-15)
        np.testing.assert_allclose(blk[3:, 3:], Iw, rtol=1e-13, atol=1e-18)
        np.testing.assert_allclose(blk[:3, 3:], 0, atol=1e-15)
        w = v[6 * b + 3:6 * b + 6]
        np.testing.assert_allclose(c[6 * b:6 * b + 3], -m * s["gravity"], rtol=1e-14)
        np.testing.assert_allclose(c[6 * b + 3:6 * b + 6], np.cross(w, Iw @ w), rtol=1e-12,
                                   atol=1e-15)
    off = M.copy()
    for b in range(s["nbody"]):
        off[6 * b:6 * b + 6, 6 * b:6 * b + 6] = 0
    assert np.abs(off).max() == 0


def test_double_pendulum_textbook_dynamics():
    """Planar two-link arm: M, Coriolis and gravity terms of the textbook form
    (relative joint angles, link COMs at lc1, lc2)."""
    l1, lc1, lc2, m1, m2 = 0.6, 0.3, 0.25, 1.3, 0.7
    i1, i2 = (0.02, 0.03, 0.01), (0.015, 0.01, 0.02)
    s = scenes.double_pendulum(l1=l1, lc1=lc1, lc2=lc2, m1=m1, m2=m2, i1=i1, i2=i2)
    o = Oracle(s)
    I1, I2 = s["body_inertia"][0, 0, 1], s["body_inertia"][0, 1, 1]  # about the hinge (y) axis
    m1, m2 = s["body_mass"][0]
    l1 = s["body_pos"][1, 0]
    lc1, lc2 = s["body_ipos"][0, 0], s["body_ipos"][1, 0]
    g = -s["gravity"][2]
    rng = np.random.default_rng(0)
    for _ in range(5):
        th = rng.uniform(-2, 2, 2)
        dth = rng.uniform(-3, 3, 2)
        M = o.mass_matrix(0, th)
        c = o.bias(0, th, dth)
        c2 = math.cos(th[1])
        M11 = m1 * lc1 ** 2 + m2 * (l1 ** 2 + lc2 ** 2 + 2 * l1 * lc2 * c2) + I1 + I2
        M12 = m2 * (lc2 ** 2 + l1 * lc2 * c2) + I2
        M22 = m2 * lc2 ** 2 + I2
        np.testing.assert_allclose(M, [[M11, M12], [M12, M22]], rtol=1e-12)
        hh = -m2 * l1 * lc2 * math.sin(th[1])
        cor = np.array([hh * (2 * dth[0] * dth[1] + dth[1] ** 2), -hh * dth[0] ** 2])
        grav = np.array([(m1 * lc1 + m2 * l1) * g * math.cos(th[0])
                         + m2 * lc2 * g * math.cos(th[0] + th[1]),
                         m2 * lc2 * g * math.cos(th[0] + th[1])])
        np.testing.assert_allclose(c, cor + grav, rtol=1e-11, atol=1e-12)


def _random_tree_scene(seed):
    rng = np.random.default_rng(seed)
    b = scenes._Builder(1)
    nb = 6
    for i in range(nb):
        jt = scenes.JNT_HINGE if rng.random() < 0.6 else scenes.JNT_SLIDE
        parent = -1 if i == 0 else int(rng.integers(-1, i))
        ax = rng.normal(size=3)
        b.body(jt, parent, pos=rng.uniform(-0.3, 0.3, 3), quat=rng.normal(size=4),
               ipos=rng.uniform(-0.2, 0.2, 3), axis=ax / np.linalg.norm(ax),
               mass=rng.uniform(0.2, 2.0), inertia=rng.uniform(0.01, 0.1, 3))
    return b.build(gravity=(0.1, -0.2, -9.81))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tree_mass_matrix_and_power_balance(seed):
    """Random hinge/slide trees: M symmetric positive definite; Jacobian matches
    finite differences of the COM positions; the velocity-product part of c
    satisfies v^T c_v = 1/2 v^T Mdot v (its power equals the rate of change of
    kinetic energy at fixed v)."""
    s = _random_tree_scene(seed)
    o = Oracle(s)
    rng = np.random.default_rng(100 + seed)
    q = rng.uniform(-1, 1, o.nq)
    v = rng.uniform(-1, 1, o.nv)
    M = o.mass_matrix(0, q)
    np.testing.assert_allclose(M, M.T, rtol=1e-13, atol=1e-15)
    assert np.linalg.eigvalsh(M).min() > 0
    eps = 1e-6
    com_p, _ = o.frames(0, q + eps * v)
    com_m, _ = o.frames(0, q - eps * v)
    for b in range(s["nbody"]):
        J = o.jacobian(0, q, b)
        np.testing.assert_allclose(J[:3] @ v, (com_p[b] - com_m[b]) / (2 * eps), rtol=1e-7,
                                   atol=1e-9)
    g0 = o.bias(0, q, np.zeros(o.nv))
    cv = o.bias(0, q, v) - g0
    Md = (o.mass_matrix(0, q + eps * v) - o.mass_matrix(0, q - eps * v)) / (2 * eps)
    np.testing.assert_allclose(v @ cv, 0.5 * v @ Md @ v, rtol=1e-6, atol=1e-9)
    # gravity part: generalized gravity is minus the gradient of the potential
    pot = lambda qq: -sum(s["body_mass"][0, b] * (s["gravity"] @ o.frames(0, qq)[0][b])
                          for b in range(s["nbody"]))
    grad = np.array([(pot(q + eps * e) - pot(q - eps * e)) / (2 * eps) for e in np.eye(o.nq)])
    np.testing.assert_allclose(g0, grad, rtol=1e-6, atol=1e-8)


def test_pendulum_small_angle_period():
    """Single hinge pendulum: small-angle period 2 pi sqrt(I_pivot / (m g l))."""
    L, m, r = 0.5, 1.0, 0.02
    s = scenes.pendulum(length=L, mass=m, radius=r, h=0.0005)
    s["h"] = float(scenes.f32(0.0002))
    s["q0"][0, 0] = 0.01
    o = Oracle(s)
    Ipiv = s["body_inertia"][0, 0, 1] + s["body_mass"][0, 0] * L ** 2
    T = 2 * math.pi * math.sqrt(Ipiv / (s["body_mass"][0, 0] * G * L))
    q, v = s["q0"].astype(float), s["v0"].astype(float)
    ths, ts = [], []
    for n in range(int(2.5 * T / s["h"])):
        q, v, _ = o.step(q, v, outputs=False)
        ths.append(q[0, 0])
    ths = np.array(ths)
    # downward zero crossings (linear interpolation)
    cross = [i + ths[i] / (ths[i] - ths[i + 1]) for i in range(len(ths) - 1)
             if ths[i] > 0 >= ths[i + 1]]
    period = (cross[1] - cross[0]) * s["h"]
    np.testing.assert_allclose(period, T, rtol=1e-3)


def test_trace_reading():
    """tr(J_b M^-1 J_b^T) over the COM rows: 3/m for free bodies and for the
    slide-joint point mass; l^2 / I_pivot for a pendulum."""
    s = scenes.mixed_shapes(nworld=1)
    _, _, out = Oracle(s).step(s["q0"], s["v0"])
    np.testing.assert_allclose(out["trace"][0], 3 / s["body_mass"][0], rtol=1e-12)
    s = scenes.point_mass(mass=2.0)
    _, _, out = Oracle(s).step(s["q0"], s["v0"])
    np.testing.assert_allclose(out["trace"][0, 2], 1.5, rtol=1e-13)
    s = scenes.pendulum(length=0.5, mass=1.0)
    s["q0"][0, 0] = 0.3
    _, _, out = Oracle(s).step(s["q0"], s["v0"])
    Ipiv = s["body_inertia"][0, 0, 1] + 0.25
    np.testing.assert_allclose(out["trace"][0, 0], 0.25 / Ipiv, rtol=1e-12)


# ---------------------------------------------------------------- P-geom
def test_geometry_sphere_plane_and_sphere_sphere():
    s = scenes.mixed_shapes(nworld=2, seed=3)
    o = Oracle(s)
    q = s["q0"].astype(float)
    _, _, out = o.step(q, s["v0"])
    com = [o.frames(w, q[w])[0] for w in range(2)]
    for w in range(2):
        for k in range(out["ncon"][w]):
            ga, gb = out["geom"][w, k]
            ta, tb = s["geom_type"][ga], s["geom_type"][gb]
            n = out["frame"][w, k, :3]
            np.testing.assert_allclose(np.linalg.norm(n), 1, rtol=1e-14)
            t1, t2 = out["frame"][w, k, 3:6], out["frame"][w, k, 6:9]
            np.testing.assert_allclose(np.stack([n, t1, t2]) @ np.stack([n, t1, t2]).T,
                                       np.eye(3), atol=1e-14)
            np.testing.assert_allclose(np.cross(n, t1), t2, atol=1e-14)
            if ta == scenes.PLANE and tb == scenes.SPHERE:
                qt = s["geom_quat"][w, ga] / np.linalg.norm(s["geom_quat"][w, ga])
                c = com[w][s["geom_body"][gb]]
                nrm = scenes._quat_to_mat(qt)[:, 2]
                phi = nrm @ (c - s["geom_pos"][w, ga]) - s["geom_size"][w, gb, 0]
                np.testing.assert_allclose(out["dist"][w, k], phi, atol=1e-14)
                np.testing.assert_allclose(n, nrm, atol=1e-15)
            if ta == scenes.SPHERE and tb == scenes.SPHERE:
                ca = com[w][s["geom_body"][ga]] if s["geom_body"][ga] >= 0 else s["geom_pos"][w, ga]
                cb = com[w][s["geom_body"][gb]]
                dd = np.linalg.norm(cb - ca)
                np.testing.assert_allclose(out["dist"][w, k],
                                           dd - s["geom_size"][w, ga, 0] - s["geom_size"][w, gb, 0],
                                           atol=1e-14)
                np.testing.assert_allclose(n, (cb - ca) / dd, atol=1e-14)


def _two_sphere_scene(swap):
    b = scenes._Builder(1)
    r = (0.05, 0.03)
    ids = (1, 0) if swap else (0, 1)
    bodies = [b.body(scenes.JNT_FREE, mass=1.0, inertia=(1e-3,) * 3) for _ in range(2)]
    for i in ids:
        b.geom(scenes.SPHERE, bodies[i], size=(r[i], 0, 0), friction=(0.5, 0, 0))
    s = b.build(gravity=(0, 0, 0))
    s["q0"][0, 0:3] = (0.01, 0.02, 0.03)
    s["q0"][0, 7:10] = (0.07, 0.05, 0.04)
    return s


def test_geometry_pair_swap_and_rigid_motion():
    """Swapping a pair's geom order negates the normal and keeps phi; a rigid
    motion of the whole scene keeps phi."""
    o1, o2 = Oracle(_two_sphere_scene(False)), Oracle(_two_sphere_scene(True))
    s1 = _two_sphere_scene(False)
    _, _, a = o1.step(s1["q0"], s1["v0"])
    _, _, b = o2.step(s1["q0"], s1["v0"])
    assert a["ncon"][0] == b["ncon"][0] == 1
    np.testing.assert_allclose(a["dist"][0, 0], b["dist"][0, 0], rtol=1e-15)
    np.testing.assert_allclose(a["frame"][0, 0, :3], -b["frame"][0, 0, :3], atol=1e-15)
    # rigid motion of the mixed scene (planes, static sphere and bodies)
    s = scenes.mixed_shapes(nworld=1, seed=5)
    s["q0"].reshape(-1, 7)[:, 2] -= 0.03  # press every body into the ground
    _, _, base = Oracle(s).step(s["q0"], s["v0"])
    ang = 0.7
    Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0],
                   [0, 0, 1]])
    qz = np.array([math.cos(ang / 2), 0, 0, math.sin(ang / 2)])
    t = np.array([0.3, -0.2, 0.1])
    s2 = dict(s)
    s2["geom_pos"] = s["geom_pos"].copy()
    s2["geom_quat"] = s["geom_quat"].copy()
    for g in range(s["ngeom"]):
        if s["geom_body"][g] < 0:
            s2["geom_pos"][0, g] = Rz @ s["geom_pos"][0, g] + t
            s2["geom_quat"][0, g] = qmul(qz, s["geom_quat"][0, g])
    q = s["q0"].astype(float).reshape(-1, 7).copy()
    for i in range(q.shape[0]):
        q[i, :3] = Rz @ q[i, :3] + t
        q[i, 3:] = qmul(qz, q[i, 3:])
    _, _, moved = Oracle(s2).step(q.reshape(1, -1), s["v0"])
    n = base["ncon"][0]
    assert moved["ncon"][0] == n and n > 0
    np.testing.assert_array_equal(moved["geom"][0, :n], base["geom"][0, :n])
    np.testing.assert_allclose(moved["dist"][0, :n], base["dist"][0, :n], atol=1e-13)


def test_box_and_capsule_contact_counts():
    b = scenes._Builder(1)
    b.geom(scenes.PLANE)
    bx = b.body(scenes.JNT_FREE, mass=1.0, inertia=(1e-3,) * 3)
    b.geom(scenes.BOX, bx, size=(0.05, 0.04, 0.03))
    cp = b.body(scenes.JNT_FREE, mass=1.0, inertia=(1e-3,) * 3)
    b.geom(scenes.CAPSULE, cp, size=(0.02, 0.06, 0))
    s = b.build()
    s["q0"][0, 0:7] = (0, 0, 0.0299, 1, 0, 0, 0)
    # capsule lying along x (rotate z-axis onto x), then standing
    c = math.cos(math.pi / 4)
    s["q0"][0, 7:14] = (0.5, 0, 0.0199, c, 0, c, 0)
    _, _, out = Oracle(s).step(s["q0"], s["v0"])
    assert out["ncon"][0] == 6
    assert list(out["sub"][0, :6]) == [0, 1, 2, 3, 0, 1]
    assert list(out["geom"][0, :6, 1]) == [1, 1, 1, 1, 2, 2]
    # standing capsule: only the minus end touches
    s["q0"][0, 7:14] = (0.5, 0, 0.0799, 1, 0, 0, 0)
    _, _, out = Oracle(s).step(s["q0"], s["v0"])
    assert out["ncon"][0] == 5 and out["sub"][0, 4] == 0
    np.testing.assert_allclose(out["dist"][0, 4], 0.0799 - 0.06 - 0.02, atol=1e-7)


def test_contact_order_and_overflow_truncation():
    """Contacts come in pair order then sub-index; beyond ncon_max they are
    dropped (not resolved) and counted."""
    s = scenes.boxes_drop()
    s["q0"][0, 2::7] = 0.0  # sink every box: all 8 corners of boxes that are deep enough
    full = scenes.with_params(s, ncon_max=64)
    _, _, a = Oracle(full).step(full["q0"], full["v0"])
    n = a["ncon"][0]
    keys = [(min(g), max(g), sb) for g, sb in zip(a["geom"][0, :n], a["sub"][0, :n])]
    assert keys == sorted(keys) and n > 12
    cut = scenes.with_params(s, ncon_max=12)
    _, vcut, b = Oracle(cut).step(cut["q0"], cut["v0"])
    assert b["ncon"][0] == 12 and b["overflow"][0] == n - 12
    np.testing.assert_array_equal(b["geom"][0, :12], a["geom"][0, :12])
    np.testing.assert_array_equal(b["impulse"][0, :12], a["impulse"][0, :12])


def test_invalid_descriptors_rejected():
    s = scenes.sphere_on_plane()
    for key, val in (("condim", 2), ("h", 0.0), ("k_user", -1.0)):
        bad = dict(s)
        bad[key] = val
        with pytest.raises(OracleError):
            Oracle(bad)
    bad = dict(s)
    bad["solimp"] = np.array([0.95, 0.9, 0.001, 0.5, 2.0])
    with pytest.raises(OracleError):
        Oracle(bad)


# ---------------------------------------------------------------- exact diagonal impedance
def test_exact_impedance_normal_row_single_facet():
    """Exact diagonal impedance (Sec. III.B, K h + D = (1/h)(J~ M^-1 J~^T)^-1 per
    facet): a frictionless sphere on a plane with one facet (condim 1) has
    J~ M^-1 J~^T = 1/m (the row passes through the centre), so an active
    contact leaves the normal velocity at exactly -k phi / (k h + d), whatever
    the incoming velocity."""
    for vz in (-0.3, -0.01, 0.0, 0.002):
        s = scenes.sphere_on_plane(radius=0.05, mass=0.7, mu=(0.0, 0.0, 0.0), condim=1)
        s["impedance"] = 1
        q = s["q0"].astype(np.float64).copy()
        v = s["v0"].astype(np.float64).copy()
        depth = 0.002
        q[0, 2] = 0.05 - depth
        v[0, 2] = vz
        v[0, 3:6] = (1.0, -2.0, 0.5)  # spin does not enter the normal row
        o = Oracle(s)
        q1, v1, out = o.step(q, v)
        a = s["k_user"] * s["h"] + s["d_user"]
        phi = float(out["dist"][0, 0])
        np.testing.assert_allclose(phi, q[0, 2] - float(s["geom_size"][0, 1, 0]), rtol=1e-12)
        np.testing.assert_allclose(v1[0, 2], -s["k_user"] * phi / a, rtol=1e-12)
        np.testing.assert_allclose(v1[0, 3:6], v[0, 3:6], rtol=1e-12)


def test_exact_impedance_stick_decay_point_mass():
    """Point mass on three slide joints, four tangential facets of rows n -/+ mu t:
    each has J~ M^-1 J~^T = (1 + mu^2)/m, so with every facet active the
    tangential velocity contracts by exactly (1 - mu^2)/(1 + mu^2) per step,
    independent of k_user and d_user and of the sliding direction."""
    mu = 0.5
    for k, d in ((0.1, 0.001), (0.5, 0.005)):
        for ang in (0.0, 0.7):
            s = scenes.point_mass(mu=mu, k_user=k, d_user=d)
            s["impedance"] = 1
            q = s["q0"].astype(np.float64).copy()
            v = s["v0"].astype(np.float64).copy()
            q[0, 2] = s["geom_size"][0, 1, 0] - 0.003
            u0 = 0.01
            v[0, 0:2] = (u0 * math.cos(ang), u0 * math.sin(ang))
            o = Oracle(s)
            _, v1, out = o.step(q, v)
            assert (out["impulse"][0, 0] > 0).all()
            mu32 = float(s["geom_friction"][0, 1, 0])
            fac = (1 - mu32 ** 2) / (1 + mu32 ** 2)
            np.testing.assert_allclose(v1[0, 0:2], fac * v[0, 0:2], rtol=1e-11, atol=1e-16)


def test_exact_impedance_hinge_bob_closed_form():
    """One hinge (axis a through o) holding a sphere bob on the ground: the
    generalized mass is I_o = I_yy + m L^2 (parallel axes) and a facet row
    with linear direction u at the contact point p acts on the hinge rate as
    u . (a x (p - o)), so J~ M^-1 J~^T = (u . (a x (p - o)))^2 / I_o for the
    normal row (condim 1) and for the four rows n -/+ mu d (condim 3); the
    gains and impulses follow Sec. III.B with s read from the smooth rate."""
    for condim in (1, 3):
        s = scenes.hinge_bob_on_plane(condim=condim)
        s["impedance"] = 1
        o = Oracle(s)
        _, _, out = o.step(s["q0"].astype(np.float64), s["v0"].astype(np.float64))
        assert out["ncon"][0] == 1
        L, m = -float(s["body_ipos"][0, 2]), float(s["body_mass"][0, 0])  # the model's float32 values
        i_o = float(s["body_inertia"][0, 0, 1]) + m * L * L
        a = np.array([0.0, 1.0, 0.0])
        org = s["body_pos"][0].astype(np.float64)
        p = out["pos"][0, 0]
        n, t1, t2 = out["frame"][0, 0, 0:3], out["frame"][0, 0, 3:6], out["frame"][0, 0, 6:9]
        np.testing.assert_allclose(n, (0, 0, 1), atol=1e-12)
        arm = np.cross(a, p - org)
        assert abs(arm @ n) > 0.05  # the bob sits off the vertical: the normal row is not degenerate
        mu = float(s["geom_friction"][0, 1, 0])
        rows = [n] if condim == 1 else [n - mu * d for d in (t1, t2, -t1, -t2)]
        aa = s["k_user"] * s["h"] + s["d_user"]
        phi = float(out["dist"][0, 0])
        th_s = float(out["v_smooth"][0, 0])
        for f, u in enumerate(rows):
            jrow = float(u @ arm)
            gain = 1.0 / (aa * jrow * jrow / i_o)
            np.testing.assert_allclose(out["facet_gain"][0, 0, f], gain, rtol=1e-10)
            lam = gain * max(-aa * jrow * th_s - s["k_user"] * phi, 0.0)
            np.testing.assert_allclose(out["impulse"][0, 0, f], lam, rtol=1e-10, atol=1e-18)


def test_exact_impedance_siblings_of_one_subtree():
    """Two sibling slide bodies (along y) on a carrier sliding along x, their
    spheres touching along x: the carrier's motion moves both alike, so the
    contact's rows see only the siblings' own rates and J~ M^-1 J~^T =
    mu^2 (d . y)^2 (1/m_1 + 1/m_2) for the row n - mu d (with M = diag(m_0 +
    m_1 + m_2, m_1, m_2)), not the sum of the two bodies' separate forms,
    which would add 2 / (m_0 + m_1 + m_2) from the shared carrier dof.  A row
    with d . y = 0 moves nothing and gets no gain."""
    s = scenes.sibling_sliders(condim=3)
    s["impedance"] = 1
    o = Oracle(s)
    _, _, out = o.step(s["q0"].astype(np.float64), s["v0"].astype(np.float64))
    assert out["ncon"][0] == 1
    m1, m2 = (float(x) for x in s["body_mass"][0, 1:3])
    ga, gb = out["geom"][0, 0]
    n, t1, t2 = out["frame"][0, 0, 0:3], out["frame"][0, 0, 3:6], out["frame"][0, 0, 6:9]
    assert abs(abs(n[0]) - 1.0) < 1e-12
    vs = out["v_smooth"][0]
    rate = {0: vs[1], 1: vs[2]}  # each sphere's body: its y slide rate
    vrel_y = rate[gb] - rate[ga]
    mu = float(s["geom_friction"][0, 0, 0])
    aa = s["k_user"] * s["h"] + s["d_user"]
    phi = float(out["dist"][0, 0])
    seen = 0
    for f, d in enumerate((t1, t2, -t1, -t2)):
        g = mu * mu * d[1] * d[1] * (1 / m1 + 1 / m2)
        if g < 1e-20:
            assert out["facet_gain"][0, 0, f] == 0 and out["impulse"][0, 0, f] == 0
            continue
        seen += 1
        np.testing.assert_allclose(out["facet_gain"][0, 0, f], 1.0 / (aa * g), rtol=1e-10)
        sf = -mu * d[1] * vrel_y
        lam = max(-aa * sf - s["k_user"] * phi, 0.0) / (aa * g)
        np.testing.assert_allclose(out["impulse"][0, 0, f], lam, rtol=1e-10, atol=1e-18)
    assert seen == 2


def test_exact_impedance_sphere_tangential_row():
    """Free solid sphere on a plane (I = 0.4 m R^2): a tangential facet row
    (n - mu d.t at the contact point, the middle of the overlap, lever arm
    -(R + phi/2) n) gives J~ M^-1 J~^T = (1 + mu^2)/m + mu^2 (R + phi/2)^2 / I
    (= (1 + 3.5 mu^2)/m at phi = 0), so each facet impulse is
    max(-(k h + d) s - k phi, 0) / ((k h + d) J~ M^-1 J~^T); s is read from the
    smooth velocity in the contact's own frame."""
    s = scenes.sphere_on_plane(radius=0.04, mass=0.3, mu=(0.6, 0.0, 0.0), condim=3)
    s["impedance"] = 1
    q = s["q0"].astype(np.float64).copy()
    v = s["v0"].astype(np.float64).copy()
    q[0, 2] = 0.04 - 0.001
    v[0, 0:6] = (0.02, -0.01, -0.05, 0.3, 0.2, -1.0)
    o = Oracle(s)
    _, _, out = o.step(q, v)
    m, R = float(s["body_mass"][0, 0]), float(s["geom_size"][0, 1, 0])
    inertia = float(s["body_inertia"][0, 0, 0])
    mu = float(s["geom_friction"][0, 1, 0])
    np.testing.assert_allclose((1 + mu * mu) / m + mu * mu * R * R / inertia, (1 + 3.5 * mu * mu) / m,
                               rtol=1e-6)
    phi = float(out["dist"][0, 0])
    arm = R + 0.5 * phi
    g = (1 + mu * mu) / m + mu * mu * arm * arm / inertia
    vs = out["v_smooth"][0]
    n, t1, t2 = out["frame"][0, 0, 0:3], out["frame"][0, 0, 3:6], out["frame"][0, 0, 6:9]
    r = -arm * n
    vp = vs[0:3] + np.cross(vs[3:6], r)  # contact point velocity, plane static
    a = s["k_user"] * s["h"] + s["d_user"]
    for f, (d1, d2) in enumerate(((1, 0), (0, 1), (-1, 0), (0, -1))):
        sf = n @ vp - mu * (d1 * (t1 @ vp) + d2 * (t2 @ vp))
        lam = max(-a * sf - s["k_user"] * phi, 0.0) / (a * g)
        np.testing.assert_allclose(out["impulse"][0, 0, f], lam, rtol=1e-10)
