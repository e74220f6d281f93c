"""CPU pins of the finite-difference harness used by the adjoint tests
(tests/adjoint_fd.py): on a free flight the step is affine in (x, v, tau), so
its central differences must equal the closed-form Jacobian; a stencil that
creates a contact must be flagged."""
import numpy as np

from paper_2603_12185_amd import scenes

from adjoint_fd import step_grad_fd


def test_fd_of_free_flight_matches_closed_form():
    s = scenes.sphere_on_plane(radius=0.05, mass=0.7)
    q = s["q0"].astype(np.float64).copy()
    q[0, 2] = 0.5  # far above the plane: no contact
    v = np.array([[0.3, -0.2, 0.1, 1.0, -2.0, 0.5]])
    tau = np.array([[0.1, 0.2, -0.3, 0.001, 0.002, -0.001]])
    rng = np.random.default_rng(0)
    gq_out, gv_out = rng.normal(size=(1, 7)), rng.normal(size=(1, 6))
    g, ok, out = step_grad_fd(s, 0, q, v, tau, gq_out, gv_out)
    assert out["ncon"][0] == 0 and ok.all()
    h, m = s["h"], float(s["body_mass"][0, 0])
    inertia = float(s["body_inertia"][0, 0, 0])
    nq = 7
    gx, gvl, gva = gq_out[0, :3], gv_out[0, :3], gv_out[0, 3:]
    # x+ = x + h v+, v+ = v + h (f/m + g), w+ = w + h T / I (isotropic: no gyroscopic term)
    np.testing.assert_allclose(g[0:3], gx, rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(g[nq:nq + 3], gvl + h * gx, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(g[nq + 6:nq + 9], (h / m) * (gvl + h * gx), rtol=1e-7, atol=1e-10)
    # angular: the quaternion part depends on w+ too, so compare the velocity-only adjoint
    g2, _, _ = step_grad_fd(s, 0, q, v, tau, np.zeros_like(gq_out), gv_out)
    np.testing.assert_allclose(g2[nq + 3:nq + 6], gva, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(g2[nq + 9:nq + 12], (h / inertia) * gva, rtol=1e-7, atol=1e-9)


def test_fd_flags_a_stencil_that_creates_a_contact():
    s = scenes.sphere_on_plane(radius=0.05, mass=1.0)
    q = s["q0"].astype(np.float64).copy()
    q[0, 2] = 0.05 + 4e-7  # 0.4 um above the plane: z - 1e-6 touches it
    v = np.zeros((1, 6))
    g, ok, out = step_grad_fd(s, 0, q, v, None, np.ones((1, 7)), np.ones((1, 6)))
    assert out["ncon"][0] == 0
    assert not ok[2] and ok[0] and ok[1]
