"""Pins of the FP64 reference of the learned impedance network (oracle/mlp.py):
central differences of the loss (brute force), the closed-form SiLU
derivative, a network with zero weights, and the first Adam step."""
import numpy as np

from oracle import mlp


def _data(n=37, seed=0):
    rng = np.random.default_rng(seed)
    f = np.stack([rng.normal(-1e-3, 1e-3, n), rng.normal(0, 0.05, n), rng.normal(0, 0.1, n),
                  rng.normal(0, 0.1, n), rng.uniform(0.01, 0.5, n), rng.uniform(0.3, 1.0, n),
                  np.full(n, 0.002)], 1)
    t = rng.normal(0, 1, (n, mlp.NOUT))
    return f, t


def test_loss_gradient_matches_central_differences():
    f, t = _data()
    p = mlp.init_params(f, seed=3)
    p[mlp.OFF_B1:mlp.OFF_W2] = np.random.default_rng(4).normal(0, 0.3, mlp.NH)
    for nout in (1, 4, 10):
        loss, g = mlp.loss_and_grad(p, f, t, nout)
        rng = np.random.default_rng(nout)
        idx = np.concatenate([rng.choice(np.arange(mlp.OFF_W1, mlp.NPARAM), 60, replace=False),
                              [mlp.OFF_B3, mlp.OFF_B3 + nout - 1, mlp.OFF_B1, mlp.OFF_W1]])
        eps = 1e-6
        for i in idx:
            pp, pm = p.copy(), p.copy()
            pp[i] += eps
            pm[i] -= eps
            fd = (mlp.loss_and_grad(pp, f, t, nout)[0] - mlp.loss_and_grad(pm, f, t, nout)[0]) / (2 * eps)
            assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (nout, i, fd, g[i])
        # outputs beyond nout and the normalisation get no gradient
        assert not g[:mlp.TRAIN_FROM].any()
        assert not g[mlp.OFF_B3 + nout:].any()


def test_silu_derivative_closed_form():
    z = np.linspace(-8, 8, 101)
    eps = 1e-6
    fd = (mlp.silu(z + eps) - mlp.silu(z - eps)) / (2 * eps)
    np.testing.assert_allclose(mlp.dsilu(z), fd, rtol=1e-7, atol=1e-10)
    assert mlp.silu(0.0) == 0.0
    np.testing.assert_allclose(mlp.silu(40.0), 40.0, rtol=1e-15)


def test_zero_weights_network_outputs_its_bias():
    f, t = _data(n=11)
    p = np.zeros(mlp.NPARAM)
    p[mlp.OFF_STD:mlp.OFF_W1] = 1.0
    p[mlp.OFF_B3:] = np.arange(mlp.NOUT) * 0.1
    y, _ = mlp.forward(p, f)
    np.testing.assert_array_equal(y, np.tile(p[mlp.OFF_B3:], (11, 1)))
    # d loss / d b3 = 2 (b3 - mean_n t) / nout for the used outputs
    _, g = mlp.loss_and_grad(p, f, t, 4)
    np.testing.assert_allclose(g[mlp.OFF_B3:mlp.OFF_B3 + 4], 2 * (p[mlp.OFF_B3:mlp.OFF_B3 + 4] - t[:, :4].mean(0)) / 4,
                               rtol=1e-12)


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(1)
    p = rng.normal(size=mlp.NPARAM)
    g = rng.normal(size=mlp.NPARAM)
    m = np.zeros(mlp.NPARAM)
    v = np.zeros(mlp.NPARAM)
    p1, m1, v1 = mlp.adam(p, m, v, g, 1, 1e-3)
    s = slice(mlp.TRAIN_FROM, mlp.NPARAM)
    np.testing.assert_allclose(p1[s] - p[s], -1e-3 * g[s] / (np.abs(g[s]) + 1e-8), rtol=1e-12)
    np.testing.assert_array_equal(p1[:mlp.TRAIN_FROM], p[:mlp.TRAIN_FROM])
