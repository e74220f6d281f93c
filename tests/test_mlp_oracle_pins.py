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


def test_forward_of_a_hand_worked_network():
    """A network with three active hidden units, worked out by hand from the
    stated definition (normalise, two SiLU layers, linear output; weights
    W[in][out]): pins the normalisation, SiLU after each hidden layer and not
    after the output, the layout of every weight matrix and bias, and that the
    eighth (padding) feature is ignored."""
    import math
    sig = lambda z: 1.0 / (1.0 + math.exp(-z))
    silu = lambda z: z * sig(z)
    mean = [-2e-3, 0.01, -0.02, 0.03, 0.2, 0.6, 0.002, 0.0]
    std = [1e-3, 0.05, 0.1, 0.2, 0.1, 0.25, 1.0, 1.0]
    p = np.zeros(mlp.NPARAM)
    p[mlp.OFF_MEAN:mlp.OFF_STD] = mean
    p[mlp.OFF_STD:mlp.OFF_W1] = std
    W1 = np.zeros((mlp.NIN, mlp.NH))
    W1[0, 3], W1[4, 3], W1[2, 9] = 0.7, -1.2, 0.5
    b1 = np.zeros(mlp.NH)
    b1[3], b1[9] = 0.1, -0.3
    W2 = np.zeros((mlp.NH, mlp.NH))
    W2[3, 5], W2[9, 5], W2[9, 60] = 1.5, -0.8, 2.0
    b2 = np.zeros(mlp.NH)
    b2[5], b2[60] = 0.05, -0.2
    W3 = np.zeros((mlp.NH, mlp.NOUT))
    W3[5, 0], W3[60, 0], W3[60, 3] = 0.9, -0.4, 1.1
    b3 = 0.01 * np.arange(mlp.NOUT)
    b3[0], b3[3] = 0.2, -0.1
    p[mlp.OFF_W1:mlp.OFF_B1] = W1.ravel()
    p[mlp.OFF_B1:mlp.OFF_W2] = b1
    p[mlp.OFF_W2:mlp.OFF_B2] = W2.ravel()
    p[mlp.OFF_B2:mlp.OFF_W3] = b2
    p[mlp.OFF_W3:mlp.OFF_B3] = W3.ravel()
    p[mlp.OFF_B3:] = b3
    feats = np.array([[-3.5e-3, 0.04, 0.13, -0.05, 0.31, 0.45, 0.002, 7.0],
                      [1.0e-3, -0.02, -0.27, 0.11, 0.05, 0.95, 0.002, -3.0]])
    y, _ = mlp.forward(p, feats)
    for r, f in enumerate(feats):
        x0 = (f[0] - mean[0]) / std[0]
        x2 = (f[2] - mean[2]) / std[2]
        x4 = (f[4] - mean[4]) / std[4]
        a13 = silu(0.7 * x0 - 1.2 * x4 + 0.1)
        a19 = silu(0.5 * x2 - 0.3)
        a25 = silu(1.5 * a13 - 0.8 * a19 + 0.05)
        a260 = silu(2.0 * a19 - 0.2)
        expect = 0.01 * np.arange(mlp.NOUT)
        expect[0] = 0.9 * a25 - 0.4 * a260 + 0.2
        expect[3] = 1.1 * a260 - 0.1
        np.testing.assert_allclose(y[r], expect, rtol=1e-14, atol=1e-15)
    # every hidden unit without weights sits at silu(0) = 0: a bias on an
    # unused first-layer unit does not reach the output
    p2 = p.copy()
    p2[mlp.OFF_B1 + 20] = 3.0
    np.testing.assert_array_equal(mlp.forward(p2, feats)[0], y)


def test_bf16_rounding_and_ties():
    """bf16 keeps 8 significant bits, rounding to nearest with ties to even:
    1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and goes to 1; 1 + 3 2^-8
    halfway between 1 + 2^-7 and 1 + 2^-6 goes to 1 + 2^-6; pi -> 3.140625;
    signs are symmetric; tie distance and spacing follow the grid, 2^-7 above
    1 and 2^-8 below it."""
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, np.pi, -np.pi, 0.0])
    np.testing.assert_array_equal(mlp.bf16(vals),
                                  [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, 3.140625, -3.140625, 0.0])
    np.testing.assert_allclose(mlp.bf16_tie_distance([1 + 2 ** -9, 1.0, 1 - 2 ** -10]),
                               [2 ** -9, 2 ** -9, 2 ** -10], rtol=1e-12)
    np.testing.assert_array_equal(mlp.bf16_spacing([1.5, 0.75]), [2 ** -7, 2 ** -8])


def test_bf16_operand_forward():
    """At bf16 operand precision the network rounds x, the weights and both
    hidden activations before each product (biases as given, float64 sums):
    a one-unit chain worked out with those roundings."""
    import math
    p = np.zeros(mlp.NPARAM)
    p[mlp.OFF_STD:mlp.OFF_W1] = 1.0
    p[mlp.OFF_STD] = 3.0
    p[mlp.OFF_W1 + 0 * mlp.NH + 2] = 0.3            # W1[0][2]
    p[mlp.OFF_B1 + 2] = 0.01
    p[mlp.OFF_W2 + 2 * mlp.NH + 7] = -1.7           # W2[2][7]
    p[mlp.OFF_W3 + 7 * mlp.NOUT + 1] = 0.9          # W3[7][1]
    p[mlp.OFF_B3 + 1] = 0.1
    f = np.array([[0.7, 0, 0, 0, 0, 0, 0, 0]])
    y, it = mlp.forward(p, f, operands="bf16")
    b = lambda x: float(mlp.bf16(np.array([x]))[0])
    silu = lambda z: z / (1 + math.exp(-z))
    x0 = b(0.7 / 3.0)
    a1 = b(silu(b(0.3) * x0 + 0.01))
    a2 = b(silu(b(-1.7) * a1))
    np.testing.assert_allclose(y[0, 1], b(0.9) * a2 + 0.1, rtol=1e-15)
    assert y[0, 0] == 0.0
    np.testing.assert_allclose(it["x_pre"][0, 0], 0.7 / 3.0, rtol=1e-15)
    # float64 operands: the same chain without roundings
    y64, _ = mlp.forward(p, f)
    np.testing.assert_allclose(y64[0, 1], 0.9 * silu(-1.7 * silu(0.3 * 0.7 / 3 + 0.01)) + 0.1, rtol=1e-14)
