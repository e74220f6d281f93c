"""GPU kernels of the learned impedance network (bf16 MFMA, float32
accumulation) against the FP64 reference in oracle/mlp.py.

Tolerance: inputs, weights and activations are rounded to bf16 (relative
2^-9) before each of the three products, so an output may differ from the
float64 value by a few times 2^-9 of the magnitudes that enter it; the tests
allow 3 % of the largest |y| (forward) and 5 % of the gradient's norm.
"""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_12185_amd import cfsim
    cfsim.load()
    return torch


def _data(n, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((n, 8), np.float32)
    f[:, 0] = rng.normal(-1e-3, 1.5e-3, n)
    f[:, 1] = rng.normal(0, 0.05, n)
    f[:, 2] = rng.normal(0, 0.1, n)
    f[:, 3] = rng.normal(0, 0.1, n)
    f[:, 4] = rng.uniform(0.01, 0.5, n)
    f[:, 5] = rng.uniform(0.3, 1.0, n)
    f[:, 6] = 0.002
    f[:, 7] = rng.normal(size=n)  # ignored by the network
    return f


def _params(f, seed):
    p = mlp.init_params(f, seed=seed)
    rng = np.random.default_rng(seed + 100)
    p[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0, 0.3, mlp.NH)
    p[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(0, 0.3, mlp.NH)
    p[mlp.OFF_B3:] = rng.normal(0, 0.3, mlp.NOUT)
    return p.astype(np.float32)


@pytest.mark.parametrize("n", [1, 17, 1003, 100003])
def test_forward_matches_reference(torch_cuda, n):
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    f = _data(n, n)
    p = _params(f, 1)
    net = cfsim.ImpedanceNet(p)
    y = net.forward(torch.from_numpy(f).cuda()).cpu().numpy()
    ref, _ = mlp.forward(p.astype(np.float64), f.astype(np.float64))
    err = np.abs(y - ref).max()
    print(f"n {n}: max |dy| {err:.3e}, max |y| {np.abs(ref).max():.3f}")
    assert err <= 0.03 * np.abs(ref).max() + 1e-3


@pytest.mark.parametrize("nout", [1, 4, 10])
def test_gradient_matches_reference(torch_cuda, nout):
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    n = 5003
    f = _data(n, 7 + nout)
    p = _params(f, 2)
    t = np.random.default_rng(nout).normal(0, 1, (n, 16)).astype(np.float32)
    net = cfsim.ImpedanceNet(p)
    fd, td = torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda()
    g, loss = net.gradient(fd, td, nout)
    g2, _ = net.gradient(fd, td, nout)
    g, g2 = g.cpu().numpy(), g2.cpu().numpy()
    assert np.array_equal(g, g2), "gradient is not deterministic"
    lref, gref = mlp.loss_and_grad(p.astype(np.float64), f.astype(np.float64), t.astype(np.float64), nout)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    cos = g @ gref / (np.linalg.norm(g) * np.linalg.norm(gref))
    print(f"nout {nout}: loss {float(loss.item()):.6f} vs {lref:.6f}; grad rel {rel:.3e} cos {cos:.6f}")
    assert abs(float(loss.item()) - lref) <= 0.03 * lref
    assert rel <= 0.05 and cos >= 0.998
    for lo, hi in ((mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_W2, mlp.OFF_B2), (mlp.OFF_W3, mlp.OFF_B3)):
        rb = np.linalg.norm(g[lo:hi] - gref[lo:hi]) / np.linalg.norm(gref[lo:hi])
        assert rb <= 0.05, (lo, rb)
    assert not g[:mlp.TRAIN_FROM].any()


def test_training_fits_a_smooth_target(torch_cuda):
    """Adam on the GPU fits a smooth function of the features: the loss falls
    below a tenth of its starting value, and one GPU Adam step equals the
    reference update applied to the GPU gradient."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    n = 20000
    f = _data(n, 3)
    x = (f[:, :7] - f[:, :7].mean(0)) / (f[:, :7].std(0) + 1e-12)
    t = np.zeros((n, 16), np.float32)
    t[:, 0] = np.tanh(x[:, 0] - 0.5 * x[:, 1])
    t[:, 1] = 0.5 * x[:, 2] * x[:, 5]
    t[:, 2] = np.sin(x[:, 4])
    t[:, 3] = x[:, 3] ** 2 / 3
    p = mlp.init_params(f, seed=5).astype(np.float32)
    net = cfsim.ImpedanceNet(p)
    fd, td = torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda()
    g, _ = net.gradient(fd, td, 4)
    p0 = net.params.cpu().numpy().astype(np.float64)
    net.train_step(fd, td, 4, 1e-3)
    p1 = net.params.cpu().numpy()
    pref, _, _ = mlp.adam(p0, np.zeros_like(p0), np.zeros_like(p0), g.cpu().numpy().astype(np.float64), 1, 1e-3)
    np.testing.assert_allclose(p1, pref, rtol=0, atol=2e-6)
    first = None
    for it in range(600):
        loss = net.train_step(fd, td, 4, 3e-3)
        if first is None:
            first = float(loss.item())
    last = float(net.gradient(fd, td, 4)[1].item())
    print(f"loss {first:.4f} -> {last:.4f}")
    assert last < 0.1 * first
