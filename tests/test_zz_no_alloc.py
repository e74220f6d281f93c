"""The network's gradient through the entry point that allocates nothing
(cf_mlp_gradient_noalloc: the per-wave partial sums in the library's fixed
static device array instead of a caller workspace).  It runs the same kernels
over the same per-wave partition as cf_mlp_gradient, so gradient and loss
must equal that entry point's bit for bit.  Two calls in a row, the first at
the largest partition (2048 waves) and the second much smaller, show that what
the first call left in the shared array does not reach the second's result."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((n, 8), np.float32)
    f[:, 0] = rng.normal(-1e-3, 1.5e-3, n)
    f[:, 1:4] = rng.normal(0, 0.1, (n, 3))
    f[:, 4] = rng.uniform(0.01, 0.5, n)
    f[:, 5] = rng.uniform(0.3, 1.0, n)
    f[:, 6] = 0.002
    t = rng.normal(0, 0.5, (n, 16)).astype(np.float32)
    p = mlp.init_params(f, seed=seed).astype(np.float32)
    return f, t, p


def test_noalloc_gradient_equals_workspace_gradient():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_12185_amd import cfsim
    for n, nout, seed in ((70001, 4, 1), (3001, 10, 2)):
        print(f"cf_mlp_gradient_noalloc n={n} nout={nout} seed={seed}", flush=True)
        f, t, p = _inputs(n, seed)
        net = cfsim.ImpedanceNet(p)
        F, T = torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda()
        g_ref, l_ref = net.gradient(F, T, nout)
        g = torch.full_like(g_ref, float("nan"))
        loss = torch.full_like(l_ref, float("nan"))
        net.gradient_noalloc(F, T, nout, g, loss)
        torch.cuda.synchronize()
        assert torch.isfinite(g).all() and torch.isfinite(loss).all()
        assert float(g.abs().max()) > 0
        assert torch.equal(g, g_ref), f"n={n}: max |dg| {float((g - g_ref).abs().max()):.3e}"
        assert torch.equal(loss, l_ref)


def test_noalloc_gradient_rejects_bad_arguments():
    import ctypes as C

    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_12185_amd import cfsim
    L = cfsim.load()
    x = torch.zeros((64, 16), device="cuda")
    g = torch.zeros(int(L.cf_mlp_nparam()), device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = C.c_void_p(x.data_ptr())
    assert L.cf_mlp_gradient_noalloc(s, p, p, p, 0, 4, C.c_void_p(g.data_ptr()), None) == cfsim.CF_E_INVALID_ARG
    assert L.cf_mlp_gradient_noalloc(s, p, p, p, 64, 17, C.c_void_p(g.data_ptr()), None) == cfsim.CF_E_INVALID_ARG
    assert L.cf_mlp_gradient_noalloc(s, p, p, p, 64, 4, None, None) == cfsim.CF_E_INVALID_ARG
