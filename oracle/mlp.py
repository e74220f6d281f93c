"""FP64 reference of the learned per-contact impedance network.

TEST INFRASTRUCTURE ONLY: the GPU library has its own kernels; only tests/,
the smoke check and bench.py's CPU baseline use this module.

The paper lets K and D be learned (Sec. III.B: the impedance may be
parameterised by a network instead of the heuristic of Eq. k_d_setting); it
gives no network.  This one follows the design recorded for the build:

  features of a contact (7): phi, v_n, u_1, u_2, m_eff, mu_t, h
      phi: gap; v_n, (u_1, u_2): normal and tangential (t1, t2) relative
      velocity at v_s; m_eff = 1 / (tr_a + tr_b); mu_t pair friction; h step
  normalised x_k = (f_k - mean_k) / std_k (fixed, from the training data)
  z1 = W1^T x + b1 (64), a1 = silu(z1); z2 = W2^T a1 + b2 (64), a2 = silu(z2)
  y = W3^T a2 + b3 (one output per facet of the contact)
  facet impulse gain A_f = A_heuristic * exp(clip(y_f, -L, L))

Parameters, flat float array (the GPU layout, row-major):
  mean[8], std[8] (feature 8 is padding), W1[8][64], b1[64], W2[64][64],
  b2[64], W3[64][16], b3[16] (outputs beyond the facet count unused).
Training: mean squared error between y and the clipped log target, averaged
over contacts and used outputs; Adam.
"""
from __future__ import annotations

import numpy as np

NFEAT, NIN, NH, NOUT = 7, 8, 64, 16
CLIP = float(np.log(256.0))

# offsets in the flat parameter array
OFF_MEAN = 0
OFF_STD = OFF_MEAN + NIN
OFF_W1 = OFF_STD + NIN
OFF_B1 = OFF_W1 + NIN * NH
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH * NOUT
NPARAM = OFF_B3 + NOUT
TRAIN_FROM = OFF_W1  # mean and std are not trained


def unpack(p):
    p = np.asarray(p, np.float64)
    return dict(mean=p[OFF_MEAN:OFF_STD], std=p[OFF_STD:OFF_W1],
                W1=p[OFF_W1:OFF_B1].reshape(NIN, NH), b1=p[OFF_B1:OFF_W2],
                W2=p[OFF_W2:OFF_B2].reshape(NH, NH), b2=p[OFF_B2:OFF_W3],
                W3=p[OFF_W3:OFF_B3].reshape(NH, NOUT), b3=p[OFF_B3:NPARAM])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(feats, seed=0):
    """Feature normalisation from data; Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    f = np.asarray(feats, np.float64)[:, :NFEAT]
    mean = np.zeros(NIN)
    std = np.ones(NIN)
    mean[:NFEAT] = f.mean(0)
    sd = f.std(0)
    std[:NFEAT] = np.where(sd > 1e-12, sd, 1.0)
    p[OFF_MEAN:OFF_STD] = mean
    p[OFF_STD:OFF_W1] = std

    def glorot(a, b):
        r = np.sqrt(6.0 / (a + b))
        return rng.uniform(-r, r, (a, b))

    p[OFF_W1:OFF_B1] = glorot(NIN, NH).ravel()
    p[OFF_W2:OFF_B2] = glorot(NH, NH).ravel()
    p[OFF_W3:OFF_B3] = glorot(NH, NOUT).ravel()
    return p


def bf16(a):
    """Round to bfloat16 (round to nearest, ties to even) through float32, the
    way a float32 operand is narrowed for a bf16 matrix product; returned as
    float64 values."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_neighbours(r):
    """The bf16 values next to |r| above and below (|r| itself a bf16 value;
    for 0 both are the smallest positive bf16 value)."""
    bits = np.abs(r).astype(np.float32).view(np.uint32).astype(np.int64)
    up = (bits + 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    dn = np.where(bits > 0, bits - 0x10000, bits + 0x10000).astype(np.uint32).view(np.float32)
    return up, dn.astype(np.float64)


def bf16_tie_distance(a):
    """Distance of each value to the nearest point where its bf16 rounding
    changes (the midpoints to the neighbouring bf16 values)."""
    a = np.abs(np.asarray(a, np.float64))
    r = bf16(a)
    up, dn = _bf16_neighbours(r)
    return np.minimum(np.abs(a - 0.5 * (r + up)), np.abs(a - 0.5 * (r + dn)))


def bf16_spacing(a):
    """Larger of the gaps from bf16(a) to its two neighbouring bf16 values."""
    r = np.abs(bf16(a))
    up, dn = _bf16_neighbours(r)
    return np.maximum(up - r, np.abs(r - dn))


def forward(p, feats, operands=None):
    """Outputs y [n][16] and the intermediates.

    operands="bf16" evaluates the same network at the precision of a bf16
    matrix unit: the normalised inputs, the weights and the two hidden
    activations are rounded to bf16 before each product, products and sums
    stay in float64, biases are not rounded.  The intermediates then also hold
    the values before each rounding (x_pre, a1_pre, a2_pre)."""
    P = unpack(p)
    f = np.zeros((len(feats), NIN))
    f[:, :NFEAT] = np.asarray(feats, np.float64)[:, :NFEAT]
    x = (f - P["mean"]) / P["std"]
    if operands is None:
        z1 = x @ P["W1"] + P["b1"]
        a1 = silu(z1)
        z2 = a1 @ P["W2"] + P["b2"]
        a2 = silu(z2)
        y = a2 @ P["W3"] + P["b3"]
        return y, dict(x=x, z1=z1, a1=a1, z2=z2, a2=a2)
    if operands != "bf16":
        raise ValueError("operands must be None or 'bf16'")
    xb = bf16(x)
    xb[:, NFEAT:] = 0.0
    z1 = xb @ bf16(P["W1"]) + P["b1"]
    a1 = silu(z1)
    a1b = bf16(a1)
    z2 = a1b @ bf16(P["W2"]) + P["b2"]
    a2 = silu(z2)
    a2b = bf16(a2)
    y = a2b @ bf16(P["W3"]) + P["b3"]
    return y, dict(x=xb, z1=z1, a1=a1b, z2=z2, a2=a2b, x_pre=x, a1_pre=a1, a2_pre=a2)


def loss_and_grad(p, feats, targets, nout):
    """Mean squared error over contacts and the first nout outputs, against
    targets [n][nout] (already clipped); returns (loss, grad [NPARAM])."""
    P = unpack(p)
    y, c = forward(p, feats)
    n = len(feats)
    t = np.asarray(targets, np.float64)[:, :nout]
    r = y[:, :nout] - t
    loss = float((r * r).sum() / (n * nout))
    dy = np.zeros_like(y)
    dy[:, :nout] = 2.0 * r / (n * nout)
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = (c["a2"].T @ dy).ravel()
    g[OFF_B3:NPARAM] = dy.sum(0)
    dz2 = (dy @ P["W3"].T) * dsilu(c["z2"])
    g[OFF_W2:OFF_B2] = (c["a1"].T @ dz2).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(0)
    dz1 = (dz2 @ P["W2"].T) * dsilu(c["z1"])
    g[OFF_W1:OFF_B1] = (c["x"].T @ dz1).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(0)
    return loss, g


def adam(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the trained part (step counts from 1); returns new (p, m, v)."""
    p, m, v = p.copy(), m.copy(), v.copy()
    s = slice(TRAIN_FROM, NPARAM)
    m[s] = beta1 * m[s] + (1 - beta1) * g[s]
    v[s] = beta2 * v[s] + (1 - beta2) * g[s] * g[s]
    mh = m[s] / (1 - beta1 ** step)
    vh = v[s] / (1 - beta2 ** step)
    p[s] = p[s] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def scale(y):
    """Impedance scale exp(clip(y, -L, L))."""
    return np.exp(np.clip(y, -CLIP, CLIP))
