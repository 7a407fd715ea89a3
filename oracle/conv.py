"""3D convolution U-Net for the learned preconditioner (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Not part of the paper:
this is the definition the GPU network's forward and backward kernels are
checked against.

Tensors are channels-last, [Z, Y, X, C], float64.  A 3x3x3 "same" convolution
with zero padding is
    y[v, co] = b[co] + sum_t sum_ci w[t, co, ci] x[v + off_t, ci],
tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) for offsets (dz, dy, dx) in {-1,0,1}^3;
its gradients are
    dx[v, ci]     = sum_t sum_co w[t, co, ci] dy[v - off_t, co],
    dw[t, co, ci] = sum_v dy[v, co] x[v + off_t, ci],   db[co] = sum_v dy[v, co].
Down-sampling is a 2x2x2 average, up-sampling nearest-neighbour x2.

Network (3 levels, 16/32/64 channels):
    e1 = relu(c1b(relu(c1a(x))))                     [N,   16]
    e2 = relu(c2b(relu(c2a(pool(e1)))))              [N/2, 32]
    b3 = relu(c3b(relu(c3a(pool(e2)))))              [N/4, 64]
    d2 = relu(d2b(relu(d2a(concat(up(b3), e2)))))    [N/2, 32]
    d1 = relu(d1b(relu(d1a(concat(up(d2), e1)))))    [N,   16]
    out = p(d1)  (1x1x1 conv 16 -> 2, no activation)
Losses: relative squared error ||out - t||^2 / ||t||^2, its scale- and
phase-invariant form 1 - |<o, t>|^2/(||o||^2 ||t||^2), and the residual loss: with
the network's input v as t, min over a complex d of ||v - d Ahat out||^2 / ||v||^2, the
scaled residual a preconditioner's output leaves (Ahat = A / (s/h^2) without the
damping term, built from the input's third channel).  Optimiser: Adam.

Pins (tests/test_oracle_conv.py): the convolution against a brute-force loop
over every index; the whole forward against the same network built from torch's
CPU primitives; every gradient against central finite differences.
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]

LAYERS = [  # name, cin, cout
    ("c1a", 3, 16), ("c1b", 16, 16),
    ("c2a", 16, 32), ("c2b", 32, 32),
    ("c3a", 32, 64), ("c3b", 64, 64),
    ("d2a", 96, 32), ("d2b", 32, 32),
    ("d1a", 48, 16), ("d1b", 16, 16),
]


def _shift(x, off):
    """x[v + off] with zeros outside (same shape as x)."""
    dz, dy, dx = off
    out = np.zeros_like(x)
    Z, Y, X = x.shape[:3]
    zs, ys, xs = slice(max(0, -dz), Z - max(0, dz)), slice(max(0, -dy), Y - max(0, dy)), \
        slice(max(0, -dx), X - max(0, dx))
    zs2, ys2, xs2 = slice(max(0, dz), Z + min(0, dz)), slice(max(0, dy), Y + min(0, dy)), \
        slice(max(0, dx), X + min(0, dx))
    out[zs, ys, xs] = x[zs2, ys2, xs2]
    return out


def conv3d(x, w, b=None):
    """y[v, co] = b[co] + sum_t x[v + off_t] @ w[t].T ; w: [27, cout, cin]."""
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, off in enumerate(OFFSETS):
        y += _shift(x, off) @ w[t].T
    if b is not None:
        y += b
    return y


def conv3d_dgrad(dy, w):
    """dx[v, ci] = sum_t dy[v - off_t] @ w[t]."""
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, off in enumerate(OFFSETS):
        dx += _shift(dy, tuple(-o for o in off)) @ w[t]
    return dx


def conv3d_wgrad(x, dy):
    """dw[t, co, ci] = sum_v dy[v, co] x[v + off_t, ci]; db = sum_v dy."""
    cin, cout = x.shape[3], dy.shape[3]
    dw = np.zeros((27, cout, cin))
    dyf = dy.reshape(-1, cout)
    for t, off in enumerate(OFFSETS):
        dw[t] = dyf.T @ _shift(x, off).reshape(-1, cin)
    return dw, dyf.sum(axis=0)


def pool(x):
    Z, Y, X, C = x.shape
    return x.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).mean(axis=(1, 3, 5))


def pool_back(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_back(dy):
    Z, Y, X, C = dy.shape
    return dy.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).sum(axis=(1, 3, 5))


def init_params(seed: int = 0):
    """He-normal 3x3x3 kernels, zero biases, small pointwise head."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, cin, cout in LAYERS:
        p[name + ".w"] = rng.standard_normal((27, cout, cin)) * np.sqrt(2.0 / (27 * cin))
        p[name + ".b"] = np.zeros(cout)
    p["out.w"] = rng.standard_normal((2, 16)) * 0.1
    p["out.b"] = np.zeros(2)
    return p


def forward(p, x, q=None):
    """Returns (out, cache) for input x [N, N, N, 3].

    q, if given, is applied to every stored intermediate (a storage-precision
    model, e.g. rounding to bfloat16); the arithmetic itself stays float64.
    """
    q = q or (lambda a: a)
    c = {}

    def cr(name, h):
        z = conv3d(h, p[name + ".w"], p[name + ".b"])
        c[name + ".in"] = h
        c[name + ".pre"] = z
        return q(np.maximum(z, 0.0))

    e1 = cr("c1b", cr("c1a", x))
    e2 = cr("c2b", cr("c2a", q(pool(e1))))
    b3 = cr("c3b", cr("c3a", q(pool(e2))))
    d2 = cr("d2b", cr("d2a", np.concatenate([up(b3), e2], axis=3)))
    d1 = cr("d1b", cr("d1a", np.concatenate([up(d2), e1], axis=3)))
    c["d1"] = d1
    out = d1 @ p["out.w"].T + p["out.b"]
    return out, c


def backward(p, c, dout, q=None):
    """Gradients of every parameter and of the input, given dL/dout (q as in forward)."""
    q = q or (lambda a: a)
    g = {}
    d1 = c["d1"]
    g["out.w"] = dout.reshape(-1, 2).T @ d1.reshape(-1, 16)
    g["out.b"] = dout.reshape(-1, 2).sum(axis=0)
    dh = q(dout @ p["out.w"])

    def cr_back(name, dh):
        dz = dh * (c[name + ".pre"] > 0)
        g[name + ".w"], g[name + ".b"] = conv3d_wgrad(c[name + ".in"], dz)
        return q(conv3d_dgrad(dz, p[name + ".w"]))

    dh = cr_back("d1a", cr_back("d1b", dh))          # 48 channels: [up(d2) | e1]
    d_upd2, de1 = dh[..., :32], dh[..., 32:]
    dh = cr_back("d2a", cr_back("d2b", q(up_back(d_upd2))))  # 96 channels: [up(b3) | e2]
    d_upb3, de2 = dh[..., :64], dh[..., 64:]
    dh = cr_back("c3a", cr_back("c3b", q(up_back(d_upb3))))
    de2 = q(de2 + pool_back(dh))
    dh = cr_back("c2a", cr_back("c2b", de2))
    de1 = q(de1 + pool_back(dh))
    dx = cr_back("c1a", cr_back("c1b", de1))
    return g, dx


def loss(out, t):
    """Relative squared error and its gradient with respect to out."""
    den = np.sum(t * t)
    r = out - t
    return np.sum(r * r) / den, 2.0 * r / den


def loss_phase_invariant(out, t):
    """Scale- and phase-invariant loss of the two-channel output read as a complex field:
        L = 1 - |<o, t>|^2 / (||o||^2 ||t||^2),  o = out[..., 0] + i out[..., 1] (same for t),
    i.e. the relative error of the best complex multiple of o.  Returns (L, dL/dout), the
    gradient with respect to the real and imaginary channels:
        dL/dRe o + i dL/dIm o = -2 conj(S) (t - (S/P) o) / (P Q),  S = <o, t>, P = ||o||^2, Q = ||t||^2.
    """
    o = out[..., 0] + 1j * out[..., 1]
    tc = t[..., 0] + 1j * t[..., 1]
    S = np.vdot(o, tc)
    P = np.vdot(o, o).real
    Q = np.vdot(tc, tc).real
    L = 1.0 - abs(S) ** 2 / (P * Q)
    gc = -2.0 * np.conj(S) * (tc - (S / P) * o) / (P * Q)
    return L, np.stack([gc.real, gc.imag], axis=-1)


def ahat(x, kch):
    """Ahat x on a box with zero values outside: (6 - kch) x - sum of the six neighbours,
    applied to each channel of x [Z, Y, X, C] (Ahat = A / (s/h^2) of Sec. 7.1 with
    kch = omega^2 h^2 / c^2 = kappa / (s/h^2), without the damping term).  Real and
    symmetric, so it is its own transpose."""
    y = (6.0 - kch)[..., None] * x
    for off in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        y = y - _shift(x, off)
    return y


def loss_residual(out, v, kch):
    """Residual loss of a preconditioner output against its input v:
        L = min_d ||v - d Ahat o||^2 / ||v||^2 = 1 - |<Ahat o, v>|^2 / (||Ahat o||^2 ||v||^2),
    the phase-invariant loss of p = Ahat out against v; by the chain rule through the real
    linear map Ahat (its own transpose), dL/dout = Ahat dL/dp."""
    pr = ahat(out, kch)
    L, dp = loss_phase_invariant(pr, v)
    return L, ahat(dp, kch)


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of every parameter in place; step counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
