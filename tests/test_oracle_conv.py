"""Pins of the oracle's convolution network: brute force and finite differences."""
import numpy as np
import pytest

from oracle import conv as C


def brute_conv(x, w, b):
    Z, Y, X, cin = x.shape
    cout = w.shape[1]
    y = np.zeros((Z, Y, X, cout))
    for z in range(Z):
        for yy in range(Y):
            for xx in range(X):
                for co in range(cout):
                    s = b[co]
                    for t, (dz, dy, dx) in enumerate(C.OFFSETS):
                        zz, y2, x2 = z + dz, yy + dy, xx + dx
                        if 0 <= zz < Z and 0 <= y2 < Y and 0 <= x2 < X:
                            for ci in range(cin):
                                s += w[t, co, ci] * x[zz, y2, x2, ci]
                    y[z, yy, xx, co] = s
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 2))
    w = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(3)
    assert np.allclose(C.conv3d(x, w, b), brute_conv(x, w, b), atol=1e-12)


def test_conv_gradients_by_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 3, 5, 3))
    w = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    gy = rng.standard_normal((4, 3, 5, 2))
    L = lambda x, w, b: np.sum(gy * C.conv3d(x, w, b))
    dx = C.conv3d_dgrad(gy, w)
    dw, db = C.conv3d_wgrad(x, gy)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (3, 2, 4, 2), (1, 1, 2, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((L(x + e, w, b) - L(x - e, w, b)) / (2 * h) - dx[idx]) < 1e-6
    for idx in [(0, 0, 0), (13, 1, 2), (26, 0, 1)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((L(x, w + e, b) - L(x, w - e, b)) / (2 * h) - dw[idx]) < 1e-6
    e = np.zeros_like(b)
    e[1] = h
    assert abs((L(x, w, b + e) - L(x, w, b - e)) / (2 * h) - db[1]) < 1e-6


def test_pool_up_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert np.isclose(np.sum(C.pool(x) * y), np.sum(x * C.pool_back(y)))
    assert np.isclose(np.sum(C.up(y) * x), np.sum(y * C.up_back(x)))


def test_unet_gradients_by_finite_differences():
    rng = np.random.default_rng(3)
    p = C.init_params(7)
    for k in p:  # non-zero biases so that every term is exercised
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    x = rng.standard_normal((4, 4, 4, 3))
    t = rng.standard_normal((4, 4, 4, 2))
    out, cache = C.forward(p, x)
    L, dout = C.loss(out, t)
    g, dx = C.backward(p, cache, dout)
    h = 1e-6

    def Lof(pp, xx):
        return C.loss(C.forward(pp, xx)[0], t)[0]

    for name, idx in [("c1a.w", (13, 3, 1)), ("c2b.w", (0, 5, 7)), ("c3b.w", (26, 63, 10)),
                      ("d2a.w", (4, 1, 70)), ("d1a.w", (9, 15, 40)), ("d1b.b", (2,)), ("out.w", (1, 5)),
                      ("c3a.b", (11,)), ("out.b", (0,))]:
        pp = {k: v.copy() for k, v in p.items()}
        pm = {k: v.copy() for k, v in p.items()}
        pp[name][idx] += h
        pm[name][idx] -= h
        fd = (Lof(pp, x) - Lof(pm, x)) / (2 * h)
        assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, fd, g[name][idx])
    for idx in [(0, 0, 0, 0), (3, 1, 2, 2)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (Lof(p, x + e) - Lof(p, x - e)) / (2 * h)
        assert abs(fd - dx[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_step_closed_form():
    p = {"a": np.array([1.0, -2.0])}
    g = {"a": np.array([0.5, -0.25])}
    m = {"a": np.zeros(2)}
    v = {"a": np.zeros(2)}
    C.adam_step(p, g, m, v, 1, lr=0.1)
    # first bias-corrected step moves every coordinate by lr * sign(g)
    assert np.allclose(p["a"], [1.0 - 0.1, -2.0 + 0.1], atol=1e-7)


def test_phase_invariant_loss():
    rng = np.random.default_rng(11)
    out = rng.standard_normal((3, 4, 5, 2))
    t = rng.standard_normal((3, 4, 5, 2))
    L, g = C.loss_phase_invariant(out, t)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (2, 3, 4, 1), (1, 2, 3, 0)]:
        e = np.zeros_like(out)
        e[idx] = h
        fd = (C.loss_phase_invariant(out + e, t)[0] - C.loss_phase_invariant(out - e, t)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7
    # invariant to a complex scale of the output; zero for a complex multiple of the target
    a = 0.3 - 1.7j
    tc = t[..., 0] + 1j * t[..., 1]
    oc = a * tc
    assert C.loss_phase_invariant(np.stack([oc.real, oc.imag], -1), t)[0] < 1e-14
    o2 = (out[..., 0] + 1j * out[..., 1]) * a
    assert abs(C.loss_phase_invariant(np.stack([o2.real, o2.imag], -1), t)[0] - L) < 1e-12


def test_residual_loss_pins():
    # Ahat against the operator's CSR assembly (Kronecker sums of second differences):
    # with damping 0, kappa = kch and s/h^2 = 1 the assembled matrix is Ahat itself
    import scipy.sparse.linalg as spla
    from oracle import operator as OO
    rng = np.random.default_rng(12)
    shape = (4, 5, 6)
    kch = rng.uniform(0.1, 0.9, size=shape)
    Am = OO.assemble(shape, kch, np.zeros(shape), 1.0).toarray()
    x = rng.standard_normal(shape + (2,))
    ax = C.ahat(x, kch)
    for c in range(2):
        assert np.allclose(ax[..., c].ravel(), Am @ x[..., c].ravel(), atol=1e-12)
    assert np.allclose(Am, Am.T)  # real symmetric: its own transpose
    # the loss is the brute-force least-squares minimum over one complex coefficient d
    out = rng.standard_normal(shape + (2,))
    v = rng.standard_normal(shape + (2,))
    L, g = C.loss_residual(out, v, kch)
    vc = (v[..., 0] + 1j * v[..., 1]).ravel()
    col = (Am @ (out[..., 0] + 1j * out[..., 1]).ravel())[:, None]
    d, *_ = np.linalg.lstsq(col, vc, rcond=None)
    brute = np.linalg.norm(vc - col[:, 0] * d[0]) ** 2 / np.linalg.norm(vc) ** 2
    assert abs(L - brute) < 1e-12
    # zero for a complex multiple of the exact solve Ahat e = v
    e = spla.spsolve(OO.assemble(shape, kch, np.zeros(shape), 1.0).tocsc().astype(complex), vc).reshape(shape)
    e = (0.4 + 2.1j) * e
    assert C.loss_residual(np.stack([e.real, e.imag], -1), v, kch)[0] < 1e-13
    # gradient by central differences
    h = 1e-6
    for idx in [(0, 0, 0, 0), (3, 4, 5, 1), (2, 1, 3, 0)]:
        ep = np.zeros_like(out)
        ep[idx] = h
        fd = (C.loss_residual(out + ep, v, kch)[0] - C.loss_residual(out - ep, v, kch)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7


def test_unet_forward_against_library_primitives():
    # the network of the module docstring built from torch's CPU primitives (channels-first
    # cross-correlation conv3d with zero padding, 2x2x2 average pooling, nearest x2
    # up-sampling, channel concatenation), with the oracle's parameters: pins the skip
    # order, the pooling and the up-sampling against an implementation that shares nothing
    # with the oracle's loops
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    p = C.init_params(seed=3)
    rng = np.random.default_rng(11)
    for name, _, cout in C.LAYERS:
        p[name + ".b"] = 0.1 * rng.standard_normal(cout)
    p["out.b"] = 0.1 * rng.standard_normal(2)
    x = rng.standard_normal((8, 8, 8, 3))
    out, _ = C.forward(p, x)

    def conv(h, name):
        w = p[name + ".w"]  # [27, cout, cin], tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)
        k = torch.from_numpy(w.reshape(3, 3, 3, w.shape[1], w.shape[2])).permute(3, 4, 0, 1, 2).contiguous()
        return F.relu(F.conv3d(h, k, torch.from_numpy(p[name + ".b"]), padding=1))

    def block(h, a, b):
        return conv(conv(h, a), b)

    xt = torch.from_numpy(x).permute(3, 0, 1, 2).unsqueeze(0)  # [1, C, Z, Y, X]
    e1 = block(xt, "c1a", "c1b")
    e2 = block(F.avg_pool3d(e1, 2), "c2a", "c2b")
    b3 = block(F.avg_pool3d(e2, 2), "c3a", "c3b")
    d2 = block(torch.cat([F.interpolate(b3, scale_factor=2, mode="nearest"), e2], dim=1), "d2a", "d2b")
    d1 = block(torch.cat([F.interpolate(d2, scale_factor=2, mode="nearest"), e1], dim=1), "d1a", "d1b")
    head = torch.from_numpy(p["out.w"]).reshape(2, 16, 1, 1, 1)
    ref = F.conv3d(d1, head, torch.from_numpy(p["out.b"]))[0].permute(1, 2, 3, 0).numpy()
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
    # a swapped skip order is caught: the pin is sensitive to it
    d2s = block(torch.cat([e2, F.interpolate(b3, scale_factor=2, mode="nearest")], dim=1), "d2a", "d2b")
    d1s = block(torch.cat([F.interpolate(d2s, scale_factor=2, mode="nearest"), e1], dim=1), "d1a", "d1b")
    alt = F.conv3d(d1s, head, torch.from_numpy(p["out.b"]))[0].permute(1, 2, 3, 0).numpy()
    assert np.max(np.abs(out - alt)) > 1e-3 * np.max(np.abs(ref))
