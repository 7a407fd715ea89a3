"""The Fourier-spectral operator (Sec. 7.1) on the HIP path versus the FP64 oracle, through
the C ABI.

Comparisons are element by element (max |a - ref|).  One product goes through two FFTs,
whose rounding is bounded in the 2-norm: at most 10 u log2 N s lambda_max ||x||_2 plus the
diagonal's 12 u |kappa + i D + shift| |x| (tests/fp32_bounds.py, u = 2^-24 or 2^-53).  The
max norm of an error is at most its 2-norm.  Fixed-point steps in FP32 use the product-form
chain bound of tests/fp32_bounds.py with that per-product rounding, as a 2-norm bound
(max |e| <= bar ||ref||_2).  FP64 fixed-point steps and FCI in lockstep agree to 1e-11 of
max |ref|.
"""
import numpy as np
import pytest

from oracle import fci as OF
from oracle import fixed_point as OFP
from oracle import spectral as OS

from tests.fp32_bounds import (U32, fixed_point_bar, relmax, round32, spectral_absrow, spectral_apply_bound,
                               spectral_roundings)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hf = pytest.importorskip("paper_1811_12378_amd.hfci")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hf.load_library()
    c = hf.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def inputs(x, prec):
    return x if prec == "f64" else round32(x)


def make(ctx, shape, seed, omega, cells=2, rho2=1.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 3.0, size=shape)
    h = 1.0 / shape[0]
    o = OS.SpectralOperator(c, omega, cells, rho2, h=h)
    g = hf.SpectralOperator(ctx, dev(c), h, omega, cells, rho2)
    return o, g


def contour(o, g, J, q):
    poles = OF.pole_parameters(o, J, 1.0, 0.5, q)
    cg = hf.Contour(g, J, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    return poles, cg


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 10, 12), (5, 7, 30), (1, 1, 1), (2, 3, 1)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spectral_apply_parity(ctx, shape, prec):
    o, g = make(ctx, shape, 1, 9.0)
    rng = np.random.default_rng(2)
    x = inputs(rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape), prec)
    shift = 0.37 - 1.21j
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y = host(hf.apply(g, dev(x).to(dt), shift)).astype(np.complex128)
    unit = 1.0 if prec == "f32" else 2.0 ** -53 / U32
    for k in range(3):
        ref = o.apply(x[k], shift)
        bound = unit * spectral_apply_bound(x[k], float(o.lam.max()), o.kappa, o.damp, shift)
        assert np.abs(y[k] - ref).max() <= bound, (shape, prec, k, np.abs(y[k] - ref).max(), bound)


def test_spectral_box(ctx):
    o, g = make(ctx, (10, 9, 12), 3, 14.0)
    info = g.info()
    b1, b2, rho2 = o.rectangle()
    assert abs(info["b1"] - b1) <= 1e-13 * abs(b1) and abs(info["b2"] - b2) <= 1e-12 * abs(b2)
    assert info["rho2"] == rho2


@pytest.mark.parametrize("prec,q,steps", [("f64", 8, 3), ("f64", 3, 2), ("f64", 1, 3), ("f32", 8, 3)])
def test_spectral_shifted_solve_fixed_steps(ctx, prec, q, steps):
    o, g = make(ctx, (9, 12, 16), 5, 16.0)
    poles, cg = contour(o, g, 4, q)
    rng = np.random.default_rng(6)
    f = inputs(rng.standard_normal((2,) + o.shape) + 1j * rng.standard_normal((2,) + o.shape), prec)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y, st = hf.shifted_solve(g, cg, dev(f).to(dt), steps=steps)
    y = host(y)
    assert np.all(st == steps)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, steps=steps)
            if prec == "f64":
                assert relmax(y[j, r], ref) <= 1e-11, (j, r, relmax(y[j, r], ref))
            else:
                bar2 = fixed_point_bar(p, q, steps, o.rectangle(),
                                       spectral_absrow(float(o.lam.max()), o.kappa, o.rho2),
                                       np.linalg.norm(f[r]) / np.linalg.norm(ref),
                                       roundings=spectral_roundings(o.n))
                e = np.abs(y[j, r] - ref).max()
                assert e <= bar2 * np.linalg.norm(ref), (j, r, e, bar2 * np.linalg.norm(ref))


@pytest.mark.parametrize("q", [2, 8])
def test_spectral_shifted_solve_adaptive(ctx, q):
    o, g = make(ctx, (10, 12, 14), 7, 15.0)
    poles, cg = contour(o, g, 6, q)
    rng = np.random.default_rng(8)
    f = rng.standard_normal((2,) + o.shape) + 1j * rng.standard_normal((2,) + o.shape)
    f[1] = 0.0
    y, st = hf.shifted_solve(g, cg, dev(f), reduce=5.0, max_steps=60)
    y = host(y)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        assert st[j, 1] == 0 and np.all(y[j, 1] == 0)
        ref, hist = OFP.fixed_point_solve(Am, f[0], p.z, p.z0, p.delta, q, reduce=5.0, m_max=60)
        assert st[j, 0] == len(hist) - 1, (j, st[j, 0], len(hist) - 1)
        assert relmax(y[j, 0], ref) <= 1e-11


def test_spectral_gathered_batches_past_16(ctx):
    # 12 poles x 3 right-hand sides = 36 systems; rhs 1 is zero, so after step one 24 systems
    # iterate: their vectors are gathered into a batch of 32 (8 zero padding slots), and
    # into exact batches as the poles stop one by one
    o, g = make(ctx, (8, 9, 10), 15, 12.0)
    poles, cg = contour(o, g, 12, 2)
    rng = np.random.default_rng(16)
    f = rng.standard_normal((3,) + o.shape) + 1j * rng.standard_normal((3,) + o.shape)
    f[1] = 0.0
    y, st = hf.shifted_solve(g, cg, dev(f), reduce=5.0, max_steps=60)
    y = host(y)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        assert st[j, 1] == 0 and np.all(y[j, 1] == 0)
        for r in (0, 2):
            ref, hist = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, 2, reduce=5.0, m_max=60)
            assert st[j, r] == len(hist) - 1, (j, r, st[j, r], len(hist) - 1)
            assert relmax(y[j, r], ref) <= 1e-11, (j, r)
    assert len(set(int(v) for v in st[:, 0])) > 1  # the poles stop at different steps


def test_spectral_fci_and_solve_lockstep(ctx):
    o, g = make(ctx, (8, 9, 10), 9, 12.0)
    poles, cg = contour(o, g, 6, 6)
    rng = np.random.default_rng(10)
    f = rng.standard_normal((2,) + o.shape) + 1j * rng.standard_normal((2,) + o.shape)
    out, _ = hf.fci_apply(g, cg, dev(f), hf.default_opts(fp_steps=3, precision=64))
    for r in range(2):
        assert relmax(host(out)[r], OF.fci(o, f[r], poles, steps=3)) <= 1e-11
    opts = hf.default_opts(precision=64, tol=1e-9, max_it=200, fp_steps=2, restart=20)
    u, st = hf.solve(g, cg, dev(f[:1]), opts=opts)
    assert st["status"] == "HFCI_OK"
    uo, info = OF.solve(o, f[0], poles, m=20, tol=1e-9, max_it=200, steps=2)
    assert st["its"] == info["its"]
    assert relmax(host(u)[0], uo) <= 1e-8
    b = o.s * f[0]
    assert np.linalg.norm(b - o.apply(host(u)[0])) / np.linalg.norm(b) <= 1e-9 * 1.01


def test_spectral_mixed_solve(ctx):
    o, g = make(ctx, (16, 16, 16), 11, 20.0)
    cg = hf.Contour(g, 8, 1.0, 0.5, 8)
    rng = np.random.default_rng(12)
    f = rng.standard_normal((1,) + o.shape) + 1j * rng.standard_normal((1,) + o.shape)
    u, st = hf.solve(g, cg, dev(f), opts=hf.default_opts(precision=32, tol=1e-7, max_it=400))
    assert st["status"] == "HFCI_OK"
    b = o.s * f[0]
    assert np.linalg.norm(b - o.apply(host(u)[0])) / np.linalg.norm(b) <= 1e-7 * 1.01


def test_spectral_unsupported_entry_points(ctx):
    import ctypes
    o, g = make(ctx, (6, 6, 6), 13, 9.0)
    poles, cg = contour(o, g, 4, 4)
    f = dev(np.ones((1, 6, 6, 6), dtype=np.complex128))
    for call in (lambda: hf.Operator.autotune(g, 32, 2),
                 lambda: hf.fci_apply(g, cg, f, hf.default_opts(k_in=2)),
                 lambda: hf._check(hf.load_library().hfci_op_case_two(g.h, ctypes.byref(ctypes.c_void_p()))),
                 lambda: hf.solve_batch([g], [cg], [f[0]])):
        with pytest.raises(hf.HfciError) as e:
            call()
        assert e.value.status == -6
