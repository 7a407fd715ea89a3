"""Case two (eq. mat-2x2) on the HIP path versus the FP64 oracle, through the C ABI.

Comparisons are element by element (relmax = max |a - ref| / max |ref|).  Tolerances
as for case one: FP64 1e-13 (one product with B), 1e-12 (fixed-point steps); FP32 the
point-by-point rounding bound of one product with B and, for fixed-point steps, the
first-order rounding bound of the product-form factor chains on B's box
(tests/fp32_bounds.py derives both).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import case_two as OCT
from oracle import fci as OF
from oracle import fixed_point as OFP
from oracle import operator as OO

from tests.fp32_bounds import case_two_absrow, case_two_apply_bound, fixed_point_bar, relmax, round32

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


def fp_tol(prec, o2, p, q, steps, f, ref):
    """FP64 1e-12; FP32 the product-form bound on B's box (tests/fp32_bounds.py)."""
    if prec == "f64":
        return 1e-12
    b = o2.base
    return fixed_point_bar(p, q, steps, o2.rectangle(), case_two_absrow(b.s_h2, b.kappa, b.rho2),
                           np.abs(f).max() / np.abs(ref).max())


def make(ctx, shape, seed, omega, cells, rho2):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 3.0, size=shape)
    h = 1.0 / shape[0]
    o = OO.Operator(c, omega, cells, rho2, h=h)
    g = hf.Operator(ctx, dev(c), h, omega, cells, rho2)
    return OCT.CaseTwoOperator(o), g.case_two(), g


def contour_pair(o2, g2, J, q, eps=0.5):
    poles = OCT.pole_parameters(o2, J, 1.0, eps, q)
    cg = hf.Contour(g2, J, 1.0, eps, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    return poles, cg


@pytest.mark.parametrize("shape", [(8, 8, 8), (11, 13, 37), (5, 7, 130), (1, 1, 1), (2, 3, 1)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_case_two_apply_parity(ctx, shape, prec):
    o2, g2, _ = make(ctx, shape, 1, 9.0, 2, 0.8)
    rng = np.random.default_rng(2)
    x = inputs(rng.standard_normal((3,) + o2.shape) + 1j * rng.standard_normal((3,) + o2.shape), prec)
    shift = 0.37 - 1.21j
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y = host(hf.apply(g2, dev(x).to(dt), shift)).astype(np.complex128)
    b = o2.base
    for k in range(3):
        ref = o2.apply(x[k], shift)
        if prec == "f64":
            assert relmax(y[k], ref) <= 1e-13, (shape, k, relmax(y[k], ref))
        else:
            excess = np.abs(y[k] - ref) - case_two_apply_bound(x[k], b.kappa, b.damp, b.s_h2, shift)
            assert excess.max() <= 0.0, (shape, k, excess.max())


def test_case_two_box_and_contour(ctx):
    o2, g2, g = make(ctx, (9, 10, 11), 3, 14.0, 2, 1.0)
    info, info1 = g2.info(), g.info()
    b1, b2, rho2 = o2.rectangle()
    assert math.isclose(info["b1"], b1, rel_tol=1e-13) and math.isclose(info["b2"], b2, rel_tol=1e-13)
    assert info["rho2"] == rho2 == info1["rho2"]
    # width rho2 + sqrt(rho2^2 + 4 rho1) with rho1 = b2(A) + 1 (the remark after Thm 3.2)
    rho1 = info1["b2"] + 1.0
    assert math.isclose(info["b2"] - info["b1"], rho2 + math.sqrt(rho2 ** 2 + 4 * rho1), rel_tol=1e-13)
    # the library's own contour on B's box: same poles as the oracle's, and its delta
    # search reaches the oracle's rate to the grid of the search
    poles = OCT.pole_parameters(o2, 6, 1.0, 0.5, 8)
    cg = hf.Contour(g2, 6, 1.0, 0.5, 8)
    got = cg.get()
    for j, p in enumerate(poles):
        assert abs(got["z"][j] - p.z) <= 1e-12 * abs(p.z)
        assert abs(got["z0"][j] - p.z0) <= 1e-12 * max(1.0, abs(p.z0))
        assert got["nu"][j] < 1.0


@pytest.mark.parametrize("prec,q,steps", [("f64", 8, 3), ("f64", 3, 4), ("f64", 2, 2), ("f64", 1, 3),
                                          ("f64", 4, 1), ("f64", 5, 2), ("f64", 7, 2), ("f32", 8, 3),
                                          ("f32", 3, 2), ("f32", 5, 2)])
def test_case_two_shifted_solve_fixed_steps(ctx, prec, q, steps):
    o2, g2, _ = make(ctx, (9, 17, 33), 5, 18.0, 3, 1.0)
    poles, cg = contour_pair(o2, g2, 4, q)
    rng = np.random.default_rng(6)
    f = inputs(rng.standard_normal((2,) + o2.shape) + 1j * rng.standard_normal((2,) + o2.shape), prec)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y, st = hf.shifted_solve(g2, cg, dev(f).to(dt), steps=steps)
    y = host(y)
    assert np.all(st == steps)
    Bm = lambda v, sh: o2.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Bm, f[r], p.z, p.z0, p.delta, q, steps=steps)
            e, tol = relmax(y[j, r], ref), fp_tol(prec, o2, p, q, steps, f[r], ref)
            assert e <= tol, (j, r, e, tol)


@pytest.mark.parametrize("prec,q", [("f64", 8), ("f64", 5), ("f32", 8)])
def test_case_two_shifted_solve_larger_grid(ctx, prec, q):
    # the pair and single factor kernels on a grid of several workgroups per system (48 at
    # 16 x 24 x 32 points), fixed steps and adaptive
    o2, g2, _ = make(ctx, (16, 24, 32), 21, 16.0, 3, 1.0)
    poles, cg = contour_pair(o2, g2, 4, q)
    rng = np.random.default_rng(22)
    f = inputs(rng.standard_normal((2,) + o2.shape) + 1j * rng.standard_normal((2,) + o2.shape), prec)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y, st = hf.shifted_solve(g2, cg, dev(f).to(dt), steps=2)
    y = host(y)
    assert np.all(st == 2)
    Bm = lambda v, sh: o2.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Bm, f[r], p.z, p.z0, p.delta, q, steps=2)
            e, tol = relmax(y[j, r], ref), fp_tol(prec, o2, p, q, 2, f[r], ref)
            assert e <= tol, (j, r, e, tol)
    # adaptive, with a zero right-hand side among iterating ones
    f[1] = 0.0
    y, st = hf.shifted_solve(g2, cg, dev(f).to(dt), reduce=5.0, max_steps=60)
    y = host(y)
    fn = np.linalg.norm(f[0])
    for j, p in enumerate(poles):
        assert st[j, 1] == 0 and np.all(y[j, 1] == 0)
        ref, hist = OFP.fixed_point_solve(Bm, f[0], p.z, p.z0, p.delta, q, reduce=5.0, m_max=60)
        k = int(st[j, 0])
        if prec == "f64":
            assert k == len(hist) - 1, (j, k, len(hist) - 1)
            assert relmax(y[j, 0], ref) <= 1e-12
        else:
            # an FP32 residual can fall on the other side of the threshold than the FP64
            # one: the step count may differ by one, and the iterate is the oracle's after
            # exactly the steps the GPU took, which meet the stopping rule
            assert abs(k - (len(hist) - 1)) <= 1
            ref_k, _ = OFP.fixed_point_solve(Bm, f[0], p.z, p.z0, p.delta, q, steps=k)
            e, tol = relmax(y[j, 0], ref_k), fp_tol(prec, o2, p, q, k, f[0], ref_k)
            assert e <= tol, (j, k, e, tol)
            r = np.linalg.norm(f[0] - o2.apply(y[j, 0].astype(np.complex128), p.z))
            assert r <= fn / 5 * (1 + 1e-4), (j, r / fn)


@pytest.mark.parametrize("q", [1, 2, 3, 5, 8])
def test_case_two_shifted_solve_adaptive(ctx, q):
    # every (pole, rhs) stops at the oracle's step with the oracle's iterate; rhs 1 is
    # zero: its systems stop at step 0 with y = 0 while the others iterate, so the later
    # launches skip stopped systems
    o2, g2, _ = make(ctx, (10, 12, 14), 7, 15.0, 3, 1.0)
    poles, cg = contour_pair(o2, g2, 6, q)
    rng = np.random.default_rng(8)
    f = rng.standard_normal((3,) + o2.shape) + 1j * rng.standard_normal((3,) + o2.shape)
    f[1] = 0.0
    f[2] *= 1e-3
    y, st = hf.shifted_solve(g2, cg, dev(f), reduce=5.0, max_steps=60)
    y = host(y)
    Bm = lambda v, sh: o2.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(3):
            if r == 1:
                assert st[j, r] == 0 and np.all(y[j, r] == 0)
                continue
            ref, hist = OFP.fixed_point_solve(Bm, f[r], p.z, p.z0, p.delta, q, reduce=5.0, m_max=60)
            assert st[j, r] == len(hist) - 1, (j, r, st[j, r], len(hist) - 1)
            assert relmax(y[j, r], ref) <= 1e-12, (j, r, relmax(y[j, r], ref))
            assert st[j, r] >= 1


def test_case_two_step_cap(ctx):
    o2, g2, _ = make(ctx, (8, 9, 10), 9, 12.0, 2, 1.0)
    poles, cg = contour_pair(o2, g2, 4, 4)
    rng = np.random.default_rng(10)
    f = rng.standard_normal((1,) + o2.shape) + 1j * rng.standard_normal((1,) + o2.shape)
    y, st = hf.shifted_solve(g2, cg, dev(f), reduce=1e12, max_steps=2)
    assert np.all(st == 2)
    Bm = lambda v, sh: o2.apply(v, sh)
    for j, p in enumerate(poles):
        ref, _ = OFP.fixed_point_solve(Bm, f[0], p.z, p.z0, p.delta, 4, steps=2)
        assert relmax(host(y)[j, 0], ref) <= 1e-12


def test_case_two_unsupported_entry_points(ctx):
    import ctypes
    o2, g2, g = make(ctx, (6, 6, 6), 11, 9.0, 1, 0.5)
    poles, cg = contour_pair(o2, g2, 4, 4)
    f = dev(np.ones((1, 6, 6, 6), dtype=np.complex128))
    f2 = dev(np.ones((1, 2, 6, 6, 6), dtype=np.complex128))
    for call in (lambda: hf.solve(g2, cg, f2, opts=hf.default_opts(precond=hf.HFCI_PRECOND_LEARNED)),
                 lambda: hf.Operator.set_tune(g2, 32, 1, 8, 2, 0, 0),
                 lambda: hf.Operator.autotune(g2, 32, 2),
                 lambda: hf._check(hf.load_library().hfci_op_case_two(g2.h, ctypes.byref(ctypes.c_void_p())))):
        with pytest.raises(hf.HfciError) as e:
            call()
        assert e.value.status == -6
    # a contour of the case-one operator is rejected for the case-two handle
    c1 = hf.Contour(g, 4, 1.0, 0.5, 4)
    with pytest.raises(hf.HfciError) as e:
        hf.shifted_solve(g2, c1, dev(np.ones((1, 2, 6, 6, 6), dtype=np.complex128)), steps=1)
    assert e.value.status == -6
    # the case-one operator still works after its case-two handle is released
    g2.close()
    y, st = hf.shifted_solve(g, c1, f, steps=1)
    assert np.all(st == 1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_case_two_fci_lockstep(ctx, prec):
    # Algorithm 1 on B with a fixed step count: shifted solves, quadrature, step 3 with B w
    o2, g2, _ = make(ctx, (10, 11, 12), 9, 15.0, 3, 1.0)
    poles, cg = contour_pair(o2, g2, 8, 8)
    rng = np.random.default_rng(10)
    f = inputs(rng.standard_normal((3,) + o2.shape) + 1j * rng.standard_normal((3,) + o2.shape), prec)
    opts = hf.default_opts(fp_steps=4, precision=64 if prec == "f64" else 32)
    out, st = hf.fci_apply(g2, cg, dev(f), opts)
    out = host(out)
    assert st["fp_steps"] == 8 * 3 * 4
    for r in range(3):
        ref, parts = OF.fci(o2, f[r], poles, steps=4, return_parts=True)
        if prec == "f64":
            tol = 1e-12
        else:
            # each pole's bar through the quadrature sum's cancellation, times 3 for d
            num = sum(abs(p.sigma / p.z) * fp_tol(prec, o2, p, 8, 4, f[r], y) * np.abs(y).max()
                      for p, y in zip(poles, parts["ys"]))
            tol = 3.0 * num / np.abs(parts["w"]).max()
        e = relmax(out[r], ref)
        assert e <= tol, (r, e, tol)


def test_case_two_solve_lockstep_and_direct(ctx):
    # FGMRES on eq. mat-2x2 with FCI(B), FP64 sweeps and a fixed step count: the same
    # iteration count as the oracle's, x2 = u and x1 = i u of the direct solve of A u = s f
    o2, g2, g = make(ctx, (8, 9, 10), 12, 12.0, 2, 1.0)
    poles, cg = contour_pair(o2, g2, 6, 6)
    rng = np.random.default_rng(13)
    f = rng.standard_normal(o2.base.shape) + 1j * rng.standard_normal(o2.base.shape)
    rhs = np.stack([np.zeros_like(f), f])[None]
    opts = hf.default_opts(precision=64, tol=1e-9, max_it=300, fp_steps=2, restart=20)
    x, st = hf.solve(g2, cg, dev(rhs), opts=opts)
    assert st["status"] == "HFCI_OK"
    x = host(x)[0]
    u_o, info = OCT.solve(o2.base, f, poles, m=20, tol=1e-9, max_it=300, steps=2)
    assert st["its"] == info["its"]
    A = o2.base.assemble().tocsc()
    import scipy.sparse.linalg as spla
    uref = spla.spsolve(A, (o2.base.s * f).ravel()).reshape(f.shape)
    assert relmax(x[1], uref) <= 1e-8
    assert relmax(x[0], 1j * uref) <= 1e-8
    assert relmax(x[1], u_o) <= 1e-8


def test_case_two_solve_mixed_adaptive(ctx):
    # mixed precision (FP32 sweeps, FP64 FGMRES), adaptive fixed-point steps.  FGMRES meets
    # the tolerance on the double-size system (the oracle's FP64 residual of x on B); for
    # u = x2 the residual on A is b - A x2 = i (A1 + I) r1 - r2 with [r1; r2] the residual of
    # x, so it is bounded by (rho1 + 1) times the tolerance
    o2, g2, g = make(ctx, (12, 13, 14), 14, 16.0, 3, 1.0)
    cg = hf.Contour(g2, 8, 1.0, 0.5, 8)
    rng = np.random.default_rng(15)
    f = rng.standard_normal(o2.base.shape) + 1j * rng.standard_normal(o2.base.shape)
    rhs = np.stack([np.zeros_like(f), f])[None]
    tol = 1e-7
    opts = hf.default_opts(precision=32, tol=tol, max_it=400)
    x, st = hf.solve(g2, cg, dev(rhs), opts=opts)
    assert st["status"] == "HFCI_OK" and st["fp_steps"] > 0
    x = host(x)[0]
    b = o2.base.s * f
    b2 = o2.rhs(b)
    r2 = np.linalg.norm(b2 - o2.apply(x)) / np.linalg.norm(b2)
    assert r2 <= tol * 1.01, r2
    ra = np.linalg.norm(b - o2.base.apply(x[1])) / np.linalg.norm(b)
    assert ra <= (o2.rho1() + 1.0) * tol, ra


def test_case_two_apply_every_point_at_256(ctx):
    # the headline medium at 256^3 (complex64, the precision of its sweeps): every point of
    # (B - shift) x inside the FP32 rounding bound of the oracle's product
    wl = W.config_layered_256(nrhs=1)
    g = hf.Operator(ctx, dev(wl.c), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    g2 = g.case_two()
    o = OO.Operator(wl.c, wl.omega, wl.damp_cells, wl.damp_rho2, h=wl.h)
    o2 = OCT.CaseTwoOperator(o)
    n = wl.c.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13)
    x = torch.randn((2, n, n, n), dtype=torch.complex64, device="cuda", generator=gen)
    shift = -0.21 + 0.6j
    y = host(hf.apply(g2, x, shift)).astype(np.complex128)
    xh = host(x).astype(np.complex128)
    excess = np.abs(y - o2.apply(xh, shift)) - case_two_apply_bound(xh, o.kappa, o.damp, o.s_h2, shift)
    assert excess.max() <= 0.0, excess.max()
