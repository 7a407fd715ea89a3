"""HIP path versus the FP64 oracle, through the C ABI (needs an MI355X).

Every comparison is element by element: relmax(a, ref) = max |a - ref| / max |ref|.
Tolerances (tests/fp32_bounds.py derives the FP32 ones):
  * FP64 kernels: 1e-13 (one stencil product), 1e-12 (fixed-point steps and FCI in
    lockstep), 1e-10 (a full FGMRES solve in lockstep, with fixed counts and parameters);
  * FP32, one stencil product: the point-by-point rounding bound of a nine-term complex
    sum, 12 u (|d_i| |x_i| + s/h^2 sum_j |x_j|), with u = 2^-24;
  * FP32, fixed-point steps in product form (Sec. 4.2, eq. fix-pt-exp): the first-order
    rounding bound of the Leja-ordered linear-factor chains in the eigenvalue model,
    computed from the same poles, delta and q, times the number of steps;
  * FP32 FCI (Alg. 1): each pole's bar weighted by |sigma_j / z_j| max|y_j| over max|w|
    (the quadrature sum's cancellation), times 3 for the step size d.
FP32 inputs are rounded to FP32 before they reach the oracle.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import contour as OC
from oracle import fci as OF
from oracle import fixed_point as OFP
from oracle import operator as OO
from oracle import polynomial as OP

from tests.fp32_bounds import apply_bound, fixed_point_bar, relmax, round32, stencil_absrow

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


def fp_bar(o, p, q, steps, f, ref):
    """FP32 relmax bar of `steps` fixed-point steps of pole p (tests/fp32_bounds.py)."""
    return fixed_point_bar(p, q, steps, o.rectangle(), stencil_absrow(o.s_h2, o.kappa, o.rho2),
                           np.abs(f).max() / np.abs(ref).max())


def fp_tol(prec, o, p, q, steps, f, ref):
    return 1e-12 if prec == "f64" else fp_bar(o, p, q, steps, f, ref)


def fci_tol(prec, o, poles, q, steps, f):
    """FP64 1e-12; FP32: the poles' fixed-point bars through the quadrature sum and d."""
    if prec == "f64":
        return 1e-12
    _, parts = OF.fci(o, f, poles, steps=steps, return_parts=True)
    w = parts["w"]
    num = sum(abs(p.sigma / p.z) * fp_bar(o, p, q, steps, f, y) * np.abs(y).max()
              for p, y in zip(poles, parts["ys"]))
    return 3.0 * num / np.abs(w).max()


def check_apply(y, o, x, shift, prec):
    """y = (A - shift) x from the GPU: FP64 to 1e-13 of max|ref|, FP32 inside the
    point-by-point rounding bound (x must be the FP32 value the device saw)."""
    ref = o.apply(x, shift)
    if prec == "f64":
        assert relmax(y, ref) <= 1e-13, relmax(y, ref)
    else:
        excess = np.abs(y - ref) - apply_bound(x, o.kappa, o.damp, o.s_h2, shift)
        assert excess.max() <= 0.0, (excess.max(), relmax(y, ref))


def inputs(x, prec):
    """The host array the oracle gets: x itself, or its FP32 rounding."""
    return x if prec == "f64" else round32(x)


def medium(shape, seed, lo=1.0, hi=3.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)


def make_ops(ctx, c, omega, cells, rho2, h=None):
    h = 1.0 / c.shape[0] if h is None else h
    o = OO.Operator(c, omega, cells, rho2, h=h)
    g = hf.Operator(ctx, dev(c), h, omega, cells, rho2)
    return o, g


SHAPES = [(8, 8, 8), (9, 17, 33), (70, 9, 5), (5, 7, 130), (1, 1, 1), (2, 3, 1)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_apply_parity(ctx, shape, prec):
    c = medium(shape, 1)
    o, g = make_ops(ctx, c, 9.0, 2, 0.8)
    rng = np.random.default_rng(2)
    x = inputs(rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape), prec)
    shift = 0.37 - 1.21j
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y = host(hf.apply(g, dev(x).to(dt), shift))
    for k in range(3):
        check_apply(y[k], o, x[k], shift, prec)


TUNES = [(0, 4, 1, 0, 0), (0, 4, 2, 0, 0), (0, 8, 1, 0, 0), (0, 8, 2, 3, 0), (0, 4, 2, 1, 0), (1, 4, 1, 0, 0),
         (1, 4, 2, 0, 0), (1, 4, 3, 0, 0), (1, 8, 2, 0, 0), (1, 8, 3, 0, 0), (1, 4, 3, 1, 0), (1, 4, 2, 5, 0),
         (1, 8, 3, 7, 0), (1, 8, 2, 0, 1), (1, 8, 2, 1, 1), (1, 8, 2, 5, 1), (0, 4, 1, 3, 1),
         (1, 8, 3, 0, 1), (1, 8, 3, 2, 1), (1, 8, 3, 5, 1)]


@pytest.mark.parametrize("tune", TUNES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tune_variants_apply_and_fixed_point(ctx, tune, prec):
    # every launch shape (register or LDS-staged kernel, tile height, prefetch depth,
    # z-chunk, including 1-plane chunks and chunks that do not divide nz) gives the
    # same operator and the same fixed-point iterates as the oracle
    dt = torch.complex128 if prec == "f64" else torch.complex64
    pr = 64 if prec == "f64" else 32
    rng = np.random.default_rng(31)
    for shape in [(9, 17, 33), (70, 9, 5), (5, 7, 130), (2, 3, 1), (33, 12, 70)]:
        c = medium(shape, 30)
        o, g = make_ops(ctx, c, 9.0, 2, 0.8)
        g.set_tune(pr, *tune)
        assert g.get_tune(pr) == tuple(tune) + (1,) * (6 - len(tune))
        x = inputs(rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape), prec)
        y = host(hf.apply(g, dev(x).to(dt), 0.37 - 1.21j))
        for k in range(2):
            check_apply(y[k], o, x[k], 0.37 - 1.21j, prec)
    shape = (11, 10, 70)
    c = medium(shape, 32)
    o, g = make_ops(ctx, c, 14.0, 3, 1.0)
    g.set_tune(pr, *tune)
    q = 4
    poles = oracle_poles(o, 4, 1.0, 0.5, q)
    cg = gpu_contour(g, poles, 4, q)
    f = inputs(rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape), prec)
    y, st = hf.shifted_solve(g, cg, dev(f).to(dt), steps=3)
    y = host(y)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, steps=3)
            e, tol = relmax(y[j, r], ref), fp_tol(prec, o, p, q, 3, f[r], ref)
            assert e <= tol, (j, r, e, tol)


@pytest.mark.parametrize("pr", [32, 64])
def test_autotune_picks_a_timed_shape(ctx, pr):
    o, g = make_ops(ctx, medium((40, 33, 70), 3), 9.0, 2, 0.8)
    best, rows = g.autotune(pr, 2)
    assert len(rows) >= 9
    assert all(ms > 0 for _, ms in rows)
    assert best == min(rows, key=lambda r: r[1])[0]
    assert g.get_tune(pr) == best
    # the tuned shape still gives the oracle's operator
    rng = np.random.default_rng(5)
    prec = "f64" if pr == 64 else "f32"
    x = inputs(rng.standard_normal((1, 40, 33, 70)) + 1j * rng.standard_normal((1, 40, 33, 70)), prec)
    dt = torch.complex128 if pr == 64 else torch.complex64
    y = host(hf.apply(g, dev(x).to(dt), 0.2 + 0.7j))
    check_apply(y[0], o, x[0], 0.2 + 0.7j, prec)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("pd", [2, 3])
def test_fused_factor_pairs_every_q(ctx, q, prec, pd):
    # two factors per pass: every split of step one (q-1 factors) and of later steps (q)
    # into pairs and a trailing single, adaptive stopping with the pair kernel's residual
    # partials, on a grid with ragged 64 x 12 tiles and several z-chunks; loads one plane
    # ahead (pd 2) and two (pd 3)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    pr = 64 if prec == "f64" else 32
    shape = (21, 13, 70)
    c = medium(shape, 41)
    o, g = make_ops(ctx, c, 14.0, 3, 1.0)
    g.set_tune(pr, 1, 8, pd, 8, 1)
    poles = oracle_poles(o, 4, 1.0, 0.5, q)
    cg = gpu_contour(g, poles, 4, q)
    rng = np.random.default_rng(42)
    f = inputs(rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape), prec)
    Am = lambda v, sh: o.apply(v, sh)
    y, st = hf.shifted_solve(g, cg, dev(f).to(dt), steps=3)
    y = host(y)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, steps=3)
            e, tol = relmax(y[j, r], ref), fp_tol(prec, o, p, q, 3, f[r], ref)
            assert e <= tol, (j, r, e, tol)
    if prec == "f64":
        y, st = hf.shifted_solve(g, cg, dev(f), reduce=5.0, max_steps=60)
        y = host(y)
        for j, p in enumerate(poles):
            for r in range(2):
                ref, hist = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, reduce=5.0, m_max=60)
                assert st[j, r] == len(hist) - 1
                assert relmax(y[j, r], ref) <= 1e-12


def test_profiler_times_every_kth_launch(ctx):
    # hfci_ctx_profile(k): every k-th launch of a class is bracketed by events; the counters
    # cover exactly the timed launches (7 applies, k = 3: launches 0, 3, 6)
    o, g = make_ops(ctx, medium((9, 8, 7), 1), 9.0, 1, 0.5)
    x = dev(np.ones((1, 9, 8, 7), complex)).to(torch.complex64)
    ctx.profile(True, every=3)
    for _ in range(7):
        hf.apply(g, x, 0.0)
    p = ctx.profile_read()
    ctx.profile(False)
    assert p["apply"]["launches"] == 3
    assert p["apply"]["total_ms"] > 0
    assert p["apply"]["alg_bytes"] == pytest.approx(3 * 9 * 8 * 7 * (2 * 8 + 4))
    with pytest.raises(hf.HfciError):
        ctx.profile(True, every=-1)


def test_tune_rejects_invalid(ctx):
    o, g = make_ops(ctx, medium((4, 4, 4), 1), 9.0, 1, 0.5)
    for bad in [(2, 4, 1, 0), (0, 5, 1, 0), (0, 4, 3, 0), (1, 8, 1, 0), (1, 4, 4, 0), (0, 4, 1, -1),
                (1, 8, 2, 0, 2), (2, 8, 2, 0, 2), (3, 8, 2, 0, 3), (3, 8, 3, 0, 2), (1, 8, 2, 0, 1, 0),
                (1, 8, 2, 0, 1, 17)]:
        with pytest.raises(hf.HfciError):
            g.set_tune(32, *bad)
    with pytest.raises(hf.HfciError):  # three factors per pass: complex64 only
        g.set_tune(64, 3, 8, 2, 0, 2)
    g.set_tune(32, 3, 8, 2, 0, 2, 4)
    assert g.get_tune(32) == (3, 8, 2, 0, 2, 4)


def test_op_info_matches_oracle(ctx):
    c = medium((6, 7, 8), 3)
    o, g = make_ops(ctx, c, 11.0, 3, 1.2, h=0.1)
    info = g.info()
    b1, b2, rho2 = o.rectangle()
    assert info["s"] == pytest.approx(o.s, rel=1e-15)
    assert info["s_h2"] == pytest.approx(o.s_h2, rel=1e-15)
    assert (info["b1"], info["b2"], info["rho2"]) == pytest.approx((b1, b2, rho2), rel=1e-14, abs=1e-14)


def test_contour_parameters_match_oracle(ctx):
    c = medium((12, 12, 12), 4)
    o, g = make_ops(ctx, c, 14.0, 3, 1.0)
    b1, b2, rho2 = o.rectangle()
    for J, t, eps, q in [(8, 1.0, 0.5, 8), (6, 0.1, 0.3, 3), (12, 0.5, 0.4, 4)]:
        cg = hf.Contour(g, J, t, eps, q).get()
        z, sigma, _ = OC.poles_and_weights(J, t, eps, rho2)
        assert np.abs(cg["z"] - z).max() <= 1e-13 * np.abs(z).max()
        assert np.abs(cg["sigma"] - sigma).max() <= 1e-13 * np.abs(sigma).max()
        bd = OP.rectangle_boundary(b1, b2, rho2, 2000)
        for j in range(J):
            d_o, nu_o, z0_o = OP.optimise_delta(z[j], b1, b2, rho2, q, per_side=2000)
            assert abs(cg["z0"][j] - z0_o) <= 1e-13 * abs(z0_o)
            assert np.sign(cg["delta"][j]) == np.sign(z[j].imag)
            # both minimise the same objective: equal minima, and the library's delta is
            # (near-)optimal when scored by the oracle
            assert abs(cg["nu"][j] - nu_o) <= 1e-6
            assert OP.rate(cg["delta"][j], z[j], z0_o, q, bd) <= nu_o + 1e-6


def oracle_poles(o, J, t, eps, q):
    return OF.pole_parameters(o, J, t, eps, q)


def gpu_contour(g, poles, J, q):
    return hf.Contour(g, J, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                      delta=[p.delta for p in poles])


@pytest.mark.parametrize("prec,q,steps", [("f64", 8, 3), ("f64", 3, 4), ("f64", 1, 5), ("f64", 2, 2),
                                          ("f64", 8, 1), ("f64", 2, 1), ("f64", 1, 1),
                                          ("f32", 8, 3), ("f32", 4, 2)])
def test_shifted_solve_fixed_steps(ctx, prec, q, steps):
    shape = (9, 17, 33)
    c = medium(shape, 5)
    o, g = make_ops(ctx, c, 18.0, 3, 1.0)
    poles = oracle_poles(o, 6, 1.0, 0.5, q)
    cg = gpu_contour(g, poles, 6, q)
    rng = np.random.default_rng(6)
    f = inputs(rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape), prec)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y, st = hf.shifted_solve(g, cg, dev(f).to(dt), steps=steps)
    y = host(y)
    assert np.all(st == steps)
    Am = lambda x, s: o.apply(x, s)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, steps=steps)
            e, tol = relmax(y[j, r], ref), fp_tol(prec, o, p, q, steps, f[r], ref)
            assert e <= tol, (j, r, e, tol)


def test_shifted_solve_adaptive_stop_rule(ctx):
    shape = (12, 12, 12)
    c = medium(shape, 7)
    o, g = make_ops(ctx, c, 16.0, 3, 1.0)
    poles = oracle_poles(o, 8, 1.0, 0.5, 8)
    cg = gpu_contour(g, poles, 8, 8)
    rng = np.random.default_rng(8)
    f = rng.standard_normal((1,) + shape) + 1j * rng.standard_normal((1,) + shape)
    y, st = hf.shifted_solve(g, cg, dev(f), reduce=5.0, max_steps=300)
    y = host(y)
    Am = lambda x, s: o.apply(x, s)
    fn = np.linalg.norm(f[0])
    for j, p in enumerate(poles):
        ref, hist = OFP.fixed_point_solve(Am, f[0], p.z, p.z0, p.delta, 8, reduce=5.0, m_max=300)
        k = st[j, 0]
        # the returned iterate satisfies the rule and the previous one did not
        r = np.linalg.norm(f[0] - o.apply(y[j, 0], p.z))
        assert r <= fn / 5 * (1 + 1e-9)
        assert hist[k - 1] > fn / 5 * (1 - 1e-9)
        if k == len(hist) - 1:
            assert relmax(y[j, 0], ref) <= 1e-12


def test_adaptive_many_systems_and_zero_rhs(ctx):
    # 24 poles x 12 right-hand sides = 288 systems (more than one block of the device-side
    # list compaction), stopping at different steps; rhs 5 is zero: 0 steps, y = 0
    shape = (8, 9, 10)
    c = medium(shape, 21)
    o, g = make_ops(ctx, c, 12.0, 2, 1.0)
    J, q, nrhs = 24, 4, 12
    poles = oracle_poles(o, J, 1.0, 0.5, q)
    cg = gpu_contour(g, poles, J, q)
    rng = np.random.default_rng(22)
    f = rng.standard_normal((nrhs,) + shape) + 1j * rng.standard_normal((nrhs,) + shape)
    f[3] *= 1e-3
    f[5] = 0.0
    y, st = hf.shifted_solve(g, cg, dev(f), reduce=5.0, max_steps=40)
    y = host(y)
    assert len(set(st.ravel().tolist())) >= 3  # the systems really stop at different steps
    Am = lambda x, s: o.apply(x, s)
    for j, p in enumerate(poles):
        for r in range(nrhs):
            ref, hist = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, reduce=5.0, m_max=40)
            if r == 5:
                assert st[j, r] == 0 and np.all(y[j, r] == 0)
                continue
            assert st[j, r] == len(hist) - 1, (j, r, st[j, r], len(hist) - 1)
            assert relmax(y[j, r], ref) <= 1e-12, (j, r, relmax(y[j, r], ref))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fci_lockstep(ctx, prec):
    shape = (10, 11, 12)
    c = medium(shape, 9)
    o, g = make_ops(ctx, c, 15.0, 3, 1.0)
    poles = oracle_poles(o, 8, 1.0, 0.5, 8)
    cg = gpu_contour(g, poles, 8, 8)
    rng = np.random.default_rng(10)
    f = inputs(rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape), prec)
    opts = hf.default_opts(fp_steps=4, precision=64 if prec == "f64" else 32)
    out, st = hf.fci_apply(g, cg, dev(f), opts)
    out = host(out)
    assert st["fp_steps"] == 8 * 3 * 4
    for r in range(3):
        ref = OF.fci(o, f[r], poles, steps=4)
        e, tol = relmax(out[r], ref), fci_tol(prec, o, poles, 8, 4, f[r])
        assert e <= tol, (r, e, tol)
    # chunking the poles changes only the order of the step size's sums
    opts.pole_batch = 3
    out2, _ = hf.fci_apply(g, cg, dev(f), opts)
    assert relmax(host(out2), out) <= (1e-14 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("max_steps", [1, 2])
def test_fci_adaptive_stops_after_step_one(ctx, prec, max_steps):
    # adaptive FCI where every pole stops after step one (max_steps 1) or after at most one
    # later step: the quadrature combine must take those poles' iterate from y1, which step
    # one writes instead of y; a zero right-hand side stops at the first test as well
    shape = (10, 11, 12)
    c = medium(shape, 19)
    o, g = make_ops(ctx, c, 15.0, 3, 1.0)
    poles = oracle_poles(o, 8, 1.0, 0.5, 8)
    cg = gpu_contour(g, poles, 8, 8)
    rng = np.random.default_rng(12)
    f = inputs(rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape), prec)
    f[1] = 0.0
    opts = hf.default_opts(fp_steps=0, fp_reduce=5.0, fp_max_steps=max_steps,
                           precision=64 if prec == "f64" else 32)
    out, st = hf.fci_apply(g, cg, dev(f), opts)
    out = host(out)
    for r in (0, 2):
        ref = OF.fci(o, f[r], poles, reduce=5.0, m_max=max_steps)
        e, tol = relmax(out[r], ref), fci_tol(prec, o, poles, 8, max_steps, f[r])
        assert e <= tol, (r, e, tol)
    assert np.abs(out[1]).max() == 0.0


def test_solve_lockstep_fp64(ctx):
    wl = W.config_constant_32(n=16)
    o, g = make_ops(ctx, wl.c, wl.omega, wl.damp_cells, wl.damp_rho2)
    poles = oracle_poles(o, 8, 1.0, 0.5, 8)
    cg = gpu_contour(g, poles, 8, 8)
    f = wl.rhs[0]
    # one cycle deep enough for every width of the fused CGS2 passes (up to 25 basis
    # vectors); several restarts
    for m, its in [(30, 24), (4, 10)]:
        opts = hf.default_opts(fp_steps=3, tol=0.0, max_it=its, restart=m)
        u, st = hf.solve(g, cg, dev(f[None]), opts=opts)
        uo, info = OF.solve(o, f, poles, m=m, tol=0.0, max_it=its, steps=3)
        assert st["its"] == info["its"] == its
        assert relmax(host(u)[0], uo) <= 1e-10, relmax(host(u)[0], uo)


def residual(o, u, f):
    A = o.assemble()
    return np.linalg.norm(o.s * f.ravel() - A @ u.ravel()) / np.linalg.norm(o.s * f.ravel())


@pytest.mark.parametrize("prec", [64, 32])
def test_solve_config_constant_32(ctx, prec):
    wl = W.config_constant_32(n=32)
    o, g = make_ops(ctx, wl.c, wl.omega, wl.damp_cells, wl.damp_rho2)
    cg = hf.Contour(g, 8, 1.0, 0.5, 8)
    opts = hf.default_opts(tol=1e-8, precision=prec, max_it=300)
    u, st = hf.solve(g, cg, dev(wl.rhs[0][None]), opts=opts)
    u = host(u)[0]
    assert st["status"] == "HFCI_OK"
    assert st["final_relres"] <= 1e-8
    assert residual(o, u, wl.rhs[0]) <= 1.05e-8  # checked by the oracle's assembled matrix


def test_mixed_precision_matches_fp64_solution(ctx):
    # FP32 sweeps inside FP64 FGMRES: the Krylov wrapper refines to FP64 accuracy, so the
    # mixed solution converged to 1e-10 agrees with the FP64 one to better than 1e-6
    wl = W.config_grf_96(n=24, nrhs=2)
    o, g = make_ops(ctx, wl.c, wl.omega, wl.damp_cells, wl.damp_rho2)
    cg = hf.Contour(g, 12, 1.0, 0.5, 8)
    f = dev(np.stack(wl.rhs))
    u64, s64 = hf.solve(g, cg, f, opts=hf.default_opts(tol=1e-11, precision=64, max_it=400))
    u32, s32 = hf.solve(g, cg, f, opts=hf.default_opts(tol=1e-10, precision=32, max_it=400))
    u64, u32 = host(u64), host(u32)
    for r in range(2):
        assert residual(o, u32[r], wl.rhs[r]) <= 1.05e-10
        assert residual(o, u64[r], wl.rhs[r]) <= 1.05e-11
        assert relmax(u32[r], u64[r]) <= 1e-6


def test_identity_preconditioner_is_gmres(ctx):
    shape = (6, 6, 6)
    c = medium(shape, 11)
    o, g = make_ops(ctx, c, 6.0, 2, 1.0)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    opts = hf.default_opts(precond=0, tol=0.0, max_it=7)
    u, st = hf.solve(g, None, dev(f[None]), opts=opts)
    from oracle import krylov as K
    uo = K.gmres(lambda v: o.apply(v).ravel(), o.s * f.ravel(), 7)
    assert relmax(host(u)[0].ravel(), uo) <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_size_apply_every_point(ctx, prec):
    # 256^3, the size the benchmark times, every point against the oracle's stencil
    wl_c = W.layered_medium(256, seed=0)
    omega = W.omega_for_ppw(float(wl_c.min()), 256, 8.0)
    g = hf.Operator(ctx, dev(wl_c), 1.0 / 256, omega, 8, 1.0)
    o = OO.Operator(wl_c, omega, 8, 1.0, h=1.0 / 256)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    gen = torch.Generator(device="cuda").manual_seed(13)
    x = (torch.randn(256, 256, 256, dtype=torch.float64, device="cuda", generator=gen)
         + 1j * torch.randn(256, 256, 256, dtype=torch.float64, device="cuda", generator=gen)).to(dt)
    shift = -7.1 + 0.5j
    y = host(hf.apply(g, x, shift)).astype(np.complex128)
    xh = host(x).astype(np.complex128)
    check_apply(y, o, xh, shift, prec)


def test_error_paths(ctx):
    c = medium((4, 4, 4), 14)
    o, g = make_ops(ctx, c, 5.0, 1, 1.0)
    for J in (-1, 257):  # J = 0 asks the library's rule for J
        with pytest.raises(hf.HfciError) as e:
            hf.Contour(g, J, 1.0, 0.5, 8)
        assert e.value.status == -1
    with pytest.raises(hf.HfciError) as e:  # a pole inside the damping band
        hf.Contour(g, 1, 1.0, 0.5, 4, z=[-0.5j], sigma=[1.0])
    assert e.value.status == -4
    bad = dev(-np.ones((4, 4, 4)))
    with pytest.raises(hf.HfciError):
        hf.Operator(ctx, bad, 0.25, 5.0, 1, 1.0)
    x = torch.zeros((4, 4, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(hf.HfciError):
        hf.apply(g, x, 0.0, out=x)  # overlapping buffers
    cg = hf.Contour(g, 4, 1.0, 0.5, 4)
    f = dev(np.ones((1, 4, 4, 4), dtype=complex))
    u, st = hf.solve(g, cg, f, opts=hf.default_opts(tol=1e-14, max_it=2))
    assert st["status"] == "HFCI_W_NOCONV" and st["its"] == 2


# ---- uneven batches (several operators in one launch per factor) ----

def _batch_instances(ctx, shapes, q, seed=50):
    out = []
    for k, shape in enumerate(shapes):
        c = medium(shape, seed + k, 1.0, 2.5)
        o, g = make_ops(ctx, c, 10.0 + 2.0 * k, 2 + (k % 2), 1.0)
        J = 4 + 2 * (k % 2)
        poles = oracle_poles(o, J, 1.0, 0.5, q)
        out.append((o, g, poles, gpu_contour(g, poles, J, q), J))
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("q", [2, 3, 4, 5, 8])
def test_shifted_solve_batch_matches_oracle(ctx, prec, q):
    # one launch per factor (two per pass for q >= 3) over every instance's poles: step one
    # with a lone first factor (odd q - 1) or all pairs, later steps with a trailing single
    # (odd q) or all pairs; the adaptive run stops systems at different steps, so the
    # pipelined steps launch past the live rows of the rebuilt work tables
    shapes = [(9, 12, 20), (16, 16, 16), (7, 10, 70), (12, 5, 9)]
    inst = _batch_instances(ctx, shapes, q)
    rng = np.random.default_rng(51)
    fs = [inputs(rng.standard_normal(sh) + 1j * rng.standard_normal(sh), prec) for sh in shapes]
    dt = torch.complex128 if prec == "f64" else torch.complex64
    ys, st = hf.shifted_solve_batch([i[1] for i in inst], [i[3] for i in inst], [dev(f).to(dt) for f in fs], steps=3)
    for (o, g, poles, cg, J), y, f, s in zip(inst, ys, fs, st):
        assert np.all(s == 3)
        y = host(y)
        Am = lambda v, sh, o=o: o.apply(v, sh)
        for j, p in enumerate(poles):
            ref, _ = OFP.fixed_point_solve(Am, f, p.z, p.z0, p.delta, q, steps=3)
            e, tol = relmax(y[j], ref), fp_tol(prec, o, p, q, 3, f, ref)
            assert e <= tol, (j, e, tol)
    if prec == "f64":
        # adaptive stopping: every (instance, pole) stops at the oracle's step with the oracle's iterate
        ys, st = hf.shifted_solve_batch([i[1] for i in inst], [i[3] for i in inst], [dev(f) for f in fs],
                                        reduce=5.0, max_steps=80)
        counts = set()
        for (o, g, poles, cg, J), y, f, s in zip(inst, ys, fs, st):
            y = host(y)
            Am = lambda v, sh, o=o: o.apply(v, sh)
            for j, p in enumerate(poles):
                ref, hist = OFP.fixed_point_solve(Am, f, p.z, p.z0, p.delta, q, reduce=5.0, m_max=80)
                assert s[j] == len(hist) - 1
                assert relmax(y[j], ref) <= 1e-12
                counts.add(int(s[j]))
        assert len(counts) >= 3


def test_solve_batch_equals_single_solves(ctx):
    # FP64 sweeps with a fixed step count: the batch runs the same arithmetic per point as
    # the single-operator path, so every instance's FGMRES history and solution agree
    shapes = [(12, 12, 12), (10, 14, 18), (16, 9, 11)]
    q = 4
    inst = _batch_instances(ctx, shapes, q, seed=60)
    rng = np.random.default_rng(61)
    fs = [dev(rng.standard_normal(sh) + 1j * rng.standard_normal(sh)) for sh in shapes]
    opts = hf.default_opts(precision=64, tol=1e-9, max_it=200, fp_steps=2)
    us, sts, status = hf.solve_batch([i[1] for i in inst], [i[3] for i in inst], fs, opts=opts)
    assert status == "HFCI_OK"
    for (o, g, poles, cg, J), u, f, stb in zip(inst, us, fs, sts):
        u1, st1 = hf.solve(g, cg, f[None], opts=opts)
        assert stb["its"] == st1["its"]
        assert relmax(host(u), host(u1)[0]) <= 1e-11
        # the oracle's FP64 residual of the returned solution
        b = o.s * host(f)
        assert np.linalg.norm(b - o.apply(host(u))) / np.linalg.norm(b) <= 1e-8


def test_solve_batch_mixed_precision_uneven_sizes(ctx):
    import workloads as W
    wls = W.config_uneven_batch(count=5, seed=3, sizes=(12, 16, 20, 24))
    ops, cons, fs, os_ = [], [], [], []
    for wl in wls:
        g = hf.Operator(ctx, dev(wl.c), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
        ops.append(g)
        cons.append(hf.Contour(g, wl.n_poles, 1.0, 0.25, 8))
        fs.append(dev(wl.rhs[0]))
        os_.append(OO.Operator(wl.c, wl.omega, wl.damp_cells, wl.damp_rho2))
    opts = hf.default_opts(precision=32, tol=1e-7, max_it=400)
    us, sts, status = hf.solve_batch(ops, cons, fs, opts=opts)
    assert status == "HFCI_OK"
    assert sts[0]["fp_steps"] > 0
    for o, u, f, st in zip(os_, us, fs, sts):
        b = o.s * host(f)
        r = np.linalg.norm(b - o.apply(host(u))) / np.linalg.norm(b)
        assert r <= 1e-7 * 1.01 and st["final_relres"] <= 1e-7


def test_batch_error_paths(ctx):
    o, g = make_ops(ctx, medium((6, 6, 6), 1), 9.0, 1, 0.5)
    o2, g2 = make_ops(ctx, medium((6, 6, 7), 2), 9.0, 1, 0.5)
    poles = oracle_poles(o, 4, 1.0, 0.5, 4)
    c1 = gpu_contour(g, poles, 4, 4)
    c8 = hf.Contour(g2, 4, 1.0, 0.5, 8)
    f = dev(np.ones((6, 6, 6), dtype=np.complex128))
    f2 = dev(np.ones((6, 6, 7), dtype=np.complex128))
    with pytest.raises(hf.HfciError):  # q differs across the batch
        hf.solve_batch([g, g2], [c1, c8], [f, f2])
    with pytest.raises(hf.HfciError):  # contour of another operator
        hf.solve_batch([g, g2], [c8, c1], [f, f2])


# ---- fixed-point steps replayed from captured HIP graphs ----

@pytest.mark.parametrize("prec,kern,fused,fixed,q", [(64, 1, 0, 0, 8), (32, 1, 0, 0, 8), (32, 1, 1, 0, 8),
                                                    (64, 1, 1, 2, 8), (32, 1, 0, 3, 8), (32, 3, 2, 0, 10),
                                                    (32, 3, 2, 2, 10)])
def test_graph_replay_equals_direct_launches(ctx, prec, kern, fused, fixed, q):
    # each FCI application replays the captured step graph many times, with the eager
    # Arnoldi work of FGMRES between replays; every replay must give exactly what direct
    # launches give, so the whole solve is bitwise identical (kern 3 with fuse 2 and
    # q = 10: later steps of 2 + 3 + 3 + 2 factors per pass)
    wl = W.config_grf_96(n=20, nrhs=2)
    g = hf.Operator(ctx, dev(wl.c), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    g.set_tune(prec, kern, 8, 2, 0, fused)
    c = hf.Contour(g, 8, 1.0, 0.25, q)
    f = dev(np.stack(wl.rhs))
    res = {}
    for gr in (0, 1, 1):  # the second graph run reuses the cached instantiation
        o = hf.default_opts(precision=prec, tol=1e-8, max_it=120, graphs=gr, fp_steps=fixed)
        u, st = hf.solve(g, c, f, opts=o)
        res.setdefault(gr, []).append((host(u), st))
    u0, st0 = res[0][0]
    for u1, st1 in res[1]:
        assert st1["its"] == st0["its"] and st1["matvecs"] == st0["matvecs"]
        assert np.array_equal(u1, u0)
    # and the replayed solve is a solve: the oracle's FP64 residual of every right-hand side
    # is at most the tolerance, or, if the iteration cap came first, the residual FGMRES
    # reported (the largest over the right-hand sides)
    o = OO.Operator(wl.c, wl.omega, wl.damp_cells, wl.damp_rho2)
    u1, st1 = res[1][-1]
    for r in range(2):
        b = o.s * wl.rhs[r]
        rr = np.linalg.norm(b - o.apply(u1[r])) / np.linalg.norm(b)
        assert rr <= max(1.01e-8, 1.01 * st1["final_relres"]), (r, rr, st1["final_relres"])
