"""The benchmark's own launch path against the FP64 oracle, at full size (needs an MI355X).

The pair kernel (two factors of a fixed-point step per pass over HBM) renumbers its
workgroups into per-XCD slabs only when a system has at least 64 tiles and the count is
a multiple of 8.  At 256^3 the fused shape (1, 8, 2, 64, 1) gives 4 x 22 x 4 = 352 tiles
per system.  The small-grid tests never reach that mapping.  These tests do:
  * every pair-kernel kind on a grid of 2 x 4 x 8 = 64 ragged tiles per system:
    plain middle pairs, the residual pair (first of a later step), the y1-adding pair
    (last of a later step), the pair reading f (step one when q - 1 is even) and the
    dual-output pair (step one as the only step), with the systems of a launch taken
    one, three or four at a time tile by tile (sg), and adaptive stopping under groups;
  * 256^3 lockstep fixed-point steps at the benchmark's shape, 2 poles x 2 sources, over
    the full grid;
  * 256^3 and 96^3 solves to 1e-6, the 256^3 one with the autotuner's shape as the
    benchmark picks it, each residual recomputed in FP64 by the oracle.
Comparisons are element by element (relmax); the FP32 bars are derived in
tests/fp32_bounds.py.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fci as OF
from oracle import fixed_point as OFP
from oracle import operator as OO
from tests.fp32_bounds import ROUNDINGS, SAFETY, U32, fixed_point_bar, relmax, round32, stencil_absrow

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


def pair_tiles(shape, cz):
    nz, ny, nx = shape
    return -(-nx // 64) * -(-ny // 12) * -(-nz // cz)


def tol_of(prec, o, p, q, steps, f, ref):
    if prec == "f64":
        return 1e-12
    return fixed_point_bar(p, q, steps, o.rectangle(), stencil_absrow(o.s_h2, o.kappa, o.rho2),
                           np.abs(f).max() / np.abs(ref).max())


# (q, steps): q = 8 with 3 steps runs the fan-out, plain pairs, the residual pair and the
# y1 pair; q = 8 with 1 step ends step one with the dual-output pair; q = 5 and q = 7 start
# step one with the pair that reads f (q - 1 even) and end later steps with a lone factor
KIND_CASES = [(8, 3), (8, 1), (5, 2), (7, 2)]


SLAB_SHAPE = (60, 45, 100)  # ragged in x (64 + 36), y (3 x 12 + 9) and z (7 x 8 + 4)


def slab_operator(ctx, seed=71):
    assert pair_tiles(SLAB_SHAPE, 8) == 64  # >= 64 and a multiple of 8: XCD slabs on
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 3.0, size=SLAB_SHAPE)
    h = 1.0 / 60
    return OO.Operator(c, 20.0, 3, 1.0, h=h), hf.Operator(ctx, dev(c), h, 20.0, 3, 1.0), rng


# sg = 3 over the 8 systems of a launch: groups of 3, 3 and a ragged 2; kern 2 is the
# complex64 pair kernel whose streams go straight into LDS (pd 2: two planes ahead, pd 3:
# four)
@pytest.mark.parametrize("q,steps", KIND_CASES)
@pytest.mark.parametrize("prec,kern,pd,sg", [("f64", 1, 2, 1), ("f64", 1, 3, 1), ("f64", 1, 2, 3), ("f64", 1, 3, 4),
                                             ("f32", 1, 2, 1), ("f32", 1, 3, 1), ("f32", 1, 2, 3), ("f32", 1, 3, 4),
                                             ("f32", 2, 2, 1), ("f32", 2, 3, 1), ("f32", 2, 2, 3), ("f32", 2, 3, 4)])
def test_pair_kinds_with_xcd_slabs(ctx, q, steps, prec, kern, pd, sg):
    shape = SLAB_SHAPE
    o, g, rng = slab_operator(ctx)
    pr = 64 if prec == "f64" else 32
    g.set_tune(pr, kern, 8, pd, 8, 1, sg)
    assert g.get_tune(pr) == (kern, 8, pd, 8, 1, sg)
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, q)
    cg = hf.Contour(g, 4, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    f = rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape)
    if prec == "f32":
        f = round32(f)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    y, st = hf.shifted_solve(g, cg, dev(f).to(dt), steps=steps)
    y = host(y).astype(np.complex128)
    assert np.all(st == steps)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, steps=steps)
            e, tol = relmax(y[j, r], ref), tol_of(prec, o, p, q, steps, f[r], ref)
            assert e <= tol, (j, r, e, tol)


@pytest.mark.parametrize("sg", [1, 3])
def test_adaptive_stops_with_system_groups(ctx, sg):
    # adaptive stopping at the XCD-slab geometry: the launches after each test are sized for
    # the systems active one test earlier, so the compacted list ends in -1 entries that a
    # group of systems must skip; rhs 1 is zero (stops at step 0), rhs 2 is small
    o, g, rng = slab_operator(ctx, seed=73)
    g.set_tune(64, 1, 8, 2, 8, 1, sg)
    q = 8
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, q)
    cg = hf.Contour(g, 4, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    f = rng.standard_normal((3,) + SLAB_SHAPE) + 1j * rng.standard_normal((3,) + SLAB_SHAPE)
    f[1] = 0.0
    f[2] *= 1e-3
    y, st = hf.shifted_solve(g, cg, dev(f), reduce=5.0, max_steps=60)
    y = host(y)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        assert st[j, 1] == 0 and np.all(y[j, 1] == 0)
        for r in (0, 2):
            ref, hist = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, reduce=5.0, m_max=60)
            assert st[j, r] == len(hist) - 1, (j, r, st[j, r], len(hist) - 1)
            assert relmax(y[j, r], ref) <= 1e-12, (j, r, relmax(y[j, r], ref))
    assert len(set(int(v) for v in st[:, 0])) > 1  # the poles stop at different steps


@pytest.mark.parametrize("q,steps", KIND_CASES + [(3, 3)])
@pytest.mark.parametrize("pd,cz", [(2, 8), (3, 8), (2, 0), (3, 5)])
def test_streams_into_lds_match_the_register_pair_kernel(ctx, q, steps, pd, cz):
    # kern 2 gives every point the same arithmetic as kern 1, up to how the compiler fuses
    # multiply-adds: each is within the FP32 product-form bar of the oracle, so the two are
    # within twice that bar of each other, pole by pole, every kind of pair launch; z-chunks
    # of 8 planes (several per column, ragged last), the grid's own choice and 5
    o, g, rng = slab_operator(ctx, seed=75)
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, q)
    cg = hf.Contour(g, 4, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    fh = round32(rng.standard_normal((2,) + SLAB_SHAPE) + 1j * rng.standard_normal((2,) + SLAB_SHAPE))
    f = dev(fh).to(torch.complex64)
    out = {}
    for kern in (1, 2):
        g.set_tune(32, kern, 8, pd, cz, 1, 2)
        y, st = hf.shifted_solve(g, cg, f, steps=steps)
        assert np.all(st == steps)
        out[kern] = host(y).astype(np.complex128)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, fh[r], p.z, p.z0, p.delta, q, steps=steps)
            bar = tol_of("f32", o, p, q, steps, fh[r], ref)
            scale = np.abs(ref).max()
            assert np.abs(out[2][j, r] - out[1][j, r]).max() <= 2 * bar * scale, (j, r)
            assert relmax(out[2][j, r], ref) <= bar, (j, r)


TALL_SHAPE = (90, 70, 100)  # ragged in x (64 + 36), y (28 + 28 + 14) and z (11 x 8 + 2)


def tall_tiles(shape, cz):
    nz, ny, nx = shape
    return -(-nx // 64) * -(-ny // 28) * -(-nz // cz)


@pytest.mark.parametrize("q,steps", KIND_CASES + [(3, 3)])
@pytest.mark.parametrize("cz,sg", [(8, 3), (0, 1)])
def test_tall_tiles_match_the_oracle_and_the_register_kernel(ctx, q, steps, cz, sg):
    # kern 3: the pairs without an extra stream on 64 x 28 tiles (the residual and y1 pairs
    # as kern 2), at a geometry whose tall tiles split into XCD slabs (72 per system with
    # cz 8), groups of systems taken sg at a time, every kind of pair launch; each result
    # within the FP32 bar of the oracle and within twice it of the register pair kernel
    assert tall_tiles(TALL_SHAPE, 8) == 72
    rng = np.random.default_rng(81)
    c = rng.uniform(1.0, 3.0, size=TALL_SHAPE)
    h = 1.0 / 100
    o, g = OO.Operator(c, 30.0, 3, 1.0, h=h), hf.Operator(ctx, dev(c), h, 30.0, 3, 1.0)
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, q)
    cg = hf.Contour(g, 4, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    fh = round32(rng.standard_normal((2,) + TALL_SHAPE) + 1j * rng.standard_normal((2,) + TALL_SHAPE))
    f = dev(fh).to(torch.complex64)
    out = {}
    for kern in (1, 3):
        g.set_tune(32, kern, 8, 2, cz, 1, sg)
        assert g.get_tune(32) == (kern, 8, 2, cz, 1, sg)
        y, st = hf.shifted_solve(g, cg, f, steps=steps)
        assert np.all(st == steps)
        out[kern] = host(y).astype(np.complex128)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, fh[r], p.z, p.z0, p.delta, q, steps=steps)
            bar = tol_of("f32", o, p, q, steps, fh[r], ref)
            assert relmax(out[3][j, r], ref) <= bar, (j, r, relmax(out[3][j, r], ref), bar)
            assert np.abs(out[3][j, r] - out[1][j, r]).max() <= 2 * bar * np.abs(ref).max(), (j, r)


def trip_tiles(shape, cz):
    nz, ny, nx = shape
    return -(-nx // 64) * -(-ny // 18) * -(-nz // cz)


def launch_plan(count, kind_first, kind_last, pairs, single_first, triples):
    """(first factor, width, kind bits) of the launches of `count` factors, as the library
    plans them: pairs (an odd count leaves one single, first or last), then with triples
    each run of middle pairs (kind 0) split again into threes and at most two pairs."""
    v, j = [], 0
    while j < count:
        lone = single_first and j == 0 and count % 2 == 1
        w = 2 if (pairs and j + 1 < count and not lone) else 1
        kind = (kind_first if j == 0 else 0) | (kind_last if j + w == count else 0)
        v.append((j, w, kind))
        j += w
    if not triples:
        return v
    out, i = [], 0
    while i < len(v):
        if v[i][1] != 2 or v[i][2] != 0:
            out.append(v[i])
            i += 1
            continue
        j = i
        while j < len(v) and v[j][1] == 2 and v[j][2] == 0:
            j += 1
        m = 2 * (j - i)
        npair = 0 if m % 3 == 0 else (1 if m % 3 == 2 else 2)
        k = v[i][0]
        for _ in range((m - 2 * npair) // 3):
            out.append((k, 3, 0))
            k += 3
        for _ in range(npair):
            out.append((k, 2, 0))
            k += 2
        i = j
    return out


# (q, steps): the run of middle pairs of a later step (q - 4 factors, q - 3 for odd q) and
# step one's run of pairs are split into threes and at most two pairs (q = 8: later steps
# 2 + 2 + 2 + 2, step one 1 + 3 + 3; q = 10: later 2 + 3 + 3 + 2); q = 8 with one step ends
# step one with the dual-output pair, which is not regrouped
TRIP_CASES = [(8, 3), (8, 1), (9, 3), (10, 3), (11, 2), (12, 2), (13, 2), (7, 2), (6, 3)]


@pytest.mark.parametrize("q,steps", TRIP_CASES)
@pytest.mark.parametrize("cz,sg", [(4, 3), (0, 1)])
def test_three_factor_passes_match_the_oracle(ctx, q, steps, cz, sg):
    # kern 3 with fuse 2: the middle factors three per pass on 64 x 18 tiles and z-chunks of
    # 2 cz planes, at a geometry whose tiles split into XCD slabs (96 per system with cz 4),
    # ragged in x, y and z, systems taken sg at a time; each result within the FP32 bar of
    # the oracle and within twice it of the same shape with pairs only (fuse 1)
    assert trip_tiles(TALL_SHAPE, 2 * 4) == 96
    rng = np.random.default_rng(83)
    c = rng.uniform(1.0, 3.0, size=TALL_SHAPE)
    h = 1.0 / 100
    o, g = OO.Operator(c, 30.0, 3, 1.0, h=h), hf.Operator(ctx, dev(c), h, 30.0, 3, 1.0)
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, q)
    cg = hf.Contour(g, 4, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    fh = round32(rng.standard_normal((2,) + TALL_SHAPE) + 1j * rng.standard_normal((2,) + TALL_SHAPE))
    f = dev(fh).to(torch.complex64)
    out = {}
    for fuse in (1, 2):
        g.set_tune(32, 3, 8, 2, cz, fuse, sg)
        assert g.get_tune(32) == (3, 8, 2, cz, fuse, sg)
        ctx.profile(True)
        y, st = hf.shifted_solve(g, cg, f, steps=steps)
        prof = ctx.profile_read()
        ctx.profile(False)
        assert np.all(st == steps)
        out[fuse] = host(y).astype(np.complex128)
        # launches of three factors: step one's plan once, a later step's plan per later step
        # (a fixed count of one step ends step one with the dual-output pair)
        first = launch_plan(max(q - 1, 1), 8, 4 if steps == 1 else 0, True, True, fuse == 2)
        later = launch_plan(q, 1, 2, q >= 3, False, fuse == 2)
        want = sum(w == 3 for _, w, _ in first) + (steps - 1) * sum(w == 3 for _, w, _ in later)
        assert prof["fp_stage_triple"]["launches"] == want, (fuse, want, prof["fp_stage_triple"])
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, fh[r], p.z, p.z0, p.delta, q, steps=steps)
            bar = tol_of("f32", o, p, q, steps, fh[r], ref)
            assert relmax(out[2][j, r], ref) <= bar, (j, r, relmax(out[2][j, r], ref), bar)
            assert np.abs(out[2][j, r] - out[1][j, r]).max() <= 2 * bar * np.abs(ref).max(), (j, r)


@pytest.mark.parametrize("kern,fuse,q", [(2, 1, 8), (3, 1, 8), (3, 2, 10)])
def test_streams_into_lds_adaptive(ctx, kern, fuse, q):
    # adaptive stopping in FP32 with kerns 2 and 3 (and three factors per pass): each system
    # stops within one step of the oracle's count (an FP32 residual can land on the other
    # side of the threshold), its iterate is the oracle's after the steps it took, within
    # the FP32 bar, and it meets the stopping rule; a zero right-hand side stops at once
    o, g, rng = slab_operator(ctx, seed=79)
    g.set_tune(32, kern, 8, 2, 8, fuse, 3)
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, q)
    cg = hf.Contour(g, 4, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    fh = round32(rng.standard_normal((3,) + SLAB_SHAPE) + 1j * rng.standard_normal((3,) + SLAB_SHAPE))
    fh[1] = 0.0
    y, st = hf.shifted_solve(g, cg, dev(fh).to(torch.complex64), reduce=5.0, max_steps=40)
    y = host(y).astype(np.complex128)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        assert st[j, 1] == 0 and np.all(y[j, 1] == 0)
        for r in (0, 2):
            _, hist = OFP.fixed_point_solve(Am, fh[r], p.z, p.z0, p.delta, q, reduce=5.0, m_max=40)
            k = int(st[j, r])
            assert abs(k - (len(hist) - 1)) <= 1, (j, r, k, len(hist) - 1)
            ref, _ = OFP.fixed_point_solve(Am, fh[r], p.z, p.z0, p.delta, q, steps=k)
            e, tol = relmax(y[j, r], ref), tol_of("f32", o, p, q, k, fh[r], ref)
            assert e <= tol, (j, r, e, tol)
            # a system that stopped before the cap of 40 steps met the rule; the test decided
            # on the FP32 residual the kernel formed, whose error per point is at most
            # ROUNDINGS u (|f| + |A - z| |y|): in the 2-norm at most that times
            # (||f|| + absrow ||y||), |A - z| being symmetric with row sums <= absrow (with
            # q = 10 the pole nearest the origin reaches the cap, in the oracle too)
            if k < 40:
                rn = np.linalg.norm(fh[r] - o.apply(y[j, r], p.z))
                absrow = stencil_absrow(o.s_h2, o.kappa, o.rho2)(p.z)
                slack = SAFETY * ROUNDINGS * U32 * (np.linalg.norm(fh[r]) + absrow * np.linalg.norm(y[j, r]))
                assert rn <= np.linalg.norm(fh[r]) / 5 + slack, (j, r, rn, np.linalg.norm(fh[r]) / 5, slack)


def test_streams_into_lds_need_an_even_nx(ctx):
    # an odd nx (pairs of x-neighbours would straddle rows) falls back to kern 1's kernel,
    # for the three-factor shape too (its plan keeps pairs)
    shape = (20, 26, 67)
    rng = np.random.default_rng(77)
    c = rng.uniform(1.0, 3.0, size=shape)
    o = OO.Operator(c, 14.0, 3, 1.0, h=1 / 20)
    g = hf.Operator(ctx, dev(c), 1 / 20, 14.0, 3, 1.0)
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, 8)
    cg = hf.Contour(g, 4, 1.0, 0.5, 8, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    f = dev(round32(rng.standard_normal((1,) + shape) + 1j * rng.standard_normal((1,) + shape))).to(torch.complex64)
    res = []
    for kern, fuse in ((1, 1), (2, 1), (3, 2)):
        # kern 2 and kern 3 with three factors per pass both run kern 1's pairs here
        g.set_tune(32, kern, 8, 2, 0, fuse)
        res.append(host(hf.shifted_solve(g, cg, f, steps=2)[0]))
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])
    with pytest.raises(hf.HfciError):  # a complex64 kernel only
        g.set_tune(64, 2, 8, 2, 0, 1)


def layered(n, nrhs):
    return W.config_layered_256(n=n, nrhs=nrhs)


@pytest.mark.parametrize("kern,pd,fuse,q", [(1, 2, 1, 8), (2, 2, 1, 8), (2, 3, 1, 8), (3, 2, 1, 8), (3, 2, 2, 10)])
def test_headline_shape_lockstep_256(ctx, kern, pd, fuse, q):
    # the benchmark's workload and fused complex64 shapes: 2 of its 16 poles (the one
    # nearest the origin, the slowest, and one across the contour) x 2 of its point
    # sources, two fixed-point steps (step one, then residual / middle / y1 pairs; with
    # fuse 2 and q = 10 step one runs 1 + 3 + 3 + 2 factors per pass and the later step
    # 2 + 3 + 3 + 2)
    wl = layered(256, 2)
    o = OO.Operator(wl.c, wl.omega, wl.damp_cells, wl.damp_rho2)
    g = hf.Operator(ctx, dev(wl.c), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    g.set_tune(32, kern, 8, pd, 64, fuse, 2)
    assert pair_tiles(o.shape, 64) == 352 and trip_tiles(o.shape, 2 * 64) == 120
    allp = OF.pole_parameters(o, 16, 1.0, 0.25, q)
    poles = [allp[0], allp[8]]
    cg = hf.Contour(g, 2, 1.0, 0.25, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    f = round32(np.stack(wl.rhs))
    y, st = hf.shifted_solve(g, cg, dev(f).to(torch.complex64), steps=2)
    assert np.all(st == 2)
    y = host(y)
    Am = lambda v, sh: o.apply(v, sh)
    for j, p in enumerate(poles):
        for r in range(2):
            ref, _ = OFP.fixed_point_solve(Am, f[r], p.z, p.z0, p.delta, q, steps=2)
            e, tol = relmax(y[j, r].astype(np.complex128), ref), tol_of("f32", o, p, q, 2, f[r], ref)
            assert e <= tol, (j, r, e, tol)
            del ref


def oracle_relres(o, f, u):
    b = o.s * f
    return float(np.linalg.norm(b - o.apply(u)) / np.linalg.norm(b))


def test_headline_mixed_solve_256(ctx):
    # the benchmark's solve with one of its sources: the autotuner's complex64 shape,
    # FP32 sweeps in FP64 FGMRES(30), to 1e-6; the oracle recomputes the FP64 residual
    wl = layered(256, 1)
    o = OO.Operator(wl.c, wl.omega, wl.damp_cells, wl.damp_rho2)
    g = hf.Operator(ctx, dev(wl.c), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    best, _ = g.autotune(32, 2)
    cg = hf.Contour(g, 16, 1.0, 0.25, 8)
    u, st = hf.solve(g, cg, dev(wl.rhs[0][None]), opts=hf.default_opts(precision=32, tol=1e-6, max_it=1000))
    assert st["status"] == "HFCI_OK", st
    assert st["final_relres"] <= 1e-6
    assert oracle_relres(o, wl.rhs[0], host(u)[0]) <= 1e-6 * 1.01


@pytest.mark.parametrize("prec", [32, 64])
def test_grf_96_four_sources(ctx, prec):
    # the 96^3 random-field configuration: 12 poles, 4 Gaussian right-hand sides, plain FP64
    # and mixed precision to 1e-6, every residual recomputed by the oracle
    wl = W.config_grf_96()
    o = OO.Operator(wl.c, wl.omega, wl.damp_cells, wl.damp_rho2)
    g = hf.Operator(ctx, dev(wl.c), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    g.set_tune(prec, 1, 8, 2, 0, 1)
    cg = hf.Contour(g, 12, 1.0, 0.25, 8)
    f = np.stack(wl.rhs)
    u, st = hf.solve(g, cg, dev(f), opts=hf.default_opts(precision=prec, tol=1e-6, max_it=1000))
    assert st["status"] == "HFCI_OK", st
    u = host(u)
    for r in range(len(wl.rhs)):
        assert oracle_relres(o, f[r], u[r]) <= 1e-6 * 1.01, r
