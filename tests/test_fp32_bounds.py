"""The FP32 tolerances of the GPU parity tests hold for an FP32 evaluation on the CPU.

A NumPy complex64 evaluation rounds every operation to binary32, as the kernels do,
though in another order.  It must stay inside apply_bound() for one stencil product and
inside fixed_point_bar() for product-form fixed-point steps, each against the FP64
oracle.  A tolerance model that failed here would be too tight for the kernels too.
"""
import numpy as np
import pytest

from oracle import fci as OF
from oracle import fixed_point as OFP
from oracle import operator as OO
from tests.fp32_bounds import (_factors, apply_bound, fixed_point_bar, relmax, round32, stencil_absrow,
                               step_growth)


def stencil32(x, kappa, damp, s_h2, shift):
    """(A - shift) x with every operation in complex64."""
    x = x.astype(np.complex64)
    nb = np.zeros_like(x)
    nb[1:] += x[:-1]
    nb[:-1] += x[1:]
    nb[:, 1:] += x[:, :-1]
    nb[:, :-1] += x[:, 1:]
    nb[:, :, 1:] += x[:, :, :-1]
    nb[:, :, :-1] += x[:, :, 1:]
    d = (6.0 * s_h2 - kappa - 1j * damp - shift).astype(np.complex64)
    return d * x - np.complex64(s_h2) * nb


def medium(shape, seed):
    return np.random.default_rng(seed).uniform(1.0, 3.0, size=shape)


def test_relmax_is_elementwise():
    ref = np.ones(10000)
    a = ref.copy()
    a[17] += 0.03  # one point 3 % off: norm-wise 3e-4, element-wise 3e-2
    assert relmax(a, ref) == pytest.approx(0.03)
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref) < 1e-3


@pytest.mark.parametrize("seed", [1, 2])
def test_fp32_stencil_within_pointwise_bound(seed):
    c = medium((9, 11, 13), seed)
    o = OO.Operator(c, 9.0, 2, 0.8, h=1 / 9)
    rng = np.random.default_rng(seed + 10)
    x = round32(rng.standard_normal(o.shape) + 1j * rng.standard_normal(o.shape))
    shift = 0.37 - 1.21j
    ref = o.apply(x, shift)
    y = stencil32(x, o.kappa, o.damp, o.s_h2, shift).astype(np.complex128)
    bound = apply_bound(x, o.kappa, o.damp, o.s_h2, shift)
    assert np.all(np.abs(y - ref) <= bound)
    assert np.abs(y - ref).max() > 0  # the emulation really rounds


def product_form_steps32(o, f, p, q, steps):
    """Product-form fixed-point steps from y = 0 in complex64: y1 = the y1 chain applied
    to f, then y <- L chain(y) + y1."""
    (aL, bL), (aP, bP) = _factors(p.z, p.z0, p.delta, q)
    sh = lambda w: stencil32(w, o.kappa, o.damp, o.s_h2, p.z0)
    w = f.astype(np.complex64)
    for b in bP:
        w = np.complex64(aP) * sh(w) + np.complex64(b) * w
    y1 = w
    y = y1
    for _ in range(steps - 1):
        w = y
        for b in bL:
            w = np.complex64(aL) * sh(w) + np.complex64(b) * w
        y = w + y1
    return y.astype(np.complex128)


@pytest.mark.parametrize("q,steps", [(8, 3), (4, 2), (3, 4), (1, 3)])
def test_fp32_product_form_within_fixed_point_bar(q, steps):
    c = medium((8, 9, 10), 7)
    o = OO.Operator(c, 14.0, 2, 1.0, h=1 / 8)
    poles = OF.pole_parameters(o, 4, 1.0, 0.5, q)
    rng = np.random.default_rng(3)
    f = round32(rng.standard_normal(o.shape) + 1j * rng.standard_normal(o.shape))
    box = o.rectangle()
    absrow = stencil_absrow(o.s_h2, o.kappa, o.rho2)
    Am = lambda v, s: o.apply(v, s)
    for p in poles:
        ref, _ = OFP.fixed_point_solve(Am, f, p.z, p.z0, p.delta, q, steps=steps)
        y = product_form_steps32(o, f, p, q, steps)
        bar = fixed_point_bar(p, q, steps, box, absrow, np.abs(f).max() / np.abs(ref).max())
        err = relmax(y, ref)
        assert err <= bar, (q, steps, p.z, err, bar)
        assert bar < 5e-3  # the bar is a useful one, not a blanket


def test_growth_is_that_of_the_chain_not_of_the_factors():
    # Leja order keeps partial products small: the rounding growth of a degree-8 chain is
    # far below the product of its factors' absolute row sums
    c = medium((8, 8, 8), 5)
    o = OO.Operator(c, 14.0, 2, 1.0, h=1 / 8)
    p = OF.pole_parameters(o, 4, 1.0, 0.5, 8)[0]
    absrow = stencil_absrow(o.s_h2, o.kappa, o.rho2)
    gl, gp = step_growth(p.z, p.z0, p.delta, 8, o.rectangle(), absrow)
    (aL, bL), _ = _factors(p.z, p.z0, p.delta, 8)
    crude = np.prod([abs(aL) * absrow(p.z0) + abs(b) for b in bL])
    assert gl < crude / 20
