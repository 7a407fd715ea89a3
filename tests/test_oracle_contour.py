"""Pins of the oracle's contour quadrature (Sec. 2, Sec. 6.1-6.2)."""
import math

import numpy as np
import pytest

from conftest import load_golden
from oracle import contour as C
from oracle import operator as O


def test_printed_pole_sets_sec7():
    rows = load_golden("poles_sec7.txt")
    sets = {}
    for s, eps, j, re, im in rows:
        sets.setdefault(int(s), (eps, []))[1].append((int(j), re + 1j * im))
    assert len(sets) == 4
    for eps, entries in sets.values():
        z, _, _ = C.poles_and_weights(6, 0.1, eps, 0.9)
        for j, printed in entries:
            # two printed decimals, plus the paper's own rounding of the inputs
            assert abs(z[j - 1].real - printed.real) <= 0.011
            assert abs(z[j - 1].imag - printed.imag) <= 0.011


@pytest.mark.parametrize("J,t,eps,rho2", [(6, 0.1, 0.8, 0.9), (8, 1.0, 0.5, 1.0),
                                          (16, 1.0, 0.25, 1.0), (12, 0.5, 0.5, 1.3)])
def test_pole_invariants(J, t, eps, rho2):
    z, sigma, r = C.poles_and_weights(J, t, eps, rho2)
    assert np.all(z.real <= 1e-14)                       # not more indefinite than A
    im = z.imag
    assert np.all((im >= eps - 1e-12) | (im <= -eps - rho2 + 1e-12))  # shifted systems invertible
    assert C.inside_contour(np.array([0.0]), J, t, eps, rho2)[0]       # gamma encloses 0
    # weights are dz/(2 pi i) of the trapezoid rule: integrals of 1 and z vanish
    assert abs(sigma.sum()) < 1e-13 * r
    assert abs((sigma * z).sum()) < 1e-12 * r * r
    # (1/2 pi i) \oint dz/(z - c) = 1 about the centre c = -t r cos(phi) - i rho2/2: the J-point
    # trapezoid rule is exact for t = 1 and converges geometrically in J for an ellipse
    c = -t * r * math.cos(math.pi / J) - 0.5j * rho2
    if t == 1.0:
        for k in range(-J + 1, J - 1):
            target = 1.0 if k == -1 else 0.0
            assert abs((sigma * (z - c) ** k).sum() - target) < 1e-12 * max(r, 1 / r) ** abs(k + 1)
    Jb = 400
    zb, sb, rb = C.poles_and_weights(Jb, t, eps, rho2)
    cb = -t * rb * math.cos(math.pi / Jb) - 0.5j * rho2
    assert abs((sb / (zb - cb)).sum() - 1.0) < 1e-8


def test_fig3_pole_illustration_parameters():
    # Fig. 3 of Sec. 6.2: t = 0.5, r = 0.6, J = 6.  With r given, eps = r sin(phi) - rho2/2.
    z, sigma = C.ellipse_poles_and_weights(6, 0.5, 0.6)
    assert np.allclose(np.abs(z.real / 0.5) ** 2 + np.abs(z.imag) ** 2, 0.36)


def small_operator(seed=0, shape=(4, 4, 5)):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 2.0, size=shape)
    return O.Operator(c, omega=8.0, damp_cells=1, damp_rho2=0.9, h=0.25)


def test_rational_identity_vs_dense_eig():
    # sum_j sigma_j/z_j (A - z_j)^{-1} = V diag(h_J(lambda)) V^{-1} exactly (Sec. 2 quadrature)
    op = small_operator()
    A = op.assemble().toarray()
    lam, V = np.linalg.eig(A)
    z, sigma, _ = C.poles_and_weights(8, 1.0, 0.5, op.rho2)
    n = A.shape[0]
    Q = np.zeros_like(A)
    for zj, sj in zip(z, sigma):
        Q += (sj / zj) * np.linalg.solve(A - zj * np.eye(n), np.eye(n))
    R = V @ np.diag(C.filter_value(lam, z, sigma)) @ np.linalg.inv(V)
    assert np.linalg.norm(Q - R) <= 1e-9 * np.linalg.norm(Q) * np.linalg.cond(V)


def test_filter_converges_to_projector():
    # fixed circle, growing J: h_J(lambda) lambda -> 1 outside gamma and -> 0 inside (eq. rational)
    op = small_operator(1)
    A = op.assemble().toarray()
    lam, V = np.linalg.eig(A)
    assert lam.real.min() < 0 < lam.real.max()          # indefinite
    # a circle (origin inside) with the widest gap to the spectrum and to the origin
    best = None
    for cr in np.linspace(-1.0, 3.0, 81):
        centre = cr - 0.45j
        d = np.abs(lam - centre)
        for radius in np.linspace(0.5, 4.0, 141):
            if abs(centre) >= radius or (d < radius).sum() < 3 or (d > radius).sum() < 3:
                continue
            gap = min(np.abs(d - radius).min(), radius - abs(centre))
            if best is None or gap > best[0]:
                best = (gap, centre, radius)
    gap, centre, radius = best
    assert gap > 0.03
    d = np.abs(lam - centre)
    ideal = (d > radius).astype(float)
    errs = []
    for J in [16, 64, 256, 1024]:
        z, sigma = C.ellipse_poles_and_weights(J, 1.0, radius, centre)
        errs.append(np.abs(C.filter_value(lam, z, sigma) * lam - ideal).max())
    assert errs[-1] < 1e-7
    assert all(b < a for a, b in zip(errs, errs[1:]))
    # P_J = sum sigma_j/z_j A (A - z_j)^{-1} tends to the spectral projector for the outside eigenvalues
    z, sigma = C.ellipse_poles_and_weights(1024, 1.0, radius, centre)
    n = A.shape[0]
    PJ = sum((sj / zj) * A @ np.linalg.inv(A - zj * np.eye(n)) for zj, sj in zip(z, sigma))
    P = V @ np.diag(ideal.astype(complex)) @ np.linalg.inv(V)
    assert np.linalg.norm(PJ - P) < 1e-8 * np.linalg.cond(V)
    assert np.linalg.norm(PJ @ PJ - PJ) < 1e-8 * np.linalg.cond(V) ** 2
