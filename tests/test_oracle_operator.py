"""Pins of the oracle's operator (eq. stiff-mass, Lemma 3.1) against independent facts."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import operator as O
import workloads as W


def random_setup(shape, seed, cells=2, rho2=0.8):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 3.0, size=shape)
    op = O.Operator(c, omega=7.3, damp_cells=cells, damp_rho2=rho2, h=1.0 / shape[0])
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return op, x


@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 8, 8), (3, 9, 4)])
def test_stencil_matches_assembled_csr(shape):
    op, x = random_setup(shape, 1)
    shift = 0.3 - 1.7j
    y1 = op.apply(x, shift).ravel()
    y2 = op.assemble(shift) @ x.ravel()
    assert np.linalg.norm(y1 - y2) <= 1e-14 * np.linalg.norm(y2)


def test_operator_is_complex_symmetric_not_hermitian():
    op, _ = random_setup((5, 5, 5), 2)
    A = op.assemble().toarray()
    assert np.abs(A - A.T).max() == 0.0
    assert np.abs(A - A.conj().T).max() > 0.1  # damping makes it non-Hermitian


def test_dirichlet_eigenpairs_closed_form():
    # constant kappa, no damping: sin modes are eigenvectors with
    # lambda = (s/h^2) sum_d 2(1 - cos(k_d pi/(N_d+1))) - kappa
    shape = (6, 7, 5)
    c = np.full(shape, 2.0)
    op = O.Operator(c, omega=5.0, damp_cells=0, damp_rho2=0.0, h=0.2)
    for k in [(1, 1, 1), (2, 5, 3), (6, 7, 5)]:
        mode = np.ones(shape)
        lam = -1.0  # kappa = c_min^2/c^2 = 1
        for axis, (kk, n) in enumerate(zip(k, shape)):
            i = np.arange(1, n + 1)
            v = np.sin(kk * i * math.pi / (n + 1))
            sh = [1, 1, 1]
            sh[axis] = n
            mode = mode * v.reshape(sh)
            lam += op.s_h2 * 2.0 * (1.0 - math.cos(kk * math.pi / (n + 1)))
        y = op.apply(mode)
        assert np.linalg.norm(y - lam * mode) <= 1e-13 * np.linalg.norm(lam * mode)


def test_plane_wave_dispersion_relation():
    # Constant c, D = 0: u = exp(i kvec.x) leaves zero interior residual iff
    # (2/h^2) sum_d (1 - cos(k_d h)) = omega^2/c^2, the discrete dispersion relation.
    n, c0, ppw = 24, 1.7, 10.0
    wl_c = np.full((n, n, n), c0)
    omega = W.omega_for_ppw(c0, n, ppw)
    h = 1.0 / n
    op = O.Operator(wl_c, omega, damp_cells=0, damp_rho2=0.0)
    dirn = np.array([0.3, -0.5, 0.81])
    dirn /= np.linalg.norm(dirn)
    disc = lambda k: (2 / h**2) * np.sum(1 - np.cos(k * dirn * h)) - (omega / c0) ** 2
    kd = brentq(disc, 0.5 * omega / c0, 2.0 * omega / c0)
    zz, yy, xx = np.meshgrid(*(np.arange(1, n + 1) * h,) * 3, indexing="ij")
    # dirn is given as (x, y, z) components
    for k, expect_zero in [(kd, True), (omega / c0, False)]:
        u = np.exp(1j * k * (dirn[0] * xx + dirn[1] * yy + dirn[2] * zz))
        r = op.apply(u) / op.s  # physical residual (-Laplace_h - omega^2/c^2) u
        interior = r[1:-1, 1:-1, 1:-1]
        rel = np.abs(interior).max() / (omega / c0) ** 2
        if expect_zero:
            assert rel < 1e-11
        else:
            assert rel > 1e-3  # the continuous wavenumber is not a discrete solution


def test_lemma31_rectangle_contains_dense_spectrum():
    op, _ = random_setup((6, 6, 6), 3, cells=2, rho2=1.3)
    b1, b2, rho2 = op.rectangle()
    lam = np.linalg.eigvals(op.assemble().toarray())
    tol = 1e-10
    assert lam.real.min() >= b1 - tol and lam.real.max() <= b2 + tol
    assert lam.imag.min() >= -rho2 - tol and lam.imag.max() <= tol
    # normalisation of Sec. 7.1: A1 + I >= 0, i.e. Re(lambda) >= -1
    assert lam.real.min() >= -1.0 - tol
    # the enclosing rectangle is not loose by more than the extreme Laplacian modes
    assert b2 - lam.real.max() < 0.5 * (b2 - b1)


def test_damping_profile_layer():
    D = O.damping_profile((20, 20, 20), 6, 1.0)
    assert D.max() == pytest.approx(1.0)
    assert np.all(D[6:-6, 6:-6, 6:-6] == 0.0)
    assert D[0, 10, 10] == pytest.approx(1.0)
    assert D[5, 10, 10] == pytest.approx((1 / 6) ** 2)
    assert D[10, 10, 13] == 0.0 and D[10, 10, 14] == pytest.approx((1 / 6) ** 2)


def test_pointwise_evaluator_matches_full_apply():
    op, x = random_setup((7, 5, 6), 9, cells=2, rho2=0.7)
    pts = [(0, 0, 0), (6, 4, 5), (3, 2, 1), (0, 4, 3), (6, 0, 2)]
    got = O.apply_at(x, op.kappa, 2, 0.7, op.s_h2, 0.2 + 0.4j, pts)
    full = op.apply(x, 0.2 + 0.4j)
    ref = np.array([full[p] for p in pts])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
