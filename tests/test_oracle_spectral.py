"""Pins of the Fourier-spectral operator (Sec. 7.1, eq. eig-Laplacian-spectral)."""
import math

import numpy as np

from oracle import spectral as SP


def small(seed=0, shape=(6, 5, 8), omega=9.0, cells=2, rho2=1.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 2.0, size=shape)
    return SP.SpectralOperator(c, omega, cells, rho2, h=1.0 / shape[0])


def test_plane_waves_are_eigenvectors_with_the_formula():
    op = small()
    nz, ny, nx = op.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for m in [(0, 0, 0), (1, 2, 3), (5, 4, 7), (3, 0, 4)]:
        wave = np.exp(2j * math.pi * (m[0] * z / nz + m[1] * y / ny + m[2] * x / nx))
        # the paper's formula, l_min = 2 pi c_min / (omega h), N_j per axis
        lam = sum((op.l_min() * op.h / (n * op.h)) ** 2 * min(mj, n - mj) ** 2
                  for mj, n in zip(m, op.shape))
        assert np.allclose(op.apply_S(wave), lam * wave, atol=1e-12 * max(1.0, lam))


def test_against_dense_dft_construction():
    # S = F^H Lambda F with F the unitary DFT matrix, built densely from 1D DFT matrices
    op = small(1, (4, 3, 5))
    def dft(n):
        j = np.arange(n)
        return np.exp(-2j * math.pi * np.outer(j, j) / n) / math.sqrt(n)
    F = np.kron(dft(op.shape[0]), np.kron(dft(op.shape[1]), dft(op.shape[2])))
    S = F.conj().T @ np.diag(op.lam.ravel()) @ F
    rng = np.random.default_rng(2)
    v = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    assert np.allclose(op.apply_S(v).ravel(), S @ v.ravel(), atol=1e-10)
    # S is Hermitian and positive semi-definite
    assert np.allclose(S, S.conj().T, atol=1e-10)
    assert np.linalg.eigvalsh(S).min() >= -1e-10


def test_spectral_radius_bound():
    for shape in [(8, 8, 8), (7, 9, 6)]:
        op = small(3, shape)
        assert op.lam.max() <= 0.75 * op.l_min() ** 2 * (1 + 1e-12)
    # even N attains it
    op = small(4, (8, 8, 8))
    assert math.isclose(op.lam.max(), 0.75 * op.l_min() ** 2, rel_tol=1e-12)


def test_band_limited_mode_is_differentiated_exactly():
    # -Laplace of sin(k x) on the periodic box of length L = 16 h is k^2 sin(k x), k = 2 pi 3 / L
    shape = (4, 4, 16)
    op = small(5, shape)
    L = 16 * op.h
    xs = np.arange(16) * op.h
    k = 2 * math.pi * 3 / L
    f = np.broadcast_to(np.sin(k * xs), shape).astype(complex)
    assert np.allclose(op.apply_S(f), op.s * k ** 2 * f, atol=1e-10)


def test_box_holds_the_dense_spectrum():
    op = small(6, (4, 4, 4))
    n = op.n
    cols = []
    for k in range(n):
        e = np.zeros(n, dtype=complex)
        e[k] = 1.0
        cols.append(op.apply(e).ravel())
    A = np.array(cols).T
    ev = np.linalg.eigvals(A)
    b1, b2, rho2 = op.rectangle()
    assert np.all(ev.real >= b1 - 1e-9) and np.all(ev.real <= b2 + 1e-9)
    assert np.all(ev.imag >= -rho2 - 1e-9) and np.all(ev.imag <= 1e-9)


def test_fgmres_with_fci_on_the_spectral_operator_matches_direct_solve():
    from oracle import fci as F
    op = small(7, (6, 6, 6), omega=10.0)
    cols = []
    for k in range(op.n):
        e = np.zeros(op.n, dtype=complex)
        e[k] = 1.0
        cols.append(op.apply(e).ravel())
    A = np.array(cols).T
    poles = F.pole_parameters(op, 6, 1.0, 0.5, 6)
    rng = np.random.default_rng(8)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    u, info = F.solve(op, f, poles, m=20, tol=1e-10, max_it=300)
    uref = np.linalg.solve(A, op.s * f.ravel())
    assert np.linalg.norm(u.ravel() - uref) <= 1e-8 * np.linalg.norm(uref)
