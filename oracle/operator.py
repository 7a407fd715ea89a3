"""Discrete Helmholtz operator (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The continuous operator is -Laplace - omega^2/c(x)^2 (Sec. 1.1, eq. helmholtz-op).
Sec. 7.1 writes the test matrix as S - M + iD with S the negative discrete
Laplacian, M the (diagonal) mass matrix carrying the wavespeed and D >= 0 a
diagonal damping that is positive near the boundary (eq. stiff-mass).

Readings adopted (the paper does not fix them):
  * Damping sign.  Lemma 3.1 needs A = A1 - i A2 with A2 >= 0 and Sec. 6.2 puts
    the contour centre at -i rho2/2, so the spectrum lies in the lower half
    plane: the oracle uses A = S - M - iD.
  * Normalisation.  M_ii = l_min^2 / l_i^2 (Sec. 7.1) means A is scaled by
    s = c_min^2/omega^2, so that M = kappa with kappa_i = c_min^2/c_i^2 <= 1:
        A = s * (-Laplace_h) - diag(kappa) - i diag(D).
    The physical system (-Laplace_h - omega^2/c^2) u = f is A u = s f.
  * Grid / boundary.  N^3 interior nodes, h = 1/N, homogeneous Dirichlet
    (ghost values zero); 7-point second-order differences.
  * Damping profile.  D_i = rho2 * (d_i / L)^2, d_i = max over axes of the
    depth max(0, L - distance-to-face) into an L-cell layer; rho(D) = rho2.

Pins (tests/test_oracle_operator.py): stencil == assembled CSR; complex
symmetry; closed-form Dirichlet eigenpairs; discrete plane-wave dispersion;
Lemma 3.1 rectangle versus dense eigenvalues.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def normalisation(c: np.ndarray, omega: float, h: float):
    """Return (s, s/h^2, kappa) with s = c_min^2/omega^2 and kappa = c_min^2/c^2 (Sec. 7.1)."""
    c = np.asarray(c, dtype=np.float64)
    cmin = float(c.min())
    s = cmin**2 / omega**2
    kappa = (cmin / c) ** 2
    return s, s / h**2, kappa


def damping_profile(shape, cells: int, rho2: float) -> np.ndarray:
    """Diagonal of D: rho2 * (depth/L)^2 inside an L-cell layer at every face, 0 elsewhere."""
    nz, ny, nx = shape
    if cells <= 0 or rho2 == 0.0:
        return np.zeros(shape)

    def depth(n):
        i = np.arange(n)
        return np.maximum(0, cells - np.minimum(i, n - 1 - i))

    d = np.maximum(np.maximum(depth(nz)[:, None, None], depth(ny)[None, :, None]),
                   depth(nx)[None, None, :])
    return rho2 * (d / cells) ** 2


def neg_laplacian(x: np.ndarray) -> np.ndarray:
    """6 x_i - sum of the six neighbours (zero ghosts): the 7-point stencil without 1/h^2."""
    y = 6.0 * x
    y[1:, :, :] -= x[:-1, :, :]
    y[:-1, :, :] -= x[1:, :, :]
    y[:, 1:, :] -= x[:, :-1, :]
    y[:, :-1, :] -= x[:, 1:, :]
    y[:, :, 1:] -= x[:, :, :-1]
    y[:, :, :-1] -= x[:, :, 1:]
    return y


def apply_shifted(x: np.ndarray, kappa: np.ndarray, damp: np.ndarray, s_h2: float,
                  shift: complex = 0.0) -> np.ndarray:
    """y = (A - shift I) x with A = (s/h^2)(-Laplace stencil) - kappa - i D."""
    x = np.asarray(x, dtype=np.complex128)
    return s_h2 * neg_laplacian(x) - (kappa + 1j * damp) * x - shift * x


class Operator:
    """Normalised operator A for a wavespeed grid c (indexed [z, y, x]) and frequency omega."""

    def __init__(self, c, omega: float, damp_cells: int, damp_rho2: float, h: float | None = None):
        c = np.asarray(c, dtype=np.float64)
        self.shape = c.shape
        self.h = 1.0 / c.shape[0] if h is None else h
        self.omega = omega
        self.s, self.s_h2, self.kappa = normalisation(c, omega, self.h)
        self.damp = damping_profile(c.shape, damp_cells, damp_rho2)
        self.rho2 = float(self.damp.max()) if self.damp.size else 0.0
        self.n = int(np.prod(self.shape))

    def apply(self, x, shift: complex = 0.0):
        return apply_shifted(np.asarray(x).reshape(self.shape), self.kappa, self.damp,
                             self.s_h2, shift)

    def assemble(self, shift: complex = 0.0) -> sp.csr_matrix:
        return assemble(self.shape, self.kappa, self.damp, self.s_h2, shift)

    def rectangle(self):
        return spectrum_rectangle(self.shape, self.kappa, self.damp, self.s_h2)


def second_difference(n: int) -> sp.csr_matrix:
    """1D Dirichlet second difference tridiag(-1, 2, -1)."""
    return sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def assemble(shape, kappa, damp, s_h2: float, shift: complex = 0.0) -> sp.csr_matrix:
    """Explicit sparse A - shift I, built as a Kronecker sum of 1D second differences.

    Row index = x + nx*(y + ny*z), i.e. C order of an [z, y, x] array.
    """
    nz, ny, nx = shape
    ix, iy, iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    lap = (sp.kron(iz, sp.kron(iy, second_difference(nx)))
           + sp.kron(iz, sp.kron(second_difference(ny), ix))
           + sp.kron(second_difference(nz), sp.kron(iy, ix)))
    diag = -(np.asarray(kappa).ravel() + 1j * np.asarray(damp).ravel()) - shift
    return (s_h2 * lap.astype(np.complex128) + sp.diags(diag)).tocsr()


def dirichlet_laplacian_extremes(shape, s_h2: float):
    """Smallest and largest eigenvalue of S = (s/h^2) * 7-point stencil (Dirichlet).

    1D eigenvalues are 2(1 - cos(k pi/(n+1))), k = 1..n; the 3D ones are sums.
    """
    lo = sum(2.0 * (1.0 - math.cos(math.pi / (n + 1))) for n in shape)
    hi = sum(2.0 * (1.0 + math.cos(math.pi / (n + 1))) for n in shape)
    return s_h2 * lo, s_h2 * hi


def spectrum_rectangle(shape, kappa, damp, s_h2: float):
    """Rectangle [b1, b2] x [-rho2, 0] holding spec(A) (Lemma 3.1).

    A1 = S - M is Hermitian and A2 = D >= 0.  By Weyl's inequality
    spec(A1) lies in [lmin(S) - max kappa, lmax(S) - min kappa]; this is inside
    the lemma's [-1, rho1 - 1] because kappa <= 1 after normalisation.
    """
    smin, smax = dirichlet_laplacian_extremes(shape, s_h2)
    b1 = smin - float(np.max(kappa))
    b2 = smax - float(np.min(kappa))
    rho2 = float(np.max(damp)) if np.size(damp) else 0.0
    return b1, b2, rho2


def apply_at(x: np.ndarray, kappa: np.ndarray, damp_cells: int, damp_rho2: float, s_h2: float,
             shift: complex, points) -> np.ndarray:
    """(A - shift I) x evaluated only at the given (z, y, x) nodes, term by term.

    For sampled checks on grids too large for the full oracle: each value is
    the 7-point formula written out with zero ghosts, and D from its definition.
    """
    nz, ny, nx = x.shape
    out = np.empty(len(points), dtype=np.complex128)

    def val(k, j, i):
        if 0 <= k < nz and 0 <= j < ny and 0 <= i < nx:
            return complex(x[k, j, i])
        return 0.0

    def depth(i, n):
        return max(0, damp_cells - min(i, n - 1 - i))

    for t, (k, j, i) in enumerate(points):
        nb = (val(k - 1, j, i) + val(k + 1, j, i) + val(k, j - 1, i) + val(k, j + 1, i)
              + val(k, j, i - 1) + val(k, j, i + 1))
        d = max(depth(k, nz), depth(j, ny), depth(i, nx)) if damp_cells > 0 else 0
        dmp = damp_rho2 * (d / damp_cells) ** 2 if damp_cells > 0 else 0.0
        xc = val(k, j, i)
        out[t] = s_h2 * (6.0 * xc - nb) - (float(kappa[k, j, i]) + 1j * dmp) * xc - shift * xc
    return out
