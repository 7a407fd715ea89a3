"""Regularised inverse of the discrete Laplacian, the inner preconditioner of Alg. 1 step 4 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1 step 4 solves the remainder A v = f - d A w approximately by a few GMRES steps.
Sec. 6.3 preconditions those steps with an approximate inverse of the discrete
Laplacian, which deflates the large eigenvalues of the Helmholtz operator.  In Sec. 7.3
the spectral discretisation uses the FFT-diagonalised inverse with eigenvalues
1/max(lambda_i, 1) (lambda_i of eq. eig-Laplacian-spectral), and finite differences use
ILU(0) of the 7-point Laplacian.

Reading (the paper's ILU(0) is a sequential triangular solve): for the 7-point stencil
with homogeneous Dirichlet ghosts, the normalised Laplacian S = (s/h^2)(7-point stencil)
is diagonalised exactly by the orthonormal sine transform (DST-I) along each axis, with
eigenvalues s/h^2 * sum over axes of 2 (1 - cos(k pi / (n + 1))), k = 1..n.  The
preconditioner is the FD analogue of the spectral one:
    M = V diag(1 / max(lambda, 1)) V^T,   V = DST-I (orthonormal) along z, y and x.

Pins (tests/test_oracle_laplacian.py): M against V diag(..) V^T built from a dense
eigendecomposition of the assembled S; M S x = x on the modes with lambda >= 1 and
M x = x on the others; Alg. 1 step 4 with M = A^{-1} gives A^{-1} f.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft as sfft


def laplacian_eigenvalues(shape, s_h2: float) -> np.ndarray:
    """lambda[k, j, i] of S = (s/h^2) * 7-point stencil for the sine mode (k+1, j+1, i+1)."""
    nz, ny, nx = shape

    def ev(n):
        m = np.arange(1, n + 1)
        return 2.0 * (1.0 - np.cos(m * math.pi / (n + 1)))

    return s_h2 * (ev(nz)[:, None, None] + ev(ny)[None, :, None] + ev(nx)[None, None, :])


def apply_inverse(x, shape, s_h2: float) -> np.ndarray:
    """M x = V diag(1 / max(lambda, 1)) V^T x for x of the grid's shape (complex)."""
    x = np.asarray(x, dtype=np.complex128).reshape(shape)
    lam = laplacian_eigenvalues(shape, s_h2)
    # DST-I with norm="ortho" is orthonormal and its own inverse
    c = sfft.dstn(x, type=1, norm="ortho")
    c = c / np.maximum(lam, 1.0)
    return sfft.dstn(c, type=1, norm="ortho")


def dst_matrix(n: int) -> np.ndarray:
    """Orthonormal DST-I matrix: sqrt(2/(n+1)) sin(pi (j+1)(k+1)/(n+1)), symmetric."""
    j = np.arange(1, n + 1)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * math.pi / (n + 1))
