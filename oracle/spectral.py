"""Fourier-spectral discretisation of the Helmholtz operator (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 7.1: the method needs only products with the discrete Laplacian, so a Fourier
spectral S may replace the 7-point stencil.  S is diagonalised by the 3D FFT,
S = F^H Lambda F, with eigenvalues (eq. eig-Laplacian-spectral)
    lambda_i = (l_min / N)^2 sum_j min(i_j^2, (N - i_j)^2),
i a zero-based multi-index of the N^3 grid, l_min the minimum number of points per
wavelength; rho(S) <= (3/4) l_min^2.

Readings: the grid is periodic with spacing h (domain N h per axis).  In the normalisation
of operator.py (A = s(-Laplace) - kappa - i D, s = c_min^2/omega^2) the eigenvalue of the
Fourier mode m is s * sum_j (2 pi min(m_j, N_j - m_j) / (N_j h))^2, which is the paper's
formula since l_min = 2 pi c_min / (omega h).  kappa and the damping layer D are those of
operator.py.  The spectrum box of Lemma 3.1 is [-max kappa, lambda_max - min kappa] x
[-rho2, 0] (lambda_min = 0, the constant mode).

Pins (tests/test_oracle_spectral.py): plane waves are eigenvectors with the formula's
eigenvalues; S against a dense eigendecomposition of the DFT-diagonal operator built from
the DFT matrix; rho(S) <= (3/4) l_min^2; a band-limited Fourier mode's exact -Laplacian;
the box holds the dense spectrum of A.
"""
from __future__ import annotations

import math

import numpy as np

from . import operator


def eigenvalues(shape, h: float, s: float) -> np.ndarray:
    """s * sum_j (2 pi min(m_j, N_j - m_j) / (N_j h))^2 for every Fourier mode m (FFT order)."""
    out = np.zeros(shape)
    for ax, n in enumerate(shape):
        m = np.arange(n)
        k = 2.0 * math.pi * np.minimum(m, n - m) / (n * h)
        sh = [1, 1, 1]
        sh[ax] = n
        out = out + (k ** 2).reshape(sh)
    return s * out


class SpectralOperator:
    """A = S - kappa - i D with the Fourier-spectral S, for a wavespeed grid c [z, y, x]."""

    def __init__(self, c, omega: float, damp_cells: int, damp_rho2: float, h: float | None = None):
        c = np.asarray(c, dtype=np.float64)
        self.shape = c.shape
        self.h = 1.0 / c.shape[0] if h is None else h
        self.omega = omega
        self.s, _, self.kappa = operator.normalisation(c, omega, self.h)
        self.damp = operator.damping_profile(c.shape, damp_cells, damp_rho2)
        self.rho2 = float(self.damp.max()) if self.damp.size else 0.0
        self.n = int(np.prod(self.shape))
        self.lam = eigenvalues(self.shape, self.h, self.s)

    def apply_S(self, x):
        """S x = F^H Lambda F x (unitary FFT pair)."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.shape)
        return np.fft.ifftn(self.lam * np.fft.fftn(x))

    def apply(self, x, shift: complex = 0.0):
        """(A - shift I) x."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.shape)
        return self.apply_S(x) - (self.kappa + 1j * self.damp) * x - shift * x

    def rectangle(self):
        """[-max kappa, lambda_max - min kappa] x [-rho2, 0] (Lemma 3.1, Weyl bounds)."""
        return -float(np.max(self.kappa)), float(self.lam.max()) - float(np.min(self.kappa)), self.rho2

    def l_min(self) -> float:
        """Minimum points per wavelength, 2 pi c_min / (omega h)."""
        return 2.0 * math.pi * math.sqrt(self.s) / self.h
