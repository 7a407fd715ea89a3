"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module only *draws inputs*: wavespeed grids c(x), angular frequencies
omega, and right-hand sides f.  It contains none of the solver's arithmetic
(no operator, no contour, no polynomial iteration), so that the oracle and the
GPU path can both be fed the very same arrays without sharing method code.

The paper's own media (the eight-anomaly model of the scaling test in Sec. 7
and the SEG/EAGE salt dome of Sec. 8) are not available; the generators below
stand in for them with media of the same character: smooth random fields and
layered models with wavespeeds in the 1.5-4.5 km/s range the salt model spans.

Grid convention (used by every consumer): an N^3 grid of interior nodes on the
unit cube with spacing h = 1/N, arrays indexed [z, y, x] so that x is the
fastest-varying (C-order) index.  "Points per wavelength" (ppw) is measured at
the slowest wavespeed, so omega = 2*pi*c_min*N/ppw.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "omega_for_ppw",
    "gaussian_random_field",
    "constant_medium",
    "grf_medium",
    "layered_medium",
    "point_source",
    "gaussian_rhs",
    "config_constant_32",
    "config_grf_96",
    "config_layered_256",
    "config_uneven_batch",
]


def omega_for_ppw(c_min: float, n: int, ppw: float) -> float:
    """Angular frequency giving `ppw` grid points per wavelength at c_min (h = 1/n)."""
    return 2.0 * math.pi * c_min * n / ppw


def gaussian_random_field(shape, corr_len: float, seed: int) -> np.ndarray:
    """Unit-variance stationary Gaussian random field on the unit cube.

    White noise filtered by a Gaussian kernel exp(-|x|^2 / (2 l^2)) through the
    FFT (periodic), then rescaled to zero mean and unit sample variance.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    noise = rng.standard_normal(shape)
    kz = np.fft.fftfreq(nz, d=1.0 / nz) * 2.0 * math.pi
    ky = np.fft.fftfreq(ny, d=1.0 / ny) * 2.0 * math.pi
    kx = np.fft.rfftfreq(nx, d=1.0 / nx) * 2.0 * math.pi
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    filt = np.exp(-0.5 * k2 * corr_len**2)
    g = np.fft.irfftn(np.fft.rfftn(noise) * filt, s=shape, axes=(0, 1, 2))
    g -= g.mean()
    std = g.std()
    return g / std if std > 0 else g


def constant_medium(n: int, c: float = 1.0) -> np.ndarray:
    return np.full((n, n, n), float(c))


def grf_medium(n: int, seed: int, mean: float = 2.5, amp: float = 1.0,
               corr_len: float = 0.1, lo: float = 1.0, hi: float = 4.5) -> np.ndarray:
    """c = clip(mean + amp * g, lo, hi) with g a unit-variance Gaussian random field."""
    g = gaussian_random_field((n, n, n), corr_len, seed)
    return np.clip(mean + amp * g, lo, hi)


def layered_medium(n: int, seed: int, layers: int = 8, vmin: float = 1.5,
                   vmax: float = 4.5, pert: float = 0.1, corr_len: float = 0.1,
                   lo: float = 1.0, hi: float = 5.0) -> np.ndarray:
    """Equal-thickness z-layers with velocities ~ U[vmin, vmax], times (1 + pert*g)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(vmin, vmax, size=layers)
    idx = np.minimum((np.arange(n) * layers) // n, layers - 1)
    base = v[idx][:, None, None] * np.ones((1, n, n))
    g = gaussian_random_field((n, n, n), corr_len, seed + 7919)
    return np.clip(base * (1.0 + pert * g), lo, hi)


def point_source(n: int, at=None) -> np.ndarray:
    """Unit point source (complex128) at node `at` = (z, y, x); default the centre n//2."""
    f = np.zeros((n, n, n), dtype=np.complex128)
    if at is None:
        at = (n // 2, n // 2, n // 2)
    f[tuple(at)] = 1.0
    return f


def gaussian_rhs(n: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) + i N(0,1) entries."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))


@dataclass
class Workload:
    """One problem instance: medium, frequency, damping layer and right-hand sides."""
    name: str
    c: np.ndarray                 # wavespeed, shape (n, n, n), float64
    omega: float                  # angular frequency
    damp_cells: int               # thickness of the absorbing layer (cells)
    damp_rho2: float              # peak normalised damping, = spectral radius of D
    rhs: list = field(default_factory=list)   # list of complex128 (n, n, n) arrays
    n_poles: int = 8
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.c.shape[0]

    @property
    def h(self) -> float:
        return 1.0 / self.n


def config_constant_32(n: int = 32, ppw: float = 10.0) -> Workload:
    """Constant c = 1 on n^3, omega for `ppw`, 6-cell layer, unit point source at the centre."""
    c = constant_medium(n, 1.0)
    return Workload("constant_c1_%d" % n, c, omega_for_ppw(1.0, n, ppw), 6, 1.0,
                    [point_source(n)], n_poles=8, meta={"ppw": ppw})


def config_grf_96(n: int = 96, seed: int = 0, nrhs: int = 4, ppw: float = 10.0) -> Workload:
    """c = clip(2.5 + g, 1, 4.5), g a GRF with correlation length 0.1; Gaussian complex RHS."""
    c = grf_medium(n, seed)
    rhs = [gaussian_rhs(n, 1000 + seed * 100 + r) for r in range(nrhs)]
    return Workload("grf_%d" % n, c, omega_for_ppw(float(c.min()), n, ppw), 8, 1.0,
                    rhs, n_poles=12, meta={"ppw": ppw, "seed": seed})


def source_nodes(n: int, count: int, seed: int, margin: int) -> list:
    """`count` distinct interior nodes (z, y, x) at least `margin` cells from every face."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        p = tuple(int(v) for v in rng.integers(margin, n - margin, size=3))
        if p not in out:
            out.append(p)
    return out


def config_layered_256(n: int = 256, seed: int = 0, nrhs: int = 8, ppw: float = 8.0,
                       damp_cells: int = 8) -> Workload:
    """Eight layers, velocities U[1.5, 4.5] times (1 + 0.1 g); point sources outside the layer."""
    c = layered_medium(n, seed)
    nodes = source_nodes(n, nrhs, seed + 17, damp_cells + 1)
    rhs = [point_source(n, p) for p in nodes]
    return Workload("layered_%d" % n, c, omega_for_ppw(float(c.min()), n, ppw), damp_cells,
                    1.0, rhs, n_poles=16, meta={"ppw": ppw, "seed": seed, "sources": nodes})


def config_uneven_batch(count: int = 64, seed: int = 0, sizes=(48, 64, 96, 128),
                        ppw_range=(6.0, 12.0)) -> list:
    """`count` independent instances with sizes drawn from `sizes` and ppw ~ U[ppw_range]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.choice(sizes))
        ppw = float(rng.uniform(*ppw_range))
        c = grf_medium(n, seed * 1000 + k)
        f = gaussian_rhs(n, seed * 1000 + 500 + k)
        out.append(Workload("uneven_%d_%d" % (k, n), c, omega_for_ppw(float(c.min()), n, ppw),
                            6, 1.0, [f], n_poles=8, meta={"ppw": ppw}))
    return out
