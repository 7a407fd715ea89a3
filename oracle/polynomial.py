"""Exponential-Taylor residual polynomial and its parameters (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4: a polynomial fixed-point iteration for (A - zI) y = f has residual
polynomial R(lambda) = 1 - (lambda - z) p(lambda - z) (eq. res-poly), and a good
p makes max |R| small on the rectangle B holding the spectrum (eq. minimax).

Sec. 4.2 takes R = p~(lambda)/p~(z) with the truncated exponential
    p~^(q)(lambda) = sum_{j=0..q} (-i delta (lambda - z0))^j / j!   (eq. exp-taylor)
and the heuristic parameters
    z0 = (b1 + b2)/2 + i Im z,
    delta = argmin over real delta of max_{lambda on dB} |p~(lambda)/p~(z)|  (eq. fix-pt-conv),
with nu the attained minimum; q is preferred where nu^(1/q) is smallest.

Readings: the search is one-dimensional in delta (the paper calls it a "2D
optimization problem"); delta carries the sign of Im z, which makes
delta * Im(lambda - z0) < 0 on B (the robustness argument of Sec. 4.2);
dB is sampled densely (vertices included).  Ties go to the smallest |delta|.
The estimated cost to reduce the residual by a factor F is q*ceil(ln F/(-ln nu))
matrix-vector products (the reading that reproduces Tables 2 and 4).

Pins: Table 1 (delta* on the paper's 1/16 grid, nu), Table 2, Table 4 and
Thm 4.1's closed form at q = 1 (tests/test_oracle_polynomial.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import minimize_scalar


def ptilde(lam, z0: complex, delta: float, q: int):
    """p~^(q)(lambda) of eq. exp-taylor, summed term by term."""
    x = -1j * delta * (np.asarray(lam, dtype=np.complex128) - z0)
    term = np.ones_like(x)
    total = np.ones_like(x)
    for j in range(1, q + 1):
        term = term * x / j
        total = total + term
    return total


def rectangle_boundary(b1: float, b2: float, rho2: float, per_side: int = 4000):
    """Points on the boundary of [b1, b2] x [-rho2, 0], vertices included."""
    t = np.linspace(0.0, 1.0, per_side + 1)
    top = b1 + (b2 - b1) * t + 0j
    bottom = top - 1j * rho2
    left = b1 - 1j * rho2 * t
    right = b2 - 1j * rho2 * t
    return np.concatenate([top, bottom, left, right])


def default_z0(z: complex, b1: float, b2: float) -> complex:
    """z0 = (b1 + b2)/2 + i Im z (Sec. 4.2)."""
    return complex(0.5 * (b1 + b2), complex(z).imag)


def rate(delta: float, z: complex, z0: complex, q: int, boundary) -> float:
    """max over the sampled boundary of |p~(lambda)/p~(z)| (the objective of eq. fix-pt-conv)."""
    return float(np.max(np.abs(ptilde(boundary, z0, delta, q))) / abs(ptilde(z, z0, delta, q)))


def optimise_delta(z: complex, b1: float, b2: float, rho2: float, q: int,
                   grid_step: float | None = None, per_side: int = 4000,
                   z0: complex | None = None):
    """Return (delta, nu, z0) minimising eq. fix-pt-conv over real delta with sign(delta) = sign(Im z).

    With `grid_step`, delta is restricted to multiples of it (the paper's
    Table 1 values all lie on a 1/16 grid); otherwise a log-spaced scan is
    refined by a bounded scalar minimisation.
    """
    z = complex(z)
    if z0 is None:
        z0 = default_z0(z, b1, b2)
    sgn = 1.0 if z.imag > 0 else -1.0
    bd = rectangle_boundary(b1, b2, rho2, per_side)
    if grid_step is not None:
        ks = np.arange(1, int(round(8.0 / grid_step)) + 1)
        best = (math.inf, None)
        for k in ks:
            nu = rate(sgn * k * grid_step, z, z0, q, bd)
            if nu < best[0] - 1e-12:
                best = (nu, sgn * k * grid_step)
        return best[1], best[0], z0
    scan = np.geomspace(1e-4, 50.0, 600)
    vals = np.array([rate(sgn * d, z, z0, q, bd) for d in scan])
    k = int(np.argmin(vals))
    lo = scan[max(k - 1, 0)]
    hi = scan[min(k + 1, len(scan) - 1)]
    res = minimize_scalar(lambda d: rate(sgn * d, z, z0, q, bd), bounds=(lo, hi),
                          method="bounded", options={"xatol": 1e-10})
    d, nu = (res.x, res.fun) if res.fun < vals[k] else (scan[k], vals[k])
    return sgn * float(d), float(nu), z0


def choose_q(z: complex, b1: float, b2: float, rho2: float, qmax: int = 8, per_pass: int = 1, **kw):
    """q in 1..qmax minimising nu^(1/q) (Sec. 4.2: products per unit of residual reduction,
    q / (-ln nu)); with per_pass factors applied per pass over memory, the passes
    ceil(q / per_pass) / (-ln nu) instead (per_pass = 1 is the rule as written).  Returns
    (q, delta, nu); ties go to the smaller q."""
    best = None
    for q in range(1, qmax + 1):
        d, nu, _ = optimise_delta(z, b1, b2, rho2, q, **kw)
        if not nu < 1.0:
            continue
        key = math.ceil(q / per_pass) / -math.log(nu)
        if best is None or key < best[0]:
            best = (key, q, d, nu)
    return best[1], best[2], best[3]


def estimated_matvecs(nu: float, q: int, factor: float) -> int:
    """q * ceil(ln(factor) / (-ln nu)): matvecs to reduce the residual by `factor`."""
    return q * int(math.ceil(math.log(factor) / (-math.log(nu))))


def richardson_closed_form(z: complex, b1: float, b2: float, rho2: float):
    """Thm 4.1: optimal constant p* and minimax value for the stationary Richardson iteration.

    alpha = (b1 - z, b2 - z) if Im z > 0, else (beta1 - z, beta2 - z) with
    beta_k = b_k - i rho2; value |a1 - a2| / (|a1| + |a2|),
    p* = (|a1|/a1 + |a2|/a2) / (|a1| + |a2|).
    """
    z = complex(z)
    if z.imag > 0:
        a1, a2 = b1 - z, b2 - z
    else:
        a1, a2 = (b1 - 1j * rho2) - z, (b2 - 1j * rho2) - z
    value = abs(a1 - a2) / (abs(a1) + abs(a2))
    pstar = (abs(a1) / a1 + abs(a2) / a2) / (abs(a1) + abs(a2))
    return pstar, value
