"""Polynomial fixed-point iteration for a shifted system (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Solves (A - zI) y = f (eq. shifted-lin-sys) with the scheme of eq. fix-pt-exp,
taken as written in Sec. 4.2:
    k_1 = -i delta ((A - z0 I) y^(m) - f),
    k_j = (-i delta / j) ((A - z0 I) k_{j-1} - (-i delta (z - z0))^{j-1}/(j-1)! f),  j = 2..q,
    y^(m+1) = (y^(m) + k_1 + ... + k_q) / p~^(q)(z).
Each step costs q products with A - z0 I.  Thm 4.2: y solves the system iff
it is a fixed point, and y^(m) - y = (p~(A)/p~(z))^m (y^(0) - y).

Readings: y^(0) = 0; the residual r^(m) = f - (A - zI) y^(m) is computed
explicitly here (an extra product, the oracle is not tuned); a solve stops
when ||r^(m)|| <= ||f|| / reduce (Table 4 uses reduce = 5) or after m_max
steps; `steps` fixes the count exactly (lockstep parity mode).

Pins: Thm 4.2 with dense matrix functions; the exact solution is a fixed
point; contraction rate tracks max_i |p~(lambda_i)/p~(z)| for decreasing Im z.
"""
from __future__ import annotations

import math

import numpy as np

from .polynomial import ptilde


def fixed_point_step(apply_A_minus, y, f, z: complex, z0: complex, delta: float, q: int):
    """One step of eq. fix-pt-exp.  apply_A_minus(x, shift) returns (A - shift I) x."""
    k = -1j * delta * (apply_A_minus(y, z0) - f)
    total = y + k
    beta = -1j * delta * (z - z0)
    for j in range(2, q + 1):
        coef = beta ** (j - 1) / math.factorial(j - 1)
        k = (-1j * delta / j) * (apply_A_minus(k, z0) - coef * f)
        total = total + k
    return total / ptilde(z, z0, delta, q)


def fixed_point_solve(apply_A_minus, f, z: complex, z0: complex, delta: float, q: int,
                      y0=None, steps: int | None = None, reduce: float = 5.0,
                      m_max: int = 1000):
    """Iterate eq. fix-pt-exp; returns (y, residual-norm history incl. the initial one)."""
    f = np.asarray(f, dtype=np.complex128)
    y = np.zeros_like(f) if y0 is None else np.array(y0, dtype=np.complex128)
    fnorm = np.linalg.norm(f)
    hist = [np.linalg.norm(f - apply_A_minus(y, z))]
    m = 0
    while True:
        if steps is not None:
            if m >= steps:
                break
        elif hist[-1] <= fnorm / reduce or m >= m_max:
            break
        y = fixed_point_step(apply_A_minus, y, f, z, z0, delta, q)
        hist.append(np.linalg.norm(f - apply_A_minus(y, z)))
        m += 1
    return y, hist
