"""Contour parameters chosen by rule (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 7.3 uses a small fixed number of poles (six) and sets eps per frequency.  The rule
written out here chooses eps from the spectrum box [b1, b2] x [-rho2, 0] and the grid size
alone: among 31 geometric candidates over [0.01, 0.64] it takes the first one minimising
the predicted solve time

    T(eps) = eps * (Q * S + Q * M * LAUNCH / npoints + ITER),  Q = per_pass * ceil(q / per_pass),
    S = sum_j c_j,  M = max_j c_j,  c_j = ceil(STEP_FRAC * ln(reduce) / -ln nu_j),

where nu_j is the rate of eq. fix-pt-conv (Sec. 4.2: the delta search with
z0 = (b1 + b2)/2 + i Im z) for pole j of eq. quad-points at (J, t, eps) and degree q.  By
Thm 4.2 the error of the fixed-point iteration is multiplied by p~(A)/p~(z) each step,
whose size on the box is at most nu_j (maximum principle), so s_j steps reduce the residual
by `reduce` for any normal operator with its spectrum in the box.  The rule charges
c_j, STEP_FRAC = 1/2 of that worst case in the logarithm: the adaptive stops, whose
right-hand sides are not concentrated on the worst eigenvalue, measured 0.45-0.6 of s_j
for eps >= 0.08 and less below (ten media and grids).  Q c_j are their products when
per_pass factors run in one pass (a pass counts per_pass products).  The iteration
count of FGMRES is taken proportional to eps; LAUNCH (grid points of one system's pass
that a launch's latency costs) and ITER (the Arnoldi step's work in products) are measured
constants of the hardware, not of the paper.  J = 0 means 6 (Sec. 7.3).  With q = 0 the
degree at each candidate is Sec. 4.2's choice for the pole nearest the origin, counted in
passes (polynomial.choose_q with per_pass, over 1..16).

The rates use the oracle's own delta search on a boundary of `per_side` samples per side.

Pins (tests/test_contour_rule.py): on a diagonal operator whose eigenvalues fill the box,
the oracle's fixed-point iteration needs at most s_j steps at every pole, and exactly s_j
(up to the boundary sampling) when the right-hand side sits on the worst eigenvalue;
mirror-image poles have the same rate; the per-pole charges never grow with eps; with
the launch and iteration terms removed the rule reduces to the product count alone.
"""
from __future__ import annotations

import math

import numpy as np

from .contour import poles_and_weights
from .polynomial import choose_q, optimise_delta

RULE_J, QMAX, LAUNCH, ITER, STEP_FRAC = 6, 16, 2.0e6, 100.0, 0.5
CANDIDATES = 0.01 * 64.0 ** (np.arange(31) / 30.0)


def pole_steps(b1: float, b2: float, rho2: float, J: int, t: float, eps: float, q: int,
               reduce: float = 5.0, per_side: int = 200):
    """(s_j, nu_j, delta_j, z_j, z0_j) for the poles of eq. quad-points at (J, t, eps)."""
    z, _, _ = poles_and_weights(J, t, eps, rho2)
    out = []
    for zj in z:
        d, nu, z0 = optimise_delta(zj, b1, b2, rho2, q, per_side=per_side)
        s = math.ceil(math.log(reduce) / -math.log(nu)) if nu < 1.0 else math.inf
        out.append((s, nu, d, complex(zj), z0))
    return out


def charged_steps(steps, reduce: float = 5.0, frac: float = STEP_FRAC):
    """c_j = ceil(frac ln(reduce) / -ln nu_j) for the (s_j, nu_j, ...) of pole_steps."""
    return [math.ceil(frac * math.log(reduce) / -math.log(p[1])) if p[1] < 1.0 else math.inf for p in steps]


def predicted_time(steps, eps: float, q: int, npoints: float, launch: float = LAUNCH, it: float = ITER,
                   per_pass: int = 2, reduce: float = 5.0) -> float:
    c = charged_steps(steps, reduce)
    Q = per_pass * math.ceil(q / per_pass)
    return eps * (Q * sum(c) + Q * max(c) * launch / npoints + it)


def rule_parameters(b1: float, b2: float, rho2: float, npoints: float, J: int = 0, t: float = 1.0, q: int = 0,
                    per_pass: int = 2, reduce: float = 5.0, per_side: int = 200, launch: float = LAUNCH,
                    it: float = ITER):
    """Returns (J, eps, q, table) with table[k] = (eps_k, T(eps_k), q_k) over the candidates."""
    J = J if J > 0 else RULE_J
    table = []
    for eps in CANDIDATES:
        eps = float(eps)
        qk = q
        if qk <= 0:
            z, _, _ = poles_and_weights(J, t, eps, rho2)
            z1 = z[int(np.argmin(np.abs(z)))]
            qk = choose_q(z1, b1, b2, rho2, qmax=QMAX, per_pass=per_pass, per_side=per_side)[0]
        st = pole_steps(b1, b2, rho2, J, t, eps, qk, reduce, per_side)
        table.append((eps, predicted_time(st, eps, qk, npoints, launch, it, per_pass, reduce), qk))
    k = min(range(len(table)), key=lambda i: (table[i][1], i))
    return J, table[k][0], table[k][2], table
