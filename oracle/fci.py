"""FCI preconditioner (Algorithm 1) and the full solver (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1 (FCI) for a right-hand side f:
  1. solve (A - z_i I) y_i = f for every quadrature pole z_i
     (here: the polynomial fixed-point iteration of eq. fix-pt-exp);
  2. w = sum_i sigma_i / z_i y_i   (quadrature of P A^{-1} f);
  3. d = argmin_d ||f - d A w||_2 = (Aw)^H f / (Aw)^H (Aw);
  4. v = argmin_v ||A v - (f - d A w)|| by a few GMRES steps (k_in; default 0,
     in which case v = 0), optionally right-preconditioned by an approximate
     inverse M of the Laplacian (Sec. 6.3; see laplacian.py): v = M t with t from
     k_in steps on A M;
  return v + d w.
The solver wraps FCI in FGMRES (Sec. 2).

Pins: with exact shifted solves and a large-J contour, w tends to P A^{-1} f
(dense check); end-to-end solutions match a direct sparse solve.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import contour, fixed_point, krylov, operator, polynomial


@dataclass
class PoleParams:
    z: complex
    sigma: complex
    z0: complex
    delta: float
    q: int


def pole_parameters(op: operator.Operator, J: int, t: float, eps: float, q: int,
                    deltas=None):
    """Poles/weights (eq. quad-points) and per-pole (z0, delta) from eq. fix-pt-conv."""
    b1, b2, rho2 = op.rectangle()
    z, sigma, _ = contour.poles_and_weights(J, t, eps, rho2)
    out = []
    for j in range(J):
        if deltas is None:
            d, _, z0 = polynomial.optimise_delta(z[j], b1, b2, rho2, q, per_side=2000)
        else:
            d, z0 = deltas[j], polynomial.default_z0(z[j], b1, b2)
        out.append(PoleParams(complex(z[j]), complex(sigma[j]), complex(z0), float(d), q))
    return out


def fci(op: operator.Operator, f, poles, steps=None, reduce: float = 5.0, m_max: int = 1000,
        k_in: int = 0, shifted_solver=None, return_parts: bool = False, inner_precond=None):
    """Algorithm 1.  `steps` fixes the fixed-point step count per pole (int or list)."""
    f = np.asarray(f, dtype=np.complex128).reshape(op.shape)
    Am = lambda x, shift: op.apply(x, shift)
    w = np.zeros(op.shape, dtype=np.complex128)
    ys = []
    for j, p in enumerate(poles):
        if shifted_solver is not None:
            y = shifted_solver(f, p.z)
        else:
            st = steps[j] if isinstance(steps, (list, tuple)) else steps
            y, _ = fixed_point.fixed_point_solve(Am, f, p.z, p.z0, p.delta, p.q, steps=st,
                                                 reduce=reduce, m_max=m_max)
        ys.append(y)
        w = w + (p.sigma / p.z) * y
    Aw = op.apply(w)
    den = np.vdot(Aw, Aw)
    d = np.vdot(Aw, f) / den if den != 0 else 0.0
    out = d * w
    if k_in > 0:
        rem = (f - d * Aw).ravel()
        if inner_precond is None:
            v = krylov.gmres(lambda x: op.apply(x).ravel(), rem, k_in)
        else:
            # right preconditioning: FGMRES with a fixed M is GMRES on A M, returning M t
            v, _ = krylov.fgmres(lambda x: op.apply(x).ravel(), rem, lambda x: np.ravel(inner_precond(x)),
                                 m=k_in, tol=0.0, max_it=k_in)
        out = out + v.reshape(op.shape)
    if return_parts:
        return out, {"w": w, "d": d, "ys": ys}
    return out


def solve(op: operator.Operator, f_phys, poles, m: int = 30, tol: float = 1e-8,
          max_it: int = 1000, steps=None, reduce: float = 5.0, m_max: int = 1000,
          k_in: int = 0, inner_precond=None):
    """Solve the physical system (-Laplace_h - omega^2/c^2) u = f_phys by FGMRES + FCI.

    The normalised system is A u = s f_phys (Sec. 7.1); relative residuals are
    the same in both scalings.
    """
    b = op.s * np.asarray(f_phys, dtype=np.complex128).ravel()
    pre = lambda v: fci(op, v, poles, steps=steps, reduce=reduce, m_max=m_max, k_in=k_in,
                        inner_precond=inner_precond).ravel()
    return krylov.fgmres(lambda x: op.apply(x).ravel(), b, pre, m=m, tol=tol, max_it=max_it)
