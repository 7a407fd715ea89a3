"""Krylov solvers (oracle): flexible GMRES and plain GMRES.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2: because one FCI application is not an accurate solve, it is used as a
preconditioner inside flexible GMRES (Saad's FGMRES) or iterative refinement.
This module writes FGMRES(m) out in full:
  * right-preconditioned Arnoldi with a preconditioner that may change every
    step: z_j = M_j(v_j), w = A z_j, solution update u += Z_m y_m;
  * orthogonalisation by classical Gram-Schmidt applied twice (CGS2):
    h = V^H w, w -= V h, h' = V^H w, w -= V h', h += h';
  * the small least-squares problem min ||beta e1 - H y|| by Givens rotations;
  * restarts recompute the true residual r = f - A u (this is iterative
    refinement with the FGMRES cycle as the correction solve).
Givens rotation convention: c = |a|/rho, s = (a/|a|) conj(b)/rho with
rho = sqrt(|a|^2 + |b|^2), applied as [x; y] -> [c x + s y; -conj(s) x + c y].

Pins: with M = identity, FGMRES equals the minimum-residual solution over the
Krylov space (checked against a least-squares solve on an explicit basis);
with M = A^{-1} it converges in one step; solutions match a direct solve.
"""
from __future__ import annotations

import numpy as np


def givens(a: complex, b: complex):
    """Rotation (c, s, rho) with [c s; -conj(s) c] [a; b] = [rho; 0]."""
    if a == 0:
        return 0.0, 1.0 + 0j, b
    rho = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    phase = a / abs(a)
    return abs(a) / rho, phase * np.conj(b) / rho, phase * rho


def fgmres(apply_A, f, precond, m: int = 30, tol: float = 1e-8, max_it: int = 1000,
           u0=None, true_residual_on_exit: bool = True):
    """Restarted flexible GMRES.  Returns (u, info).

    info: dict(its, restarts, history (estimated relative residual per step),
    true_relres (at every restart and on exit)).
    """
    f = np.asarray(f, dtype=np.complex128).ravel()
    n = f.size
    A = lambda x: np.asarray(apply_A(x), dtype=np.complex128).ravel()
    M = lambda x: np.asarray(precond(x), dtype=np.complex128).ravel()
    u = np.zeros(n, dtype=np.complex128) if u0 is None else np.array(u0, dtype=np.complex128).ravel()
    fnorm = np.linalg.norm(f)
    # relative residuals; for f = 0 the iteration stops at once with u = 0 (if u0 is None),
    # and its history records the absolute residual instead of 0/0
    rel_den = fnorm if fnorm > 0 else 1.0
    its, restarts = 0, 0
    hist, true_hist = [], []
    while True:
        r = f - A(u)
        beta = np.linalg.norm(r)
        true_hist.append(beta / rel_den)
        if beta <= tol * fnorm or its >= max_it:
            break
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Z = np.zeros((m, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            h = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0:
                V[j + 1] = w / hn
            for i in range(j):
                x, y = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * x + sn[i] * y
                H[i + 1, j] = -np.conj(sn[i]) * x + cs[i] * y
            c, s, rho = givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j], H[j + 1, j] = rho, 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            its += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / rel_den)
            if abs(g[j + 1]) <= tol * fnorm or its >= max_it or hn == 0:
                break
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1: k] @ y[i + 1: k]) / H[i, i]
        u = u + Z[:k].T @ y
        restarts += 1
    return u, {"its": its, "restarts": restarts, "history": hist, "true_relres": true_hist}


def gmres(apply_A, b, steps: int, x0=None):
    """`steps` steps of plain GMRES from x0 (no restart): minimum residual over K_steps."""
    ident = lambda x: x
    x, _ = fgmres(apply_A, b, ident, m=max(steps, 1), tol=0.0, max_it=steps, u0=x0)
    return x
