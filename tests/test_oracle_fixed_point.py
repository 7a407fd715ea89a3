"""Pins of the oracle's polynomial fixed-point iteration (eq. fix-pt-exp, Thm 4.2)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fixed_point as FP
from oracle import operator as O
from oracle import polynomial as P


def tiny(seed=0, shape=(4, 4, 4), omega=8.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 2.0, size=shape)
    return O.Operator(c, omega=omega, damp_cells=1, damp_rho2=1.0, h=1.0 / shape[0])


def dense_poly(A, z0, delta, q):
    """p~(A) as a dense matrix polynomial: sum_j (-i delta (A - z0))^j / j!."""
    n = A.shape[0]
    X = -1j * delta * (A - z0 * np.eye(n))
    term = np.eye(n, dtype=complex)
    total = np.eye(n, dtype=complex)
    for j in range(1, q + 1):
        term = term @ X / j
        total = total + term
    return total


@pytest.mark.parametrize("q,z", [(1, 0.5j), (3, 0.5j), (8, 0.25j), (8, -1.4j), (5, 2.0j)])
def test_thm42_error_propagation(q, z):
    op = tiny()
    A = op.assemble().toarray()
    b1, b2, rho2 = op.rectangle()
    delta, nu, z0 = P.optimise_delta(z, b1, b2, rho2, q, per_side=800)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    y0 = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    ystar = np.linalg.solve(A - z * np.eye(A.shape[0]), f.ravel())
    G = dense_poly(A, z0, delta, q) / P.ptilde(z, z0, delta, q)
    Am = lambda x, s: op.apply(x, s)
    y = y0.copy()
    e = y0.ravel() - ystar
    for m in range(1, 6):
        y = FP.fixed_point_step(Am, y, f, z, z0, delta, q)
        e = G @ e
        assert np.linalg.norm(y.ravel() - ystar - e) <= 1e-12 * (np.linalg.norm(ystar) + np.linalg.norm(e))


def test_solution_is_a_fixed_point():
    op = tiny(1, (5, 4, 6))
    z = 0.3j
    b1, b2, rho2 = op.rectangle()
    delta, _, z0 = P.optimise_delta(z, b1, b2, rho2, 8, per_side=800)
    rng = np.random.default_rng(2)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    ystar = spla.spsolve(op.assemble(z).tocsc(), f.ravel()).reshape(op.shape)
    y1 = FP.fixed_point_step(lambda x, s: op.apply(x, s), ystar, f, z, z0, delta, 8)
    assert np.linalg.norm(y1 - ystar) <= 1e-13 * np.linalg.norm(ystar)


def test_contraction_for_decreasing_imag_shift():
    # Sec. 4.2: the asymptotic contraction factor is rho(p~(A)/p~(z)) = max_i |p~(lambda_i)/p~(z)|,
    # bounded by nu of eq. fix-pt-conv; it approaches 1 as Im z -> 0 and the cost grows.
    op = tiny(3, (5, 5, 5), omega=9.0)
    A = op.assemble().toarray()
    lam = np.linalg.eigvals(A)
    b1, b2, rho2 = op.rectangle()
    rng = np.random.default_rng(4)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    q = 4
    prev_rate, prev_steps = 0.0, 0
    for imz in [1.0, 0.5, 0.25, 0.125]:
        z = 1j * imz
        delta, nu, z0 = P.optimise_delta(z, b1, b2, rho2, q, per_side=800)
        spec = np.abs(P.ptilde(lam, z0, delta, q)).max() / abs(P.ptilde(z, z0, delta, q))
        assert spec <= nu + 1e-9
        y, hist = FP.fixed_point_solve(lambda x, s: op.apply(x, s), f, z, z0, delta, q,
                                       reduce=1e6, m_max=5000)
        assert hist[-1] <= np.linalg.norm(f) / 1e6
        measured = (hist[-1] / hist[-11]) ** 0.1
        assert measured <= spec * 1.05 + 1e-3
        assert measured >= spec * 0.5
        assert spec > prev_rate
        steps = len(hist) - 1
        assert steps >= prev_steps
        prev_rate, prev_steps = spec, steps
        ystar = spla.spsolve(op.assemble(z).tocsc(), f.ravel())
        assert np.linalg.norm(y.ravel() - ystar) <= 1e-4 * np.linalg.norm(ystar)


def test_stopping_rule_reduce_by_five():
    op = tiny(6)
    z = 0.5j
    b1, b2, rho2 = op.rectangle()
    delta, _, z0 = P.optimise_delta(z, b1, b2, rho2, 3, per_side=800)
    f = np.ones(op.shape, dtype=complex)
    y, hist = FP.fixed_point_solve(lambda x, s: op.apply(x, s), f, z, z0, delta, 3, reduce=5.0)
    assert hist[0] == pytest.approx(np.linalg.norm(f))
    assert hist[-1] <= hist[0] / 5 and all(h > hist[0] / 5 for h in hist[:-1])
    y2, hist2 = FP.fixed_point_solve(lambda x, s: op.apply(x, s), f, z, z0, delta, 3, steps=2)
    assert len(hist2) == 3
