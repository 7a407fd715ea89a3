"""Pins of the case-two oracle (eq. mat-2x2, Thm 3.2 and its remark, eq. shifted-2x2)."""
import math

import numpy as np
import scipy.sparse.linalg as spla

from oracle import case_two as CT
from oracle import fixed_point as FP
from oracle import operator as O


def small_op(seed=0, shape=(5, 4, 6), omega=9.0, cells=2, rho2=1.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 2.0, size=shape)
    return O.Operator(c, omega=omega, damp_cells=cells, damp_rho2=rho2, h=1.0 / shape[0])


def blocks_from_matrix(op):
    """A1, A2 of Lemma 3.1 taken from the assembled matrix A = A1 - i A2 (A1, A2 real symmetric)."""
    A = op.assemble().toarray()
    return A.real, -A.imag


def dense_B(op, shift=0.0):
    """iC - I - shift I with C = [[0, I], [-(A1 + I), -A2]] built from the dense matrix A."""
    A1, A2 = blocks_from_matrix(op)
    n = op.n
    I = np.eye(n)
    C = np.block([[np.zeros((n, n)), I], [-(A1 + I), -A2]])
    return 1j * C - (1.0 + shift) * np.eye(2 * n)


def test_apply_matches_blockwise_iC_minus_I():
    op = small_op()
    op2 = CT.CaseTwoOperator(op)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(op2.shape) + 1j * rng.standard_normal(op2.shape)
    for shift in (0.0, 0.3 - 0.7j):
        ref = dense_B(op, shift) @ x.ravel()
        assert np.allclose(op2.apply(x, shift).ravel(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.allclose(op2.assemble(shift) @ x.ravel(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_solution_blocks_are_i_u_and_u():
    # eq. mat-2x2: (iC - I)[iu; u] = [0; f] with A u = f
    op = small_op(2)
    op2 = CT.CaseTwoOperator(op)
    rng = np.random.default_rng(3)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    u = spla.spsolve(op.assemble().tocsc(), f.ravel())
    x = spla.spsolve(op2.assemble().tocsc(), op2.rhs(f).ravel()).reshape(op2.shape)
    assert np.linalg.norm(x[1].ravel() - u) <= 1e-10 * np.linalg.norm(u)
    assert np.linalg.norm(x[0].ravel() - 1j * u) <= 1e-10 * np.linalg.norm(u)


def test_theorem_3_2_bound_on_dense_spectrum():
    op = small_op(4, rho2=1.5)
    A1, A2 = blocks_from_matrix(op)
    n = op.n
    rho1 = np.linalg.eigvalsh(A1 + np.eye(n)).max()
    rho2 = np.linalg.eigvalsh(A2).max()
    assert np.linalg.eigvalsh(A1 + np.eye(n)).min() >= -1e-12 and np.linalg.eigvalsh(A2).min() >= -1e-12
    C = np.block([[np.zeros((n, n)), np.eye(n)], [-(A1 + np.eye(n)), -A2]])
    mu = np.linalg.eigvals(C)
    R = rho2 / 2 + math.sqrt(rho2 ** 2 / 4 + rho1)
    assert np.all(np.abs(mu) <= R * (1 + 1e-10))
    assert np.all(mu.real <= 1e-10) and np.all(mu.real >= -rho2 - 1e-10)


def test_theorem_3_2_undamped_closed_form():
    # rho2 = 0: spec(C) = {+-i sqrt(lambda_i(A1 + I))}
    op = small_op(5, cells=0, rho2=0.0)
    A1, A2 = blocks_from_matrix(op)
    assert np.abs(A2).max() == 0.0
    n = op.n
    lam = np.linalg.eigvalsh(A1 + np.eye(n))
    C = np.block([[np.zeros((n, n)), np.eye(n)], [-(A1 + np.eye(n)), np.zeros((n, n))]])
    mu = np.linalg.eigvals(C)
    assert np.abs(mu.real).max() <= 1e-8
    got = np.sort(mu.imag)
    ref = np.sort(np.concatenate([np.sqrt(lam), -np.sqrt(lam)]))
    assert np.allclose(got, ref, atol=1e-8)
    # with rho2 = 0 the radius of Thm 3.2 is sqrt(rho1), attained by the largest pair
    assert math.isclose(np.abs(mu).max(), math.sqrt(lam.max()), rel_tol=1e-10)


def test_rectangle_holds_spectrum_of_B_and_is_narrower():
    op = small_op(6, shape=(6, 6, 6), omega=14.0)
    op2 = CT.CaseTwoOperator(op)
    b1, b2, rho2 = op2.rectangle()
    ev = np.linalg.eigvals(dense_B(op))
    tol = 1e-9
    assert np.all(ev.real >= b1 - tol) and np.all(ev.real <= b2 + tol)
    assert np.all(ev.imag >= -rho2 - tol) and np.all(ev.imag <= tol)
    # the remark's disc: |mu + 1| <= R
    assert np.all(np.abs(ev + 1.0) <= op2.radius() * (1 + 1e-10))
    # width rho2 + sqrt(rho2^2 + 4 rho1) against A's rho1 (remark after Thm 3.2)
    a1, a2, _ = op.rectangle()
    rho1 = op2.rho1()
    assert math.isclose(b2 - b1, rho2 + math.sqrt(rho2 ** 2 + 4 * rho1), rel_tol=1e-14)
    assert math.isclose(a2 + 1.0, rho1, rel_tol=1e-14)


def test_shifted_2x2_equivalent_to_shifted_1x1():
    # Sec. 7.2: A Hermitian, z + 1 = (s + 1)^2: (B - s)[iy; (s+1)y] = [0; (A - z)y]
    op = small_op(7, cells=0, rho2=0.0)
    op2 = CT.CaseTwoOperator(op)
    rng = np.random.default_rng(8)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    for s in (0.2 + 0.5j, -0.4 + 0.25j):
        z = (s + 1.0) ** 2 - 1.0
        y = spla.spsolve(op.assemble(z).tocsc(), f.ravel())
        x = spla.spsolve(op2.assemble(s).tocsc(), op2.rhs(f).ravel()).reshape(op2.shape)
        assert np.linalg.norm(x[0].ravel() - 1j * y) <= 1e-10 * np.linalg.norm(y)
        assert np.linalg.norm(x[1].ravel() - (s + 1.0) * y) <= 1e-10 * np.linalg.norm(y)


def test_fixed_point_on_B_converges_to_dense_shifted_solution():
    op = small_op(9, shape=(5, 5, 5), omega=8.0)
    op2 = CT.CaseTwoOperator(op)
    poles = CT.pole_parameters(op2, 6, 1.0, 0.5, 8)
    rng = np.random.default_rng(10)
    g = rng.standard_normal(op2.shape) + 1j * rng.standard_normal(op2.shape)
    Bm = lambda v, shift: op2.apply(v, shift)
    for p in poles[:3]:
        assert p.z.real <= 1e-12 and (p.z.imag >= 0.5 - 1e-12 or p.z.imag <= -0.5 - op.rho2 + 1e-12)
        y, hist = FP.fixed_point_solve(Bm, g, p.z, p.z0, p.delta, p.q, reduce=1e10, m_max=400)
        ref = spla.spsolve(op2.assemble(p.z).tocsc(), g.ravel())
        assert np.linalg.norm(y.ravel() - ref) <= 1e-8 * np.linalg.norm(ref)
        assert hist[-1] < hist[0]


def test_fgmres_with_fci_on_case_two_matches_direct_solve():
    op = small_op(11, shape=(6, 5, 7), omega=10.0)
    op2 = CT.CaseTwoOperator(op)
    poles = CT.pole_parameters(op2, 6, 1.0, 0.5, 6)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    u, info = CT.solve(op, f, poles, m=20, tol=1e-10, max_it=300)
    uref = spla.spsolve(op.assemble().tocsc(), (op.s * f).ravel())
    assert np.linalg.norm(u.ravel() - uref) <= 1e-8 * np.linalg.norm(uref)
    assert info["its"] < 300
