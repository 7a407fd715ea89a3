"""Pins of the oracle's FGMRES (Sec. 2 wrapper) and FCI (Algorithm 1)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import contour as C
from oracle import fci as F
from oracle import krylov as K
from oracle import operator as O
import workloads as W


def small_op(seed=0, shape=(6, 6, 6), omega=10.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 2.0, size=shape)
    return O.Operator(c, omega=omega, damp_cells=2, damp_rho2=1.0, h=1.0 / shape[0])


def test_fgmres_identity_is_minimum_residual_over_krylov_space():
    op = small_op()
    A = op.assemble()
    rng = np.random.default_rng(1)
    b = rng.standard_normal(op.n) + 1j * rng.standard_normal(op.n)
    k = 7
    x = K.gmres(lambda v: A @ v, b, k)
    # independent: orthonormal basis of K_k(A, b) by QR of the power basis, then least squares
    Kb = np.empty((op.n, k), dtype=complex)
    v = b.copy()
    for i in range(k):
        Kb[:, i] = v
        v = A @ v
    Q, _ = np.linalg.qr(Kb)
    coef, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    xref = Q @ coef
    assert np.linalg.norm(x - xref) <= 1e-8 * np.linalg.norm(xref)
    assert np.linalg.norm(b - A @ x) <= np.linalg.norm(b - A @ xref) * (1 + 1e-10)


def test_fgmres_exact_preconditioner_one_step():
    op = small_op(2)
    A = op.assemble().tocsc()
    lu = spla.splu(A)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(op.n) + 1j * rng.standard_normal(op.n)
    u, info = K.fgmres(lambda v: A @ v, b, lu.solve, m=5, tol=1e-12)
    assert info["its"] == 1
    assert np.linalg.norm(b - A @ u) <= 1e-12 * np.linalg.norm(b)


def test_fgmres_restarts_reach_direct_solution():
    op = small_op(4, omega=6.0)
    A = op.assemble().tocsc()
    rng = np.random.default_rng(5)
    b = rng.standard_normal(op.n) + 1j * rng.standard_normal(op.n)
    u, info = K.fgmres(lambda v: A @ v, b, lambda v: v, m=10, tol=1e-10, max_it=3000)
    ustar = spla.spsolve(A, b)
    assert info["true_relres"][-1] <= 1e-10
    assert info["restarts"] > 1
    assert np.linalg.norm(u - ustar) <= 1e-6 * np.linalg.norm(ustar)


def test_givens_rotation_annihilates():
    for a, b in [(1 + 2j, 3.0), (0.0, 2.0), (-0.5j, 1e-3)]:
        c, s, rho = K.givens(a, b)
        assert abs(c * a + s * b - rho) < 1e-14
        assert abs(-np.conj(s) * a + c * b) < 1e-14
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-14


def test_fci_with_exact_solves_approximates_projected_inverse():
    # Algorithm 1 steps 1-2 with exact shifted solves: w = sum sigma/z (A - z)^{-1} f, which for a
    # fine quadrature on a fixed circle is P A^{-1} f (eq. rational)
    op = small_op(6, (4, 5, 4), omega=7.0)
    A = op.assemble().toarray()
    lam, V = np.linalg.eig(A)
    centre, radius = 0.0 - 0.5j, None
    d = np.abs(lam - centre)
    radii = np.linspace(0.6, 3.0, 241)
    radius = radii[np.argmax([np.abs(d - r).min() for r in radii])]
    z, sigma = C.ellipse_poles_and_weights(512, 1.0, radius, centre)
    poles = [F.PoleParams(complex(zz), complex(ss), 0j, 0.0, 1) for zz, ss in zip(z, sigma)]
    rng = np.random.default_rng(7)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    solver = lambda rhs, zz: np.linalg.solve(A - zz * np.eye(op.n), rhs.ravel()).reshape(op.shape)
    out, parts = F.fci(op, f, poles, shifted_solver=solver, return_parts=True)
    PAinv = V @ np.diag((d > radius) / lam) @ np.linalg.inv(V)
    ref = PAinv @ f.ravel()
    assert np.linalg.norm(parts["w"].ravel() - ref) <= 1e-6 * np.linalg.norm(ref) * np.linalg.cond(V)
    # step 3: d minimises ||f - d A w||
    Aw = A @ parts["w"].ravel()
    res = lambda dd: np.linalg.norm(f.ravel() - dd * Aw)
    dd = parts["d"]
    for pert in [1e-3, -1e-3, 1e-3j, -1e-3j]:
        assert res(dd) < res(dd + pert * (1 + abs(dd)))


def test_fci_step4_gmres_reduces_remainder():
    op = small_op(8)
    poles = F.pole_parameters(op, 8, 1.0, 0.5, 4)
    f = np.ones(op.shape, dtype=complex)
    out0 = F.fci(op, f, poles, steps=3)
    out5 = F.fci(op, f, poles, steps=3, k_in=5)
    r0 = np.linalg.norm(f - op.apply(out0))
    r5 = np.linalg.norm(f - op.apply(out5))
    assert r5 < r0


def test_end_to_end_small_solve_matches_direct():
    wl = W.config_constant_32(n=10, ppw=10.0)
    op = O.Operator(wl.c, wl.omega, 3, 1.0)
    poles = F.pole_parameters(op, 8, 1.0, 0.5, 8)
    u, info = F.solve(op, wl.rhs[0], poles, m=30, tol=1e-10, max_it=200)
    A = op.assemble().tocsc()
    b = op.s * wl.rhs[0].ravel()
    ustar = spla.spsolve(A, b)
    assert info["true_relres"][-1] <= 1e-10
    # forward error bounded by the condition number times the residual
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(u - ustar) <= 2 * cond * 1e-10 * np.linalg.norm(ustar)
    # physical residual matches as well (scale invariance)
    r_phys = wl.rhs[0].ravel() - (A @ u) / op.s
    assert np.linalg.norm(r_phys) <= 1.01e-10 * np.linalg.norm(wl.rhs[0])
