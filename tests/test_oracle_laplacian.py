"""Pins of the inner preconditioner (Sec. 6.3) and of Alg. 1 step 4 with it."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import fci as F
from oracle import laplacian as L
from oracle import operator as O


def small_op(seed=0, shape=(5, 4, 6), omega=9.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 2.0, size=shape)
    return O.Operator(c, omega=omega, damp_cells=2, damp_rho2=1.0, h=1.0 / shape[0])


def dense_laplacian(op):
    """S = (s/h^2) * 7-point stencil, assembled (kappa = 0, no damping)."""
    return O.assemble(op.shape, np.zeros(op.shape), np.zeros(op.shape), op.s_h2).toarray().real


def test_inverse_matches_dense_eigendecomposition():
    for shape, omega in (((5, 4, 6), 9.0), ((3, 7, 2), 6.0)):
        op = small_op(1, shape, omega)
        S = dense_laplacian(op)
        lam, V = np.linalg.eigh(S)
        Md = V @ np.diag(1.0 / np.maximum(lam, 1.0)) @ V.T
        rng = np.random.default_rng(2)
        x = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
        got = L.apply_inverse(x, op.shape, op.s_h2).ravel()
        ref = Md @ x.ravel()
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        # both clamps are exercised: some eigenvalues below 1, some above
        assert lam.min() < 1.0 < lam.max()
        # the closed-form eigenvalues are the dense ones
        assert np.allclose(np.sort(L.laplacian_eigenvalues(op.shape, op.s_h2).ravel()), lam, atol=1e-10)


def test_inverse_on_modes():
    # M S x = x on sine modes with lambda >= 1, M x = x on the others
    op = small_op(3, (6, 5, 7), 20.0)
    lam = L.laplacian_eigenvalues(op.shape, op.s_h2)
    Sz, Sy, Sx = (L.dst_matrix(n) for n in op.shape)
    for (k, j, i) in [(0, 0, 0), (5, 4, 6), (2, 1, 3)]:
        mode = np.einsum("a,b,c->abc", Sz[:, k], Sy[:, j], Sx[:, i]).astype(complex)
        Sm = op.s_h2 * O.neg_laplacian(mode)
        assert np.allclose(Sm, lam[k, j, i] * mode, atol=1e-12)
        out = L.apply_inverse(mode, op.shape, op.s_h2)
        assert np.allclose(out, mode / max(lam[k, j, i], 1.0), atol=1e-13)
    assert lam.min() < 1.0 < lam.max()


def test_dst_matrix_orthonormal_and_symmetric():
    for n in (1, 2, 7, 16):
        S = L.dst_matrix(n)
        assert np.allclose(S, S.T)
        assert np.allclose(S @ S, np.eye(n), atol=1e-13)


def test_step_four_with_exact_inner_preconditioner_solves():
    # with M = A^{-1}, one preconditioned GMRES step solves the remainder exactly: the FCI
    # output becomes A^{-1} f whatever the quadrature did
    op = small_op(4)
    A = op.assemble().tocsc()
    poles = F.pole_parameters(op, 4, 1.0, 0.5, 4)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    Minv = lambda x: spla.spsolve(A, np.ravel(x))
    out = F.fci(op, f, poles, steps=2, k_in=1, inner_precond=Minv)
    ref = spla.spsolve(A, f.ravel())
    assert np.linalg.norm(out.ravel() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_step_four_with_laplacian_inverse_reduces_remainder():
    op = small_op(6, (6, 6, 6), 12.0)
    poles = F.pole_parameters(op, 6, 1.0, 0.5, 6)
    rng = np.random.default_rng(7)
    f = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    M = lambda x: L.apply_inverse(x, op.shape, op.s_h2)
    base, parts = F.fci(op, f, poles, steps=2, return_parts=True)
    r0 = np.linalg.norm(f - op.apply(base))
    prev = r0
    for k in (1, 2, 4):
        out = F.fci(op, f, poles, steps=2, k_in=k, inner_precond=M)
        r = np.linalg.norm(f - op.apply(out))
        assert r <= prev * (1 + 1e-12)  # minimum residual over growing spaces
        prev = r
    assert prev < 0.5 * r0
