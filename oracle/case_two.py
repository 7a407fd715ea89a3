"""Case two: the double-size formulation (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3, eq. mat-2x2: with A = A1 - i A2 (A1, A2 Hermitian, A1 + I >= 0,
A2 >= 0, Lemma 3.1) and
    C = [[0, I], [-(A1 + I), -A2]],
the system (iC - I) [x1; x2] = [0; f] has the solution x2 = u, x1 = i u where
A u = f.  Algorithm 1 may be applied to B = iC - I instead of A.

Written out blockwise,
    B [x1; x2] = [ -x1 + i x2 ;  -i (A1 + I) x1 - (I + i A2) x2 ],
so one product with B costs one 7-point stencil (on x1) plus pointwise terms.

Thm 3.2 (thm:spectrum-2x2): spec(C) lies in |mu| <= rho2/2 + sqrt(rho2^2/4 + rho1)
with Re(mu) in [-rho2, 0]; for rho2 = 0 it is {+-i sqrt(lambda_i(A1 + I))}.  The
remark after it moves this to B: |mu + 1| <= R and Im(mu) in [-rho2, 0], R the
same radius.  The rectangle handed to the contour and to the delta search is the
bounding box of that set, [-1 - R, -1 + R] x [-rho2, 0] (reading: the paper
compares the two cases by these rectangles, of width rho2 + sqrt(rho2^2 + 4 rho1)
versus rho1).

Here A1 = S - M (the Hermitian part of the normalised operator) and A2 = D, so
rho1 = rho(A1 + I) is bounded by b2 + 1 with b2 the right edge of A's rectangle
(Weyl bound, operator.spectrum_rectangle), and rho2 = max D.

Sec. 7.2 (eq. shifted-1x1, eq. shifted-2x2): for Hermitian A and z + 1 = (s+1)^2,
(B - s) [i y; (s+1) y] = [0; (A - z) y]: the two shifted problems are equivalent.

Pins (tests/test_oracle_case_two.py): B from its stencil form equals iC - I
assembled blockwise from the matrix A; the solution of eq. mat-2x2 against a
direct solve of A u = f; Thm 3.2 against dense eigenvalues (bound and the rho2 = 0
closed form); the rectangle holds spec(B); eq. shifted-2x2 against eq. shifted-1x1;
the fixed-point iteration on B converges to the dense shifted solution; FCI in
FGMRES on eq. mat-2x2 reproduces the direct solution.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import fci, krylov, operator


class CaseTwoOperator:
    """B = iC - I of eq. mat-2x2 for a normalised operator A (oracle.operator.Operator).

    Vectors have shape (2,) + op.shape: block 0 is x1, block 1 is x2."""

    def __init__(self, op: operator.Operator):
        self.base = op
        self.shape = (2,) + tuple(op.shape)
        self.n = 2 * op.n
        self.s = op.s

    def apply(self, x, shift: complex = 0.0):
        """(B - shift I) x, blockwise (see the module docstring)."""
        op = self.base
        x = np.asarray(x, dtype=np.complex128).reshape(self.shape)
        x1, x2 = x[0], x[1]
        a1x1 = op.s_h2 * operator.neg_laplacian(x1) - op.kappa * x1   # A1 x1 = (S - M) x1
        out = np.empty_like(x)
        out[0] = -x1 + 1j * x2 - shift * x1
        out[1] = -1j * (a1x1 + x1) - (x2 + 1j * op.damp * x2) - shift * x2
        return out

    def rho1(self) -> float:
        """Upper bound of rho(A1 + I) = b2 + 1 (Lemma 3.1 with the Weyl bound of A1)."""
        _, b2, _ = self.base.rectangle()
        return b2 + 1.0

    def radius(self) -> float:
        """R = rho2/2 + sqrt(rho2^2/4 + rho1) (Thm 3.2)."""
        rho2 = self.base.rho2
        return rho2 / 2.0 + math.sqrt(rho2 * rho2 / 4.0 + self.rho1())

    def rectangle(self):
        """[-1 - R, -1 + R] x [-rho2, 0]: the box around the remark's disc-and-band set."""
        R = self.radius()
        return -1.0 - R, -1.0 + R, self.base.rho2

    def rhs(self, f):
        """[0; f] of eq. mat-2x2."""
        f = np.asarray(f, dtype=np.complex128).reshape(self.base.shape)
        return np.stack([np.zeros_like(f), f])

    def assemble(self, shift: complex = 0.0) -> sp.csr_matrix:
        """B - shift I as a sparse 2n x 2n matrix, from the stencil form of A1 and A2."""
        op = self.base
        n = op.n
        eye = sp.identity(n, dtype=np.complex128, format="csr")
        a1 = operator.assemble(op.shape, op.kappa, np.zeros(op.shape), op.s_h2).astype(np.complex128)
        a2 = sp.diags(op.damp.ravel().astype(np.complex128))
        top = sp.hstack([-(1.0 + shift) * eye, 1j * eye])
        bot = sp.hstack([-1j * (a1 + eye), -(1.0 + shift) * eye - 1j * a2])
        return sp.vstack([top, bot]).tocsr()


def pole_parameters(op2: CaseTwoOperator, J: int, t: float, eps: float, q: int, deltas=None):
    """Poles, weights and per-pole (z0, delta) on B's rectangle (eq. quad-points, eq. fix-pt-conv)."""
    return fci.pole_parameters(op2, J, t, eps, q, deltas=deltas)


def solve(op: operator.Operator, f_phys, poles, m: int = 30, tol: float = 1e-8, max_it: int = 1000,
          steps=None, reduce: float = 5.0, m_max: int = 1000):
    """Solve A u = s f_phys through eq. mat-2x2: FGMRES on B with FCI(B), u = x2.

    Returns (u, info) with info from krylov.fgmres on the double-size system."""
    op2 = CaseTwoOperator(op)
    b = op2.rhs(op.s * np.asarray(f_phys, dtype=np.complex128)).ravel()
    pre = lambda v: fci.fci(op2, v, poles, steps=steps, reduce=reduce, m_max=m_max).ravel()
    x, info = krylov.fgmres(lambda v: op2.apply(v).ravel(), b, pre, m=m, tol=tol, max_it=max_it)
    return x.reshape(op2.shape)[1], info
