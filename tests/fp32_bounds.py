"""Error measures and FP32 tolerances of the GPU parity tests, derived from rounding bounds.

Every comparison is element by element: relmax(a, ref) = max_i |a_i - ref_i| / max_i |ref_i|.
A norm-wise measure would let a few wrong points hide among many right ones.

FP32 bars
---------
u = 2^-24 is the unit roundoff of binary32.

* One stencil product y = (A - shift) x.  Each output point is a sum of nine complex
  terms: the diagonal term, the six neighbours and, inside the kernel, the shift folded
  into the diagonal.  It is formed with at most about a dozen roundings.  The standard
  bound for such a sum gives, point by point,
      |y_i - fl(y_i)| <= 12 u (|d_i| |x_i| + (s/h^2) sum_j |x_j|),   d_i = 6 s/h^2 - kappa_i - i D_i - shift,
  where x is the FP32 input.  apply_bound() returns that array, and the tests check it
  point by point.

* A fixed-point step (Sec. 4.2, eq. fix-pt-exp).  The kernels evaluate it in product
  form: y <- L y + y1.  Here L = s^q prod_k (B - rho_k) and y1 = c P2(B) f, with
  B = -i delta (A - z0), c = i delta / p~(z), and the roots rho_k of p~ and mu_k of P2
  taken in Leja order (the scale c is spread over the factors of the y1 chain).
  Factor k is w <- a (A - z0) w + b_k w.  Its rounding error is at most 12 u A_k |w|,
  where A_k = |a| (max |d| + 6 s/h^2) + |b_k| is its absolute row sum.
  That error then passes through the later factors.  In the eigenvalue model (A acting
  on an eigencomponent as the scalar lambda over the spectrum box of Lemma 3.1), the
  first-order error of one chain is
      12 u * max_lambda sum_k |prod_{j>k} f_j(lambda)| A_k |prod_{j<k} f_j(lambda)|.
  The tests denote this G_L for the chain of L and G_P for the chain of y1 (per unit of
  |f|).  Both are computed here from the same poles, delta and q the kernels get.
  Over m steps the error stays below
      m * 12 u (G_L max|y| + G_P max|f|)
  relative to max|y|, because L is a contraction (nu < 1) and does not grow earlier
  errors.  The FP32 right-hand side enters the oracle already rounded to FP32, so input
  rounding is not part of the comparison.
  The model is exact for a normal operator and first order in u.  Our A is complex
  symmetric with damping in a thin layer, and the comparison uses the max norm.  For both
  reasons the tests allow a factor SAFETY = 2 on top (an FP32 emulation on the CPU stays
  hundreds of times inside the bar: tests/test_fp32_bounds.py).

This module holds the bound's arithmetic only.  The oracle it is compared against lives
in oracle/ and is imported by the tests, not by this module.
"""
from math import factorial

import numpy as np

U32 = 2.0 ** -24
ROUNDINGS = 12
SAFETY = 2.0


def relmax(a, ref):
    """max_i |a_i - ref_i| / max_i |ref_i| (0 when both are zero)."""
    a = np.ravel(np.asarray(a))
    ref = np.ravel(np.asarray(ref))
    m = np.abs(ref).max() if ref.size else 0.0
    e = np.abs(a - ref).max() if ref.size else 0.0
    return e / m if m > 0 else e


def round32(x):
    """The complex64 value the device sees for a complex128 host array."""
    return np.asarray(x).astype(np.complex64).astype(np.complex128)


def neighbour_abs_sum(x):
    """sum over the six grid neighbours of |x_j| (Dirichlet: zero outside)."""
    a = np.abs(x)
    s = np.zeros_like(a)
    for ax in range(a.ndim):
        s[(slice(None),) * ax + (slice(1, None),)] += a[(slice(None),) * ax + (slice(None, -1),)]
        s[(slice(None),) * ax + (slice(None, -1),)] += a[(slice(None),) * ax + (slice(1, None),)]
    return s


def apply_bound(x, kappa, damp, s_h2, shift):
    """Point-by-point bound of |fl32((A - shift) x) - (A - shift) x| for an FP32 input x."""
    d = 6.0 * s_h2 - kappa - 1j * damp - shift
    return ROUNDINGS * U32 * (np.abs(d) * np.abs(x) + s_h2 * neighbour_abs_sum(x))


def _leja(r):
    r = list(r)
    out = [r.pop(int(np.argmax(np.abs(r))))]
    while r:
        lp = [sum(np.log(abs(v - o) + 1e-300) for o in out) for v in r]
        out.append(r.pop(int(np.argmax(lp))))
    return np.array(out)


def _ptilde(lam, z0, delta, q):
    x = -1j * delta * (lam - z0)
    return sum(x ** j / factorial(j) for j in range(q + 1))


def _factors(z, z0, delta, q):
    """(a, [b_k]) of the L chain and of the y1 chain, in Leja order."""
    pz = _ptilde(z, z0, delta, q)
    rho = _leja(np.roots([1.0 / factorial(m) for m in range(q, -1, -1)]))
    sL = (1.0 / (factorial(q) * pz)) ** (1.0 / q)
    aL, bL = sL * (-1j * delta), -sL * rho
    gs = 1j * delta / pz
    if q == 1:
        return (aL, bL), (0.0, np.array([gs]))
    beta = -1j * delta * (z - z0)
    ce = [sum(beta ** (j - 1 - m) / factorial(j) for j in range(m + 1, q + 1)) for m in range(q)]
    mu = _leja(np.roots(ce[::-1]))
    s2 = (gs * ce[q - 1]) ** (1.0 / (q - 1))
    return (aL, bL), (s2 * (-1j * delta), -s2 * mu)


def _chain(a, bs, lam, z0, absrow):
    f = np.array([a * (lam - z0) + b for b in bs])
    tot = np.zeros(lam.shape)
    for k in range(len(bs)):
        left = np.prod(np.abs(f[:k]), axis=0) if k else 1.0
        right = np.prod(np.abs(f[k + 1:]), axis=0) if k + 1 < len(bs) else 1.0
        tot += right * (abs(a) * absrow + abs(bs[k])) * left
    return float(tot.max())


def step_growth(z, z0, delta, q, box, absrow_of_z0):
    """(G_L, G_P) of one product-form step: the eigenvalue-model rounding growth of the L
    chain (per unit of |y|) and of the y1 chain (per unit of |f|).  box = (b1, b2, rho2);
    absrow_of_z0(z0) = max |d| + 6 s/h^2, the largest absolute row sum of A - z0."""
    b1, b2, rho2 = box
    lam = (np.linspace(b1, b2, 300)[None, :] + 1j * np.linspace(-rho2, 0.0, 24)[:, None]).ravel()
    (aL, bL), (aP, bP) = _factors(z, z0, delta, q)
    absrow = absrow_of_z0(z0)
    gl = _chain(aL, bL, lam, z0, absrow)
    gp = _chain(aP, bP, lam, z0, absrow)
    return gl, gp


def stencil_absrow(s_h2, kappa, rho2):
    """absrow_of_z0 for the case-one operator A = S - M - iD (normalised units)."""
    kmin, kmax = float(np.min(kappa)), float(np.max(kappa))

    def f(z0):
        d = max(abs(6.0 * s_h2 - k - 1j * dd - z0) for k in (kmin, kmax) for dd in (0.0, rho2))
        return d + 6.0 * s_h2
    return f


def fixed_point_bar(pole, q, steps, box, absrow_of_z0, f_over_y, roundings=ROUNDINGS):
    """FP32 relmax bar of `steps` product-form steps from y = 0 for one pole; f_over_y is
    max|f| / max|y| with y the oracle's iterate; `roundings` is the relative rounding of
    one product in units of u (12 for the stencil)."""
    gl, gp = step_growth(pole.z, pole.z0, pole.delta, q, box, absrow_of_z0)
    return SAFETY * roundings * U32 * max(steps, 1) * (gl + gp * f_over_y)


def case_two_apply_bound(x, kappa, damp, s_h2, shift):
    """Point-by-point bound for (B - shift) x of case two (eq. mat-2x2), x of shape
    (2, nz, ny, nx): block one -x1 + i x2 - shift x1 is pointwise, block two carries the
    stencil of x1, -i ((S - M) + I) x1 - (1 + i D + shift) x2."""
    x1, x2 = x[0], x[1]
    b1 = ROUNDINGS * U32 * (np.abs(1.0 + shift) * np.abs(x1) + np.abs(x2))
    b2 = ROUNDINGS * U32 * (np.abs(6.0 * s_h2 - kappa + 1.0) * np.abs(x1) + s_h2 * neighbour_abs_sum(x1)
                            + np.abs(1.0 + 1j * damp + shift) * np.abs(x2))
    return np.stack([b1, b2])


def case_two_absrow(s_h2, kappa, rho2):
    """absrow_of_z0 for B - z0 of case two: the larger absolute row sum of its two blocks."""
    kmin, kmax = float(np.min(kappa)), float(np.max(kappa))

    def f(z0):
        top = abs(1.0 + z0) + 1.0
        bot = (max(abs(6.0 * s_h2 - k + 1.0) for k in (kmin, kmax)) + 6.0 * s_h2
               + max(abs(1.0 + 1j * dd + z0) for dd in (0.0, rho2)))
        return max(top, bot)
    return f


# Fourier-spectral operator (Sec. 7.1): S x = F^H Lambda F x through FP32 FFTs.  A radix-2
# transform of N points rounds to at most about 5 u log2 N of ||x||_2 (Higham, Accuracy and
# Stability of Numerical Algorithms, Sec. 24.1), two transforms and the scaling make
# 10 u log2 N, relative to s lambda_max ||x||_2.  That is a 2-norm bound: a max-norm
# comparison uses max|e| <= ||e||_2.


def spectral_roundings(n):
    """Relative rounding of one FP32 spectral product in units of u."""
    return 10.0 * np.log2(max(n, 2)) + ROUNDINGS


def spectral_apply_bound(x, s_lam_max, kappa, damp, shift):
    """Bound of max_i |fl32((A - shift) x)_i - ((A - shift) x)_i| for the spectral A."""
    n = x.size
    fft = 10.0 * np.log2(max(n, 2)) * U32 * s_lam_max * np.linalg.norm(np.ravel(x))
    diag = ROUNDINGS * U32 * (np.abs(kappa + 1j * damp + shift) * np.abs(x)).max()
    return fft + diag


def spectral_absrow(s_lam_max, kappa, rho2):
    """absrow_of_z0 for the spectral operator: ||S|| + max |kappa + i D + z0| bounds
    ||A - z0||_2."""
    kmin, kmax = float(np.min(kappa)), float(np.max(kappa))

    def f(z0):
        return s_lam_max + max(abs(k + 1j * dd + z0) for k in (kmin, kmax) for dd in (0.0, rho2))
    return f
