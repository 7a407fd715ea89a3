"""The contour-parameter rule: its oracle pinned to Thm 4.2 on normal operators, and the
library's host implementation against the oracle (CPU only: the rule does no GPU work).

Pole j of a contour needs at most s_j = ceil(ln(reduce) / -ln nu_j) fixed-point steps,
nu_j being eq. fix-pt-conv's rate: by Thm 4.2 the error (and, for a normal operator, the
residual) is multiplied by p~(A)/p~(z) each step, bounded by nu_j on the spectrum box.
The rule charges c_j = ceil(ln(reduce) / 2 / -ln nu_j) of them (the adaptive stops'
measured average is about half the worst case).
"""
import math
import os

import numpy as np
import pytest

from oracle import contour_rule as R
from oracle import fixed_point as FP
from oracle.polynomial import ptilde, rectangle_boundary

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1811_12378_amd", "libhfci.so")
B1, RHO2 = -1.0, 1.0


def fp_steps(lam, f, z, z0, delta, q, reduce=5.0):
    """Steps of the oracle's fixed-point iteration on diag(lam) to reduce the residual by `reduce`."""
    _, hist = FP.fixed_point_solve(lambda x, s: (lam - s) * x, f, z, z0, delta, q, reduce=reduce, m_max=400)
    return len(hist) - 1


@pytest.mark.parametrize("b2,J,eps,q", [(19.4, 6, 0.25, 8), (10.9, 16, 0.1, 3), (43.7, 6, 0.5, 8)])
def test_charged_steps_suffice_and_are_tight(b2, J, eps, q):
    steps = R.pole_steps(B1, b2, RHO2, J, 1.0, eps, q)
    bd = rectangle_boundary(B1, b2, RHO2, 200)
    # eigenvalues: the sampled box boundary and an interior grid (maximum principle: the
    # interior never beats the boundary)
    gx, gy = np.meshgrid(np.linspace(B1, b2, 25)[1:-1], np.linspace(-RHO2, 0.0, 7)[1:-1])
    lam = np.concatenate([bd, (gx + 1j * gy).ravel()])
    rng = np.random.default_rng(5)
    f = rng.standard_normal(lam.size) + 1j * rng.standard_normal(lam.size)
    for s, nu, d, z, z0 in steps:
        assert fp_steps(lam, f, z, z0, d, q) <= s
        # on the worst boundary eigenvalue the residual shrinks by exactly nu per step
        k = int(np.argmax(np.abs(ptilde(bd, z0, d, q))))
        assert abs(abs(ptilde(bd[k], z0, d, q) / ptilde(z, z0, d, q)) - nu) < 1e-12
        e = np.zeros(lam.size, dtype=complex)
        e[k] = 1.0
        assert fp_steps(lam, e, z, z0, d, q) == s


def test_mirror_poles_share_rates():
    # poles j and J-1-j are mirror images about Im = -rho2/2, as is the box
    for J in (6, 16):
        st = R.pole_steps(B1, 19.4, RHO2, J, 1.0, 0.2, 8)
        for j in range(J):
            assert abs(st[j][1] - st[J - 1 - j][1]) < 1e-8
            assert st[j][0] == st[J - 1 - j][0]


def test_charges_never_grow_with_eps():
    for b2 in (10.9, 43.7):
        prev = None
        for eps in R.CANDIDATES[::3]:
            s = [p[0] for p in R.pole_steps(B1, b2, RHO2, 6, 1.0, float(eps), 8)]
            cur = (sum(s), max(s))
            if prev is not None:
                assert cur[0] <= prev[0] and cur[1] <= prev[1], (b2, eps, cur, prev)
            prev = cur


def charged(st, reduce=5.0):
    # half the worst case in the logarithm, written out from the rates
    return [math.ceil(0.5 * math.log(reduce) / -math.log(p[1])) for p in st]


def test_charged_steps_are_half_the_worst_case():
    st = R.pole_steps(B1, 19.4, RHO2, 6, 1.0, 0.1, 8)
    c = R.charged_steps(st)
    assert c == charged(st)
    for cj, p in zip(c, st):
        # ceil(x / 2) <= ceil(x) <= 2 ceil(x / 2): half the worst case, rounded up
        assert cj <= p[0] <= 2 * cj


def test_rule_reduces_to_product_count_without_overheads():
    J, eps, q, table = R.rule_parameters(B1, 19.4, RHO2, 1e30, J=6, q=8, it=0.0)
    k = int(np.argmin([t for _, t, _ in table]))
    c = charged(R.pole_steps(B1, 19.4, RHO2, 6, 1.0, eps, 8))
    assert J == 6 and q == 8 and eps == table[k][0]
    assert abs(table[k][1] - eps * 8 * sum(c)) < 1e-9 * table[k][1]
    # an odd degree costs a whole pass for its lone factor: Q rounds up to even
    J, eps7, q7, table7 = R.rule_parameters(B1, 19.4, RHO2, 1e30, J=6, q=7, it=0.0)
    c7 = charged(R.pole_steps(B1, 19.4, RHO2, 6, 1.0, eps7, 7))
    assert abs(dict((e, t) for e, t, _ in table7)[eps7] - eps7 * 8 * sum(c7)) < 1e-9 * eps7 * 8 * sum(c7)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfci.so not built")
@pytest.mark.parametrize("b2,npoints,q", [(19.4, 256 ** 3, 0), (10.9, 128 ** 3, 8)])
def test_library_rule_matches_oracle(b2, npoints, q):
    from paper_1811_12378_amd import hfci
    J, eps, qc = hfci.contour_rule(B1, b2, RHO2, npoints, q=q)
    Jo, eps_o, q_o, table = R.rule_parameters(B1, b2, RHO2, npoints, q=q)
    assert J == Jo == 6
    assert q == 0 or qc == q_o == q
    # a candidate of the geometric grid (the two sides form its powers in their own order)
    assert min(abs(eps - e) for e, _, _ in table) <= 1e-12 * eps
    # equal, or (the two delta searches differ in resolution, which can move a ceil or the
    # degree) within 2 % of the oracle's minimum predicted time at that eps with that degree
    tmin = min(t for _, t, _ in table)
    if abs(eps - eps_o) > 1e-12 * eps or qc != q_o:
        st = R.pole_steps(B1, b2, RHO2, 6, 1.0, eps, qc)
        assert R.predicted_time(st, eps, qc, npoints) <= 1.02 * tmin, (eps, qc, eps_o, q_o)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfci.so not built")
def test_library_rule_rejects_bad_boxes():
    from paper_1811_12378_amd import hfci
    for args in ((1.0, -1.0, 1.0, 8.0), (-1.0, 5.0, -1.0, 8.0), (-1.0, 5.0, 1.0, 0.0)):
        with pytest.raises(hfci.HfciError):
            hfci.contour_rule(*args)
    with pytest.raises(hfci.HfciError):
        hfci.contour_rule(-1.0, 5.0, 1.0, 8.0, fp_reduce=1.0)
    with pytest.raises(hfci.HfciError):
        hfci.contour_rule(-1.0, 5.0, 1.0, 8.0, per_pass=3)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfci.so not built")
def test_library_rule_is_deterministic():
    # the candidates, the degree search and the pole rates run on host threads and are
    # reduced in order: repeated calls agree exactly
    from paper_1811_12378_amd import hfci
    for b2, npoints, q in ((19.4, 256.0 ** 3, 0), (10.9, 64.0 ** 3, 0), (43.7, 96.0 ** 3, 8)):
        first = hfci.contour_rule(B1, b2, RHO2, npoints, q=q)
        for _ in range(4):
            assert hfci.contour_rule(B1, b2, RHO2, npoints, q=q) == first
