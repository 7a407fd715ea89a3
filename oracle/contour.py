"""Contour quadrature: poles z_j and weights sigma_j (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2: for a contour gamma enclosing the origin, P A^{-1} equals the Cauchy
integral (1/2 pi i) \\oint (A - zI)^{-1} dz/z (eq. rational), where P projects
onto the eigenvalues outside gamma; a quadrature with nodes z_j and weights
sigma_j gives P A^{-1} ~ sum_j sigma_j/z_j (A - z_j I)^{-1}.

Sec. 6.1 (eq. ellipse): on t r cos(theta) + i r sin(theta), dz/(2 pi i) equals
(r cos(theta) + i t r sin(theta)) dtheta/(2 pi), so equispaced angles give
sigma_j = (r cos(theta_j) + i t r sin(theta_j)) / J.

Sec. 6.2 (eq. quad-points, eq. quad-radius): the centre is moved to
-t r cos(phi) - i rho2/2 with phi = pi/J and theta_j = (2j-1) phi, so that
    z_j = t r (cos((2j-1)phi) - cos(phi)) + i (r sin((2j-1)phi) - rho2/2),
    r   = (rho2/2 + eps) / sin(phi).
Moving the centre does not change dz, so the weights are those of eq. ellipse
at the same angles (reading: "circular contour" = t = 1).

Pins: the four pole sets printed in Sec. 7.3 (tests/golden/poles_sec7.txt);
Re z_j <= 0 and Im z_j outside (-eps - rho2, eps); the filter converges to the
exact projector filter as J grows; exact rational identity versus dense eig.
"""
from __future__ import annotations

import math

import numpy as np


def poles_and_weights(J: int, t: float, eps: float, rho2: float):
    """Return (z, sigma, r): J complex poles, their quadrature weights, and the radius r."""
    phi = math.pi / J
    r = (rho2 / 2.0 + eps) / math.sin(phi)
    j = np.arange(1, J + 1)
    theta = (2 * j - 1) * phi
    z = t * r * (np.cos(theta) - math.cos(phi)) + 1j * (r * np.sin(theta) - rho2 / 2.0)
    sigma = (r * np.cos(theta) + 1j * t * r * np.sin(theta)) / J
    return z, sigma, r


def ellipse_poles_and_weights(J: int, t: float, r: float, centre: complex = 0.0):
    """Unshifted trapezoid rule on the ellipse of eq. ellipse, angles (2j-1) pi/J."""
    theta = (2 * np.arange(1, J + 1) - 1) * math.pi / J
    z = centre + t * r * np.cos(theta) + 1j * r * np.sin(theta)
    sigma = (r * np.cos(theta) + 1j * t * r * np.sin(theta)) / J
    return z, sigma


def filter_value(lam, z, sigma):
    """h_J(lambda) = sum_j sigma_j / (z_j (lambda - z_j)), the scalar image of the quadrature."""
    lam = np.asarray(lam, dtype=np.complex128)
    out = np.zeros(lam.shape, dtype=np.complex128)
    for zj, sj in zip(z, sigma):
        out += sj / (zj * (lam - zj))
    return out


def inside_contour(lam, J: int, t: float, eps: float, rho2: float):
    """True where lambda lies inside the (shifted) ellipse of Sec. 6.2."""
    phi = math.pi / J
    r = (rho2 / 2.0 + eps) / math.sin(phi)
    centre = -t * r * math.cos(phi) - 1j * rho2 / 2.0
    d = np.asarray(lam) - centre
    return (d.real / (t * r)) ** 2 + (d.imag / r) ** 2 < 1.0
