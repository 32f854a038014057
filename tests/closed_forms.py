"""Closed-form potentials used to pin the oracle (test-side, independent code).

All potentials carry the 1/(4 pi) of eq. approx1, u = 1/(4 pi) int M . grad'(1/|r-r'|).

For a box with affine magnetisation M(r) = A r + b the potential is that of
the surface charge sigma = M.n on the six faces plus the volume charge
-div M = -tr A (integration by parts of eq. approx1):

    u(x) = 1/(4 pi) [ sum_faces int_f sigma/|x-y| dA - tr(A) int_box 1/|x-y| dV ]

The face integrals of 1, a and b over a rectangle (a, b the in-plane offsets
from x, z the height of x) and the box integral of 1/r have elementary
antiderivatives, summed over the corners with alternating signs.
"""
import math

import numpy as np


def _ln_b_plus_R(b, R, q):
    """ln(b + R) with q = R^2 - b^2 >= 0, free of cancellation for b < 0."""
    if b >= 0.0:
        return math.log(b + R)
    return math.log(q / (R - b))


def _F1(a, b, z):
    """Antiderivative of 1/R over the rectangle: a ln(b+R) + b ln(a+R) - z atan(ab/(zR))."""
    R = math.sqrt(a * a + b * b + z * z)
    s = 0.0
    if a != 0.0:
        s += a * _ln_b_plus_R(b, R, a * a + z * z)
    if b != 0.0:
        s += b * _ln_b_plus_R(a, R, b * b + z * z)
    if z != 0.0 and a != 0.0 and b != 0.0:
        s -= z * math.atan(a * b / (z * R))
    return s


def _Fa(a, b, z):
    """Antiderivative of a/R over the rectangle: (b R + (a^2+z^2) ln(b+R))/2."""
    R = math.sqrt(a * a + b * b + z * z)
    q = a * a + z * z
    s = b * R
    if q > 0.0:
        s += q * _ln_b_plus_R(b, R, q)
    return 0.5 * s


def _Fb(a, b, z):
    return _Fa(b, a, z)


def _corners2(F, a1, a2, b1, b2, z):
    return F(a2, b2, z) - F(a1, b2, z) - F(a2, b1, z) + F(a1, b1, z)


def _F3(a, b, c):
    """Antiderivative of 1/R over a box (cyclic sum of q r ln(p+R) - p^2/2 atan(q r/(p R)))."""
    R = math.sqrt(a * a + b * b + c * c)
    s = 0.0
    for p, q, r in ((a, b, c), (b, c, a), (c, a, b)):
        if q != 0.0 and r != 0.0:
            s += q * r * _ln_b_plus_R(p, R, q * q + r * r)
        if p != 0.0 and q != 0.0 and r != 0.0:
            s -= 0.5 * p * p * math.atan(q * r / (p * R))
    return s


def box_newton_potential(x, lo, hi):
    """int_box 1/|x - y| dV for the box [lo, hi]."""
    s = 0.0
    for i, ax in enumerate((lo[0], hi[0])):
        for j, ay in enumerate((lo[1], hi[1])):
            for k, az in enumerate((lo[2], hi[2])):
                sg = 1.0 if (i + j + k) % 2 == 1 else -1.0
                s += sg * _F3(ax - x[0], ay - x[1], az - x[2])
    return s


def box_potential_affine(x, A, b, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """u(x) of the box [lo, hi] magnetised with M(r) = A r + b."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tot = 0.0
    for k in range(3):
        i, j = [d for d in range(3) if d != k]
        for s, sg in ((hi[k], 1.0), (lo[k], -1.0)):
            alpha = sg * (A[k, i] * x[i] + A[k, j] * x[j] + A[k, k] * s + b[k])
            beta = sg * A[k, i]
            gamma = sg * A[k, j]
            z = s - x[k]
            a1, a2, b1, b2 = lo[i] - x[i], hi[i] - x[i], lo[j] - x[j], hi[j] - x[j]
            if alpha != 0.0:
                tot += alpha * _corners2(_F1, a1, a2, b1, b2, z)
            if beta != 0.0:
                tot += beta * _corners2(_Fa, a1, a2, b1, b2, z)
            if gamma != 0.0:
                tot += gamma * _corners2(_Fb, a1, a2, b1, b2, z)
    tr = A[0, 0] + A[1, 1] + A[2, 2]
    if tr != 0.0:
        tot -= tr * box_newton_potential(x, lo, hi)
    return tot / (4.0 * math.pi)


def box_potential_uniform(x, M, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    return box_potential_affine(x, np.zeros((3, 3)), M, lo, hi)
