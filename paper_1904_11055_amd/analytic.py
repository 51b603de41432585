"""Analytic polygon counts: the continuous approximations of Appendix B (CPU).

The estimator's normalisation is the number of closed n-gons with one side in each
shell, which the library counts exactly on the lattice (``Plan.counts``).  The paper
compares those counts with continuous approximations; this module provides them for
such comparisons (wavenumbers and shell widths in units of the fundamental k_F, so a
count is the continuous volume divided by k_F^(3(n-1))).

* Sec. 4.1 and Appendix B: the volume of closed n-gons is the radial integral
  V_n = (1 / 2 pi^2) int_0^inf x^2 prod_j iota_{k_j}(x) dx of the transforms
  iota_k(x) of the shells.
* To leading order in the shell width (label eq:approx), iota_k(x) = 4 pi k dk sin(kx)/x,
  and the radial integral reduces (label eq:master) to an integral of Dirac deltas over
  n - 2 box variables: an exact piecewise polynomial, evaluated here for every n >= 3
  (it gives the paper's triangle and quadrilateral formulas, labels eq:Ntri, eq:Nquad).
* Without that approximation (label eq:iota_exact) the transform of a shell of width
  dk decays as 1/x^2, so the radial integral converges absolutely and is evaluated
  here by quadrature; it stays accurate for collinear polygons, where the leading
  order gives half (triangles) or nothing (n >= 4).
* The paper's closed forms for collinear triangles and quadrilaterals (labels eq:bicol,
  eq:tricol) are provided in terms of the shorter sides, as printed except for one
  constant: the branch k_2 = dk of eq:tricol is printed with 12364288, but both the
  exact radial integral and the paper's own k_3 = dk branch at k_2 = dk give
  128 x 96569 = 12360832, which is used here.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = ["shell_transform", "polygon_count_leading", "polygon_count_exact",
           "triangle_count_collinear", "quadrilateral_count_collinear"]


def shell_transform(k: float, dk: float, x, exact: bool = True):
    """iota_k(x): the 3-D Fourier transform of the shell k - dk/2 <= |q| < k + dk/2 at radius x.

    exact=False gives the leading order 4 pi k dk sin(kx)/x (label eq:approx); exact=True
    the full shell integral 4 pi int q^2 sin(qx)/(qx) dq (label eq:iota_exact), whose value
    at x = 0 is the shell volume.
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-6
    xs = np.where(small, 1.0, x)
    if exact:
        h = 0.5 * dk
        val = (-xs * dk * np.cos(k * xs) * np.cos(xs * h)
               + 2.0 * (np.cos(k * xs) + k * xs * np.sin(k * xs)) * np.sin(xs * h)) / xs ** 3
        vol = ((k + h) ** 3 - (k - h) ** 3) / 3.0
        out = 4.0 * math.pi * np.where(small, vol, val)
    else:
        out = 4.0 * math.pi * k * dk * np.where(small, k, np.sin(k * xs) / xs)
    return out


def _box_convolution(widths, s: float) -> float:
    """int prod_i dkappa_i delta(sum_i kappa_i - s), kappa_i in [-w_i, w_i].

    The density of a sum of independent uniform variables (times prod 2 w_i): with
    m boxes, (1/(m-1)!) sum over signs e of (prod e_i) (s + sum e_i w_i)_+^(m-1), the
    positive part of a zero power being 1 above zero and 1/2 at zero (the paper's
    convention for the Heaviside function of a collinear polygon).
    """
    m = len(widths)
    tot = 0.0
    for signs in itertools.product((1.0, -1.0), repeat=m):
        t = s + sum(e * w for e, w in zip(signs, widths))
        if m == 1:
            p = 1.0 if t > 0 else (0.5 if t == 0 else 0.0)
        else:
            p = t ** (m - 1) if t > 0 else 0.0
        tot += math.prod(signs) * p
    return tot / math.factorial(m - 1)


def polygon_count_leading(ks, dk: float) -> float:
    """Leading-order number of closed n-gons with sides in shells k_1..k_n (n >= 3).

    N = 2^n pi^(n-1) dk^n (prod k_j) [C(k_b - k_a) - C(k_a + k_b)], C the convolution
    of boxes of half-widths k over the other n - 2 sides (label eq:master with two sides
    k_a, k_b singled out; the result does not depend on which).  Zero when the polygon
    cannot close (a side longer than the sum of the others).
    """
    ks = [float(k) for k in ks]
    n = len(ks)
    if n < 3:
        raise ValueError("polygon_count_leading needs n >= 3 sides")
    ka, kb, rest = ks[0], ks[1], ks[2:]
    bracket = _box_convolution(rest, kb - ka) - _box_convolution(rest, ka + kb)
    return 2.0 ** n * math.pi ** (n - 1) * dk ** n * math.prod(ks) * bracket


def polygon_count_exact(ks, dk: float, x_max: float | None = None, points_per_unit: int = 64) -> float:
    """Number of closed n-gons from the exact shell transforms (label eq:iota_exact), n >= 2.

    (1 / 2 pi^2) int_0^inf x^2 prod_j iota_{k_j}(x) dx by composite Simpson quadrature on
    [0, x_max]; the integrand decays as x^(2 - 2n), so the neglected tail is below
    x_max^(3 - 2n) times the product of the shell sizes.
    """
    ks = [float(k) for k in ks]
    n = len(ks)
    if n < 2:
        raise ValueError("polygon_count_exact needs n >= 2 sides")
    ktot = sum(ks) + n * dk
    if x_max is None:
        x_max = 400.0 / dk
    m = int(points_per_unit * ktot * x_max / (2.0 * math.pi)) + 1
    m += m % 2                                  # Simpson needs an even number of intervals
    x = np.linspace(0.0, x_max, m + 1)
    f = x ** 2
    for k in ks:
        f = f * shell_transform(k, dk, x, exact=True)
    w = np.ones(m + 1)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    integral = (x_max / m) / 3.0 * float(np.dot(w, f))
    return integral / (2.0 * math.pi ** 2)


def triangle_count_collinear(k2: float, k3: float, dk: float) -> float:
    """Closed form for collinear triangles k_1 = k_2 + k_3 (label eq:bicol)."""
    return 32.0 * math.pi ** 2 / 6144.0 * dk ** 3 * (
        104.0 * k3 ** 2 * dk + 5.0 * dk ** 3 + 8.0 * k2 ** 2 * (96.0 * k3 + 13.0 * dk)
        + 8.0 * k2 * k3 * (96.0 * k3 + 13.0 * dk))


def quadrilateral_count_collinear(k2: float, k3: float, k4: float, dk: float) -> float:
    """Closed form for collinear quadrilaterals k_1 = k_2 + k_3 + k_4, k_2 >= k_3 >= k_4 >= dk
    (label eq:tricol; its four branches for k_4 > dk and for k_4, k_3 or k_2 equal to dk)."""
    c = 128.0 * math.pi ** 3 / 725760.0
    if k2 == dk:
        return 12360832.0 * math.pi ** 3 * dk ** 9 / 725760.0   # 128 x 96569 (see the module notes)
    if k3 == dk:
        return c * dk ** 7 * (29196.0 * k2 ** 2 + 58392.0 * k2 * dk + 8981.0 * dk ** 2)
    if k4 == dk:
        return c * dk ** 6 * (24948.0 * k2 ** 2 * k3 + 24948.0 * k2 * k3 ** 2
                              + 36.0 * (118.0 * k2 ** 2 + 811.0 * k2 * k3 + 118.0 * k3 ** 2) * dk
                              + 4248.0 * (k2 + k3) * dk ** 2 + 485.0 * dk ** 3)
    a = 105.0 * k4 + 13.0 * dk
    return c * dk ** 5 * (
        dk * (468.0 * k4 ** 2 * dk + 17.0 * dk ** 3 + 36.0 * k3 ** 2 * a + 36.0 * k3 * k4 * a)
        + 36.0 * k2 ** 2 * (21.0 * k3 * (28.0 * k4 + 5.0 * dk) + dk * a)
        + 36.0 * k2 * (21.0 * k3 ** 2 * (28.0 * k4 + 5.0 * dk) + k4 * dk * a
                       + k3 * (588.0 * k4 ** 2 + 210.0 * k4 * dk + 13.0 * dk ** 2)))
