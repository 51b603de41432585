"""Leading-order analytic polygon counts (Sec. 4.1 and Appendix B).

TEST INFRASTRUCTURE ONLY: sanity comparisons of the exact counts with the
paper's approximations, which it reports to hold to roughly 10-20 % for
triangles away from the largest scales and about 40 % for quadrilaterals.
Wavenumbers and the bin width are in units of k_F, so the k_F powers drop out.
"""
from __future__ import annotations

import math


def n_tri_leading(k1: float, k2: float, k3: float, dk: float) -> float:
    """Number of triangles to leading order in the bin width (label eq:Ntri).

    8 pi^2 k1 k2 k3 dk^3 for an open triangle, half of that for a folded one
    (largest side equal to the sum of the other two), zero when it cannot close.
    """
    a, b, c = sorted((k1, k2, k3), reverse=True)
    if a > b + c:
        return 0.0
    base = 8.0 * math.pi ** 2 * k1 * k2 * k3 * dk ** 3
    return 0.5 * base if a == b + c else base


def n_quad_leading(k1: float, k2: float, k3: float, k4: float, dk: float) -> float:
    """Number of quadrilaterals to leading order (label eq:Nquad), k1 >= k2 >= k3 >= k4."""
    return 8.0 * math.pi ** 3 * dk ** 4 * k1 * k2 * k3 * k4 * (
        -k1 + k2 + k3 + 3.0 * k4 - abs(k1 - k2 - k3 + k4))
