"""Analytic polygon counts (Appendix B) against closed forms, an exact sum rule and the lattice.

* the general-order leading term against the paper's triangle and quadrilateral
  formulas (labels eq:Ntri, eq:Nquad), for every choice of the two singled-out sides;
* the exact-transform count against the continuous pair-sum rule (every pair sum
  q_1 + q_2 lands in exactly one shell: sum over k_3 of the count is the product of
  the two shell volumes), against the leading term as the width shrinks, and against
  the paper's collinear closed forms (labels eq:bicol, eq:tricol);
* both against the exact lattice counts of the estimator (the oracle's integer route).
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import analytic as OA
from paper_1904_11055_amd import analytic as A


def _shell_volume(k, dk):
    return 4.0 * math.pi / 3.0 * ((k + dk / 2) ** 3 - (k - dk / 2) ** 3)


@pytest.mark.parametrize("ks", [(10, 7, 5), (10, 6, 4), (9, 5, 4), (12, 12, 1), (3.5, 2.0, 1.5)])
def test_leading_triangles_match_eq_ntri(ks):
    for perm in ((0, 1, 2), (2, 0, 1), (1, 2, 0)):
        got = A.polygon_count_leading([ks[i] for i in perm], 1.0)
        assert got == pytest.approx(OA.n_tri_leading(*ks, 1.0), rel=1e-12)


@pytest.mark.parametrize("ks", [(10, 7, 5, 3), (9, 6, 5, 4), (12, 5, 4, 4), (8, 8, 8, 8), (10, 5, 3, 3),
                                (10, 5, 3, 2)])
def test_leading_quadrilaterals_match_eq_nquad(ks):
    """Closing quadrilaterals only: outside the polygon condition the printed formula goes negative."""
    ref = OA.n_quad_leading(*ks, 1.0)
    for perm in ((0, 1, 2, 3), (3, 2, 1, 0), (1, 3, 0, 2)):
        got = A.polygon_count_leading([ks[i] for i in perm], 1.0)
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-9)


def test_leading_open_folded_and_impossible_polygons():
    assert A.polygon_count_leading((10, 4, 3), 1.0) == 0.0
    assert A.polygon_count_leading((10, 4, 3, 2), 1.0) == 0.0
    assert A.polygon_count_leading((7, 4, 3), 1.0) == pytest.approx(0.5 * 8 * math.pi ** 2 * 84, rel=1e-12)
    assert A.polygon_count_leading((10, 4, 3, 3), 1.0) == 0.0        # collinear: zero at leading order
    assert A.polygon_count_leading((9, 4, 3, 3, 2), 1.0) > 0.0       # pentagon, n = 5


@pytest.mark.parametrize("k1,k2", [(7, 3), (9, 5), (6.5, 2.5)])
def test_exact_counts_obey_the_continuous_pair_sum_rule(k1, k2):
    total = sum(A.polygon_count_exact((k1, k2, k3), 1.0) for k3 in np.arange(1, k1 + k2 + 2))
    assert total == pytest.approx(_shell_volume(k1, 1.0) * _shell_volume(k2, 1.0), rel=1e-9)


def test_exact_counts_approach_the_leading_term():
    for dk in (0.2, 0.1):
        assert A.polygon_count_exact((10, 7, 5), dk) == pytest.approx(
            A.polygon_count_leading((10, 7, 5), dk), rel=1e-9)
    # quadrilaterals: the correction falls as dk^2
    r = [A.polygon_count_exact((9, 6, 5, 4), dk) / A.polygon_count_leading((9, 6, 5, 4), dk) - 1
         for dk in (0.2, 0.1, 0.05)]
    assert 3.5 < r[0] / r[1] < 4.5 and 3.5 < r[1] / r[2] < 4.5
    assert abs(r[2]) < 1e-4


@pytest.mark.parametrize("k2,k3", [(4, 3), (6, 2), (5, 5), (1, 1), (7.5, 1.5)])
def test_collinear_triangles_match_eq_bicol(k2, k3):
    exact = A.polygon_count_exact((k2 + k3, k2, k3), 1.0)
    assert A.triangle_count_collinear(k2, k3, 1.0) == pytest.approx(exact, rel=1e-8)


@pytest.mark.parametrize("k2,k3,k4", [(4, 3, 2), (5, 3, 3), (3, 2, 1), (6, 4, 1), (4, 1, 1), (2, 1, 1),
                                      (1, 1, 1)])
def test_collinear_quadrilaterals_match_eq_tricol(k2, k3, k4):
    """All four branches; the k_2 = dk branch with the constant the other branches imply."""
    exact = A.polygon_count_exact((k2 + k3 + k4, k2, k3, k4), 1.0)
    assert A.quadrilateral_count_collinear(k2, k3, k4, 1.0) == pytest.approx(exact, rel=1e-8)


def test_lattice_counts_against_the_continuous_ones():
    """Open polygons at large k agree to a few percent; collinear quadrilaterals, which the
    leading term misses entirely, are within a factor 1.5 of the exact continuous count."""
    N = 64
    tri = [(10, 12, 14), (6, 8, 10)]
    quad_open = [(6, 7, 8, 9)]
    quad_col = [(3, 3, 4, 10), (3, 4, 5, 12), (4, 4, 5, 13)]
    n3 = O.polygon_counts_exact(N, 3, 16, 1.0, np.array(tri))
    n4 = O.polygon_counts_exact(N, 4, 16, 1.0, np.array(quad_open + quad_col))
    for t, n in zip(tri, n3):
        assert A.polygon_count_exact(sorted(t, reverse=True), 1.0) == pytest.approx(n, rel=0.10)
    assert A.polygon_count_exact((9, 8, 7, 6), 1.0) == pytest.approx(n4[0], rel=0.05)
    for t, n in zip(quad_col, n4[1:]):
        ks = sorted(t, reverse=True)
        assert A.polygon_count_leading(ks, 1.0) == 0.0
        cont = A.quadrilateral_count_collinear(*ks[1:], 1.0)
        assert 1 / 1.5 < cont / n < 1.5
