"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* exact lattice counts from the sum-of-three-squares theta series,
* direct n-gon enumeration (the estimator's definition, Sec. 2),
* the pair-sum rule for triangle counts and its recursion to orders 4 to 6,
* the n = 2 reduction to the shell-averaged |delta_hat|^2 (Parseval),
* the unit spectrum giving a unit polyspectrum (Sec. 4: counting by delta(k) = 1),
* homogeneity, translation and lattice symmetry,
* the paper's leading-order triangle counts (label eq:Ntri) as a loose sanity check,
* the gradient against a closed form (n = 2) and central differences (n = 3).
"""
import itertools
import os

import numpy as np
import pytest

import fieldgen
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _r3_theta(qmax):
    """r3(Q): number of integer (a, b, c) with a^2 + b^2 + c^2 = Q, as the coefficients of theta^3."""
    theta = np.zeros(qmax + 1, dtype=np.int64)
    k = 0
    while k * k <= qmax:
        theta[k * k] += 1 if k == 0 else 2
        k += 1
    t2 = np.convolve(theta, theta)[: qmax + 1]
    return np.convolve(t2, theta)[: qmax + 1]


@pytest.mark.parametrize("width", [1.0, 2.0, 1.5, 0.75])
def test_shell_mode_counts_match_theta_series(width):
    nb = 12
    T = O.shell_thresholds(nb, width)
    r3 = _r3_theta(T[-1])
    expect = [int(r3[T[s]:T[s + 1]].sum()) for s in range(nb)]
    N = 2 * int(np.ceil((nb + 0.5) * width)) + 2
    assert list(O.shell_mode_counts(N, nb, width)) == expect


def test_shell_edges_half_open():
    # width 2: edges at odd radii; |q| = 3 (e.g. (2,2,1)) opens shell 2, |q| = 1 opens shell 1.
    s = O.shell_of_squared_norm(np.array([0, 1, 8, 9, 24, 25, 120, 121]), 5, 2.0)
    assert list(s) == [0, 1, 1, 2, 2, 3, 5, 0]
    # width 1: |q|^2 = 2 (|q| = 1.414) in shell 1, 3 (1.732) in shell 2.
    s = O.shell_of_squared_norm(np.array([0, 1, 2, 3, 6, 7]), 3, 1.0)
    assert list(s) == [0, 1, 1, 2, 2, 3]


def test_golden_shell_modes_width1():
    got = O.shell_mode_counts(132, 64, 1.0)
    ref = np.loadtxt(os.path.join(GOLDEN, "shell_modes_width1.txt"), dtype=np.int64)
    assert np.array_equal(got, ref[:, 1])
    T = O.shell_thresholds(64, 1.0)
    r3 = _r3_theta(T[-1])
    assert [int(r3[T[s]:T[s + 1]].sum()) for s in range(64)] == list(ref[:, 1])


@pytest.mark.parametrize("order,nb,width", [(2, 7, 1.0), (3, 4, 1.0), (4, 3, 1.0),
                                            (3, 3, 2.0), (3, 6, 1.0), (4, 4, 1.0)])
def test_fft_estimator_equals_direct_enumeration(order, nb, width):
    N = 16
    delta = fieldgen.gaussian_field(N, 11 + order)
    r = O.polyspectrum(delta, order, nb, width, allow_aliasing=True)
    cnt, sums = O.bruteforce_polyspectrum(delta, order, nb, width, r["candidates"])
    assert np.array_equal(cnt, r["candidate_counts"])
    keep = cnt > 0
    scale = np.abs(sums).max()
    assert np.abs(sums.imag).max() <= 1e-12 * scale
    np.testing.assert_allclose(sums[keep].real * N ** 3, r["sums"],
                               rtol=0, atol=1e-12 * scale * N ** 3)
    np.testing.assert_allclose(sums[keep].real / cnt[keep], r["B"], rtol=1e-10,
                               atol=1e-12 * np.abs(r["B"]).max())


# Orders 5 and 6 (Sec. 4.2 extends the estimator to pentagons and hexagons).  The
# enumeration cost grows as the product of the first n - 1 shell sizes, so order 6
# is pinned on the tuples whose first five shells hold at most 18^3 62^2 vectors.
@pytest.mark.parametrize("N,order,nb,tuples", [
    (16, 5, 2, None), (16, 6, 1, None), (8, 5, 2, None),
    (8, 6, 2, [(1, 1, 1, 1, 1, 1), (1, 1, 1, 1, 1, 2), (1, 1, 1, 1, 2, 2), (1, 1, 1, 2, 2, 2)])])
def test_high_order_estimator_equals_direct_enumeration(N, order, nb, tuples):
    delta = fieldgen.gaussian_field(N, 20 + order)
    r = O.polyspectrum(delta, order, nb, 1.0, allow_aliasing=True)
    cand = [tuple(t) for t in r["candidates"].tolist()]
    pick = np.arange(len(cand)) if tuples is None else np.array([cand.index(t) for t in tuples])
    t = r["candidates"][pick]
    cnt, sums = O.bruteforce_polyspectrum(delta, order, nb, 1.0, t)
    assert np.array_equal(cnt, r["candidate_counts"][pick])
    assert np.array_equal(cnt, O.polygon_counts_exact(N, order, nb, 1.0, t))
    assert np.all(cnt > 0)
    scale = np.abs(sums).max()
    assert np.abs(sums.imag).max() <= 1e-12 * scale
    kept = {tuple(u): n for n, u in enumerate(r["tuples"].tolist())}
    rows = np.array([kept[tuple(u)] for u in t.tolist()])
    np.testing.assert_allclose(sums.real * N ** 3, r["sums"][rows], rtol=0, atol=1e-12 * scale * N ** 3)
    np.testing.assert_allclose(sums.real / cnt, r["B"][rows], rtol=1e-10)


@pytest.mark.parametrize("order", [4, 5, 6])
def test_polygon_recursion_rule(order):
    """sum_s n(t, s) = prod_j |S_{t_j}| - n(t) over (n-1)-tuples t whose vector sums always land in a shell.

    Every ordered (n-1)-tuple of vectors either closes (counted by n(t)) or sums to a
    non-zero q, and q lies in exactly one shell s when sum_j (t_j + 1/2) <= N_b + 1/2;
    then -q in shell s closes the n-gon.  Components stay below N/2 at N = 32, so
    closure modulo N is true closure for every tuple involved.
    """
    N, nb, width = 32, 9, 1.0
    S = O.shell_mode_counts(N, nb, width)
    heads = [t for t in O.sorted_tuples(order - 1, nb).tolist() if 2 * sum(t) + len(t) <= 2 * nb + 1]
    assert len(heads) >= 3
    full = sorted({tuple(sorted(h + [s])) for h in heads for s in range(1, nb + 1)})
    n_full = dict(zip(full, O.polygon_counts(N, order, nb, width, np.array(full)).tolist()))
    n_head = O.polygon_counts(N, order - 1, nb, width, np.array(heads)).tolist()
    for h, nh in zip(heads, n_head):
        tot = sum(n_full[tuple(sorted(h + [s]))] for s in range(1, nb + 1))
        assert tot == int(np.prod([S[u - 1] for u in h])) - nh


def test_aliased_flag_required():
    with pytest.raises(ValueError):
        O.polyspectrum(np.zeros((16, 16, 16)), 3, 6, 1.0)


def test_candidates_cover_every_closing_tuple():
    N, nb = 16, 4
    allt = O.sorted_tuples(3, nb)
    cnt, _ = O.bruteforce_polyspectrum(np.ones((N, N, N)), 3, nb, 1.0, allt)
    cand = {tuple(t) for t in O.candidate_tuples(3, nb, True).tolist()}
    assert {tuple(t) for t, c in zip(allt.tolist(), cnt) if c > 0} <= cand


def _counts_table(N, order, nb, width):
    cand = O.candidate_tuples(order, nb, O.is_alias_free(N, order, nb, width))
    n = O.polygon_counts(N, order, nb, width, cand)
    return {tuple(t): int(c) for t, c in zip(cand.tolist(), n)}


@pytest.mark.parametrize("N,nb,width", [(64, 16, 1.0), (48, 7, 2.0)])
def test_pair_sum_rule(N, nb, width):
    """sum_k n(i, j, k) = |S_i||S_j| - [i = j] |S_i| whenever q_1 + q_2 always lands in a shell."""
    table = _counts_table(N, 3, nb, width)
    S = O.shell_mode_counts(N, nb, width)
    checked = 0
    for i in range(1, nb + 1):
        for j in range(i, nb + 1):
            if i + j + 1 > nb:
                continue
            tot = sum(table.get(tuple(sorted((i, j, k))), 0) for k in range(1, nb + 1))
            assert tot == S[i - 1] * S[j - 1] - (S[i - 1] if i == j else 0)
            checked += 1
    assert checked > 0


def test_small_triangle_counts():
    table = _counts_table(64, 3, 16, 1.0)
    cnt, _ = O.bruteforce_polyspectrum(np.ones((16, 16, 16)), 3, 3, 1.0,
                                       np.array([(1, 1, 1), (1, 1, 2), (1, 1, 3), (1, 2, 2),
                                                 (1, 2, 3), (2, 2, 2), (2, 2, 3)]))
    got = [table[t] for t in [(1, 1, 1), (1, 1, 2), (1, 1, 3), (1, 2, 2), (1, 2, 3),
                              (2, 2, 2), (2, 2, 3)]]
    assert got == list(cnt) == [120, 174, 12, 456, 414, 912, 944]


def test_golden_bispec64_counts():
    ref = np.loadtxt(os.path.join(GOLDEN, "bispec_64_counts.txt"), dtype=np.int64)
    assert ref.shape == (564, 4)
    S = O.shell_mode_counts(64, 16, 1.0)
    table = {tuple(r[:3]): int(r[3]) for r in ref}
    for i in range(1, 17):
        for j in range(i, 17):
            if i + j + 1 <= 16:
                tot = sum(table.get(tuple(sorted((i, j, k))), 0) for k in range(1, 17))
                assert tot == S[i - 1] * S[j - 1] - (S[i - 1] if i == j else 0)


def test_power_spectrum_parseval():
    N, nb = 32, 10
    delta = fieldgen.gaussian_field(N, 5)
    r = O.polyspectrum(delta, 2, nb, 1.0)
    dhat = np.fft.fftn(delta)
    sid = O.shell_id_grid(N, nb, 1.0, half=False)
    ref = np.array([np.mean(np.abs(dhat[sid == s]) ** 2) for s in range(1, nb + 1)])
    assert [tuple(t) for t in r["tuples"].tolist()] == [(s, s) for s in range(1, nb + 1)]
    np.testing.assert_allclose(r["B"], ref, rtol=1e-11)
    np.testing.assert_array_equal(r["counts"], O.shell_mode_counts(N, nb, 1.0))


@pytest.mark.parametrize("order,nb", [(3, 8), (4, 5), (5, 4), (6, 3)])
def test_unit_spectrum_gives_unit_polyspectrum(order, nb):
    N = 32
    r = O.polyspectrum(fieldgen.unit_spectrum_field(N), order, nb, 1.0)
    np.testing.assert_allclose(r["B"], 1.0, rtol=1e-11)


def test_homogeneity_and_symmetries():
    N, nb = 32, 8
    delta = fieldgen.lognormal_field(N, 7)
    base = O.polyspectrum(delta, 3, nb, 1.0)
    counts = base["candidate_counts"]
    twice = O.polyspectrum(2.0 * delta, 3, nb, 1.0, counts=counts)
    np.testing.assert_array_equal(twice["B"], 8.0 * base["B"])
    scale = np.abs(base["B"]).max()
    for moved in (np.roll(delta, (3, -5, 7), axis=(0, 1, 2)),
                  np.transpose(delta, (2, 0, 1)),
                  delta[::-1, :, :]):
        r = O.polyspectrum(np.ascontiguousarray(moved), 3, nb, 1.0, counts=counts)
        np.testing.assert_allclose(r["B"], base["B"], rtol=0, atol=1e-11 * scale)
    # raw sums are symmetric in the tuple's order: compare (i, j, k) with its rotation
    d = O.shell_fields(delta, nb, 1.0)
    t = np.array([[1, 2, 3], [2, 2, 5]])
    rot = np.array([[3, 1, 2], [5, 2, 2]])
    s1 = [np.sum(d[a - 1] * d[b - 1] * d[c - 1]) for a, b, c in t]
    s2 = [np.sum(d[a - 1] * d[b - 1] * d[c - 1]) for a, b, c in rot]
    np.testing.assert_allclose(s1, O.product_sums(d, t), rtol=1e-12)
    np.testing.assert_allclose(s2, s1, rtol=1e-12)


def test_counts_near_leading_order_triangles():
    """Eq. Ntri to within the paper's quoted ~20 % for open triangles at large k."""
    table = _counts_table(64, 3, 16, 1.0)
    rel = []
    for (a, b, c), n in table.items():
        if a >= 8 and c < a + b:      # open triangles (largest side c < a + b), away from large scales
            rel.append(n / O.n_tri_leading(c, b, a, 1.0) - 1.0)
    rel = np.abs(np.array(rel))
    assert len(rel) > 20 and np.median(rel) < 0.2


def test_gradient_power_spectrum_closed_form():
    N, nb = 16, 5
    delta = fieldgen.gaussian_field(N, 21)
    r = O.polyspectrum(delta, 2, nb, 1.0, return_fields=True)
    s = 3
    g = np.zeros(len(r["tuples"]))
    g[s - 1] = 1.0
    grad = O.gradient(delta, 2, nb, 1.0, g, result=r)
    np.testing.assert_allclose(grad, 2.0 * r["fields"][s - 1] / r["counts"][s - 1],
                               rtol=0, atol=1e-12 * np.abs(grad).max())


def test_gradient_bispectrum_central_differences():
    N, nb = 16, 4
    delta = fieldgen.gaussian_field(N, 31)
    target = 0.5 * O.polyspectrum(fieldgen.gaussian_field(N, 32), 3, nb, 1.0)["B"]
    r = O.polyspectrum(delta, 3, nb, 1.0, return_fields=True)
    counts = r["candidate_counts"]
    grad = O.gradient(delta, 3, nb, 1.0, 2.0 * (r["B"] - target), result=r)

    def loss(dl):
        return np.sum((O.polyspectrum(dl, 3, nb, 1.0, counts=counts)["B"] - target) ** 2)

    rng = np.random.default_rng(3)
    eps = 1e-3
    for flat in rng.choice(N ** 3, size=6, replace=False):
        idx = np.unravel_index(flat, (N, N, N))
        dp = delta.copy(); dp[idx] += eps
        dm = delta.copy(); dm[idx] -= eps
        fd = (loss(dp) - loss(dm)) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * np.abs(grad).max()


def test_count_integrality_check_trips():
    with pytest.raises(ArithmeticError):
        O.counts_from_sums(np.array([64.0 ** 3 * 7.3]), 64)


def test_slab_fields_match_full_fields():
    N, nb = 32, 6
    delta = fieldgen.gaussian_field(N, 8)
    full = O.shell_fields(delta, nb, 1.0)
    planes = [0, 5, 31]
    part = O.shell_fields_on_planes(np.fft.rfftn(delta), N, nb, 1.0, planes)
    np.testing.assert_allclose(part, full[:, planes], rtol=0, atol=1e-10 * np.abs(full).max())
    cpart = O.shell_fields_on_planes(None, N, nb, 1.0, planes, unit=True)
    cfull = O.count_fields(N, nb, 1.0)
    np.testing.assert_allclose(cpart, cfull[:, planes], rtol=0, atol=1e-10 * np.abs(cfull).max())


def test_compensated_sums_recover_large_integers():
    """Chunk sums near 5e19 (a 256^3 quadrilateral count times N^3) add up to the right integer."""
    from fractions import Fraction
    N = 256
    rng = np.random.default_rng(0)
    n_true = 2930376455268
    vals = rng.uniform(0.5, 1.5, 4096) * (n_true * N ** 3 / 4096)
    rest = sum(Fraction(float(v)) for v in vals[:-1])
    vals[-1] = float(n_true * N ** 3 - rest)     # exact total within half an ulp of vals[-1]
    exact = rest + Fraction(float(vals[-1]))
    assert abs(exact / N ** 3 - n_true) < 1e-3
    hi = np.zeros(1)
    lo = np.zeros(1)
    plain = 0.0
    for v in vals:
        plain += v
        s_ = hi + v
        bb = s_ - hi
        lo += (hi - (s_ - bb)) + (v - bb)
        hi = s_
    assert abs(Fraction(float(hi[0])) + Fraction(float(lo[0])) - exact) < 1e-9 * N ** 3
    assert O.counts_from_sums((hi, lo), N)[0] == n_true
    assert abs(Fraction(plain) - exact) / N ** 3 > 1e-3   # the plain FP64 sum would miss


def test_compensated_product_sums_match_plain_on_small_grid():
    N, nb = 32, 6
    c = O.count_fields(N, nb, 1.0)
    t = O.candidate_tuples(4, nb, True)
    plain = O.counts_from_sums(O.product_sums(c, t), N)
    comp = O.counts_from_sums(O.product_sums(c, t, chunk=1000, compensated=True), N)
    assert np.array_equal(plain, comp)
    d = {s + 1: c[s] for s in range(nb)}
    assert np.array_equal(O.counts_from_sums(O.tuple_product_sums(d, t[:20]), N), plain[:20])


@pytest.mark.parametrize("order,nb", [(2, 7), (3, 6), (4, 4)])
def test_exact_counts_match_direct_enumeration(order, nb):
    """Aliased 16^3 grid: every sorted tuple, integer pair-count route against brute force."""
    N = 16
    t = O.sorted_tuples(order, nb)
    cnt, _ = O.bruteforce_polyspectrum(np.ones((N, N, N)), order, nb, 1.0, t)
    assert np.array_equal(O.polygon_counts_exact(N, order, nb, 1.0, t), cnt)


@pytest.mark.parametrize("order,nb,width", [(3, 16, 1.0), (4, 10, 1.0), (4, 6, 2.0), (5, 6, 1.0),
                                            (6, 5, 1.0)])
def test_exact_counts_match_fft_counts(order, nb, width):
    N = 64
    t = O.candidate_tuples(order, nb, O.is_alias_free(N, order, nb, width))
    assert np.array_equal(O.polygon_counts_exact(N, order, nb, width, t),
                          O.polygon_counts(N, order, nb, width, t))


def test_physical_units_match_standard_estimators():
    """With box side L: P(k) = V <|delta_k|^2> and B = V^2 <delta_k1 delta_k2 delta_k3>, delta_k = delta_hat / N^3."""
    N, L = 16, 250.0
    V = L ** 3
    delta = fieldgen.gaussian_field(N, 21)
    r2 = O.polyspectrum(delta, 2, 5, 1.0, box_length=L)
    dk = np.fft.fftn(delta) / N ** 3
    sid = O.shell_id_grid(N, 5, 1.0, half=False)
    ref = np.array([V * np.mean(np.abs(dk[sid == s]) ** 2) for s in range(1, 6)])
    np.testing.assert_allclose(r2["B"], ref, rtol=1e-11)
    r3 = O.polyspectrum(delta, 3, 4, 1.0, box_length=L)
    cnt, sums = O.bruteforce_polyspectrum(delta, 3, 4, 1.0, r3["tuples"])
    np.testing.assert_allclose(r3["B"], V ** 2 * (sums.real / cnt) / float(N) ** 9, rtol=1e-10)


@pytest.mark.parametrize("width,allow", [(1.0, False), (1.0, True)])
def test_gradient_trispectrum_central_differences(width, allow):
    """Order 4 (incl. an aliased plan): the adjoint against central differences of the FP64 forward."""
    N = 16
    nb = 3 if not allow else 4
    delta = fieldgen.lognormal_field(N, 41)
    kw = dict(allow_aliasing=allow)
    target = 0.5 * O.polyspectrum(fieldgen.lognormal_field(N, 42), 4, nb, width, **kw)["B"]
    r = O.polyspectrum(delta, 4, nb, width, return_fields=True, **kw)
    counts = r["candidate_counts"]
    grad = O.gradient(delta, 4, nb, width, 2.0 * (r["B"] - target), result=r, allow_aliasing=allow)

    def loss(dl):
        return np.sum((O.polyspectrum(dl, 4, nb, width, counts=counts, **kw)["B"] - target) ** 2)

    rng = np.random.default_rng(5)
    eps = 1e-3
    for flat in rng.choice(N ** 3, size=6, replace=False):
        idx = np.unravel_index(flat, (N, N, N))
        dp = delta.copy(); dp[idx] += eps
        dm = delta.copy(); dm[idx] -= eps
        fd = (loss(dp) - loss(dm)) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * np.abs(grad).max()


def test_adjoint_weights_sum_rule():
    """sum over m and rests of W = (order) * sum_t w_t: each tuple spreads its weight over its positions."""
    for order, nb in ((3, 6), (4, 5)):
        t = O.candidate_tuples(order, nb, True)
        w = np.linspace(0.5, 2.0, len(t))
        W = O.adjoint_weights(t, w, nb)
        assert np.isclose(W.sum(), order * w.sum())
        assert W.shape == (nb, len(O.sorted_tuples(order - 1, nb)))


@pytest.mark.parametrize("order,nb", [(3, 4), (4, 3)])
def test_gradient_half_spectrum_central_differences(order, nb):
    """dL/dRe X + i dL/dIm X for a half-spectrum input X, against central differences of
    the FP64 forward taken on X itself: modes in the q2 = 0 plane (read once by the inverse
    real transform) and with q2 > 0 (read twice), real and imaginary parts."""
    N = 16
    X = O.polyspec.rfftn(fieldgen.lognormal_field(N, 51))
    target = 0.5 * O.polyspectrum(fieldgen.lognormal_field(N, 52), order, nb, 1.0)["B"]
    r = O.polyspectrum_from_hat(X, N, order, nb, 1.0, return_fields=True)
    counts = r["candidate_counts"]
    G = O.gradient_half_spectrum(N, order, nb, 1.0, r["tuples"], r["counts"], r["fields"],
                                 2.0 * (r["B"] - target))

    def loss(Xp):
        return np.sum((O.polyspectrum_from_hat(Xp, N, order, nb, 1.0, counts=counts)["B"] - target) ** 2)

    sid = O.shell_id_grid(N, nb, 1.0)
    modes = [(1, 2, 0), (N - 2, 1, 0), (0, 1, 2), (3, N - 1, 1), (0, 0, 3), (2, 2, 2)]
    eps = 1e-3 * np.abs(X).max()
    scale = np.abs(G).max()
    for m in modes:
        assert sid[m] > 0
        for unit in (1.0, 1j):
            Xp = X.copy(); Xp[m] += eps * unit
            Xm = X.copy(); Xm[m] -= eps * unit
            fd = (loss(Xp) - loss(Xm)) / (2 * eps)
            got = G[m].real if unit == 1.0 else G[m].imag
            assert abs(fd - got) <= 1e-6 * scale, (m, unit, fd, got)


def test_gradient_on_a_shell_subset_matches_full():
    """With dL/dB zero on every tuple outside a shell subset, the gradient formed from the
    subset's fields alone is the full gradient."""
    N, nb, order = 16, 4, 3
    delta = fieldgen.gaussian_field(N, 53)
    r = O.polyspectrum(delta, order, nb, 1.0, return_fields=True)
    sub = [1, 2, 4]
    g = np.where([set(int(v) for v in t) <= set(sub) for t in r["tuples"]],
                 np.linspace(1.0, 2.0, len(r["tuples"])), 0.0)
    assert np.count_nonzero(g) > 0
    full = O.gradient_spectrum(N, order, nb, 1.0, r["tuples"], r["counts"], r["fields"], g)
    part = O.gradient_spectrum(N, order, nb, 1.0, r["tuples"], r["counts"],
                               r["fields"][np.array(sub) - 1], g, shells=sub)
    np.testing.assert_allclose(part, full, rtol=0, atol=1e-12 * np.abs(full).max())
    with pytest.raises(ValueError):
        O.gradient_spectrum(N, order, nb, 1.0, r["tuples"], r["counts"], r["fields"][np.array(sub) - 1],
                            np.ones(len(r["tuples"])), shells=sub)


# ---------------------------------------------------------------------------------------
# Redshift-space multipoles (Sec. 5: the estimator on multipole-weighted fields)
# ---------------------------------------------------------------------------------------
def test_multipole_zero_is_the_monopole_of_every_leg():
    """ell = 0 weights nothing: B_0(u, v; w) is the monopole of the sorted triangle."""
    delta = fieldgen.gaussian_field(32, 61)
    mono = O.polyspectrum(delta, 3, 6, 1.0)
    m0 = O.bispectrum_multipoles(delta, 6, 1.0, 0)
    lut = {tuple(t): b for t, b in zip(mono["tuples"].tolist(), mono["B"])}
    ref = np.array([lut[tuple(sorted(t))] for t in m0["tuples"].tolist()])
    np.testing.assert_allclose(m0["B"], ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    # every closing triangle appears once per distinct weighted side
    n_sides = sum(len(set(t)) for t in mono["tuples"].tolist())
    assert len(m0["tuples"]) == n_sides


def test_multipole_equals_direct_enumeration_with_the_legendre_weight():
    """B_2 against explicit enumeration of the closed triangles, each weighted by
    L_2(mu) of its last vector, mu the cosine to the third grid axis."""
    N, nb, width, ell = 16, 3, 1.0, 2
    delta = fieldgen.gaussian_field(N, 62)
    r = O.bispectrum_multipoles(delta, nb, width, ell)

    def weight(q):
        norm = np.sqrt((q.astype(np.float64) ** 2).sum(-1))
        mu = np.where(norm > 0, q[..., 2] / np.where(norm > 0, norm, 1.0), 0.0)
        return (3.0 * mu ** 2 - 1.0) / 2.0      # L_2, written out

    cnt, sums = O.bruteforce_polyspectrum(delta, 3, nb, width, r["tuples"], last_weight=weight)
    assert np.array_equal(cnt, r["counts"])
    scale = np.abs(sums).max()
    assert np.abs(sums.imag).max() <= 1e-12 * scale
    np.testing.assert_allclose(sums.real * N ** 3, r["sums"], rtol=0, atol=1e-12 * scale * N ** 3)
    np.testing.assert_allclose(5.0 * sums.real / cnt, r["B"], rtol=1e-10, atol=1e-12 * np.abs(r["B"]).max())


def test_quadrupoles_about_the_three_axes_sum_to_zero():
    """sum over the three axes of L_2(mu_axis) = (3 |q|^2 / |q|^2 - 3) / 2 = 0 for every
    mode, so the three quadrupoles of any field cancel exactly."""
    delta = fieldgen.lognormal_field(24, 63)
    parts = [O.bispectrum_multipoles(delta, 5, 1.0, 2, axis=a)["B"] for a in range(3)]
    total = parts[0] + parts[1] + parts[2]
    assert np.abs(total).max() <= 1e-11 * max(np.abs(p).max() for p in parts)
    assert np.abs(parts[2]).max() > 1e-3 * np.abs(O.polyspectrum(delta, 3, 5, 1.0)["B"]).max()


def test_odd_multipoles_are_refused():
    with pytest.raises(ValueError):
        O.bispectrum_multipoles(fieldgen.gaussian_field(16, 64), 3, 1.0, 1)
