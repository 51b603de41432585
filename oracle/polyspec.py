"""Plain FP64 implementation of the Scoccimarro-type FFT polyspectrum estimator.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the library.  Written from Tomlinson, Jeong & Kim
(2019), "Efficient parallel algorithm for estimating higher-order polyspectra":

* Sec. 2, the direct estimator (label eq:estimateBk) averages the product of the
  density at n wave vectors, one per shell, over every closed configuration.
* Sec. 2, the Fourier form of the Dirac delta turns that sum into the grid sum of
  a product of shell-filtered inverse transforms I_k(x) (labels eq:Bkfast and
  eq:estimator); the same sum on a unit field gives the polygon volume
  (labels eq:volume, eq:Vn).
* Appendix A writes the estimator with unnormalised DFTs (FFTW convention):
  B = (V_f^{n-1}/V_n) (V^{n-1}/N^{3n}) N^-3 sum_x prod_j FFTW(I~_{k_j}), and the
  polygon count as N^-3 sum_x prod_j FFTW(iota~_{k_j}) over unit shells.

Readings taken where the paper is loose (each is also listed in the design
notes of the repository):

* Shell s (s = 1..N_b) of width D holds the modes with (s - 1/2) D <= |q| < (s + 1/2) D,
  |q| in units of k_f.  The paper writes |q - k_i| < dk/2 with strict bounds; the
  half-open interval puts every mode with D/2 <= |q| < (N_b + 1/2) D in exactly one
  shell.  The DC mode is never binned.  Membership is decided exactly, in integers.
* delta_hat is the unnormalised forward DFT (e^{-i}) of the real grid field;
  shell fields use the unnormalised inverse (e^{+i}).  The sign of the exponent
  does not change a grid sum of real products.
* The polygon count is n_t = N^-3 sum_x prod_j c_{t_j}[x] (no extra V_f factor),
  which is exactly the number of ordered closed vector n-tuples with q_j in
  shell t_j (closure taken modulo N on the periodic grid).
* Output tuples are sorted t_1 <= ... <= t_n, lexicographic with t_n fastest,
  restricted to those with n_t > 0.
"""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np

try:
    import scipy.fft as _sfft

    def _workers():
        try:
            return max(1, len(os.sched_getaffinity(0)))
        except Exception:  # pragma: no cover
            return os.cpu_count() or 1

    def rfftn(a):
        return _sfft.rfftn(a, workers=_workers())

    def irfftn(a, s):
        return _sfft.irfftn(a, s=s, workers=_workers())

    def irfft2(a, s):
        return _sfft.irfft2(a, s=s, workers=_workers())
except Exception:  # pragma: no cover
    rfftn = np.fft.rfftn

    def irfftn(a, s):
        return np.fft.irfftn(a, s=s)

    def irfft2(a, s):
        return np.fft.irfft2(a, s=s)

__all__ = [
    "shell_thresholds", "shell_of_squared_norm", "squared_norm_grid", "shell_id_grid",
    "outer_radius", "is_alias_free", "sorted_tuples", "candidate_tuples", "pair_list",
    "shell_mode_counts", "shell_fields", "shell_fields_from_hat", "count_fields",
    "shell_fields_on_planes", "product_sums", "tuple_product_sums", "counts_from_sums", "polygon_counts",
    "pair_counts", "triple_counts", "polygon_counts_exact", "triple_list",
    "polyspectrum", "polyspectrum_from_hat", "adjoint_weights", "gradient", "gradient_spectrum",
    "gradient_half_spectrum", "physical_factor",
    "legendre", "los_cosine_grid", "multipole_fields_from_hat", "multipole_tuples", "bispectrum_multipoles",
]


# ----------------------------------------------------------------------------
# Binning (Sec. 2: a mode belongs to the bin of k_i when |q - k_i| < dk/2;
# Appendix A: the unit shell iota~ is 1 inside that shell and 0 elsewhere).
# ----------------------------------------------------------------------------
def shell_thresholds(n_shells: int, width: float) -> list[int]:
    """T_1..T_{N_b+1}: T_s is the smallest integer Q = |q|^2 with 4Q >= ((2s-1) D)^2.

    Shell s holds the integer squared norms T_s <= Q < T_{s+1}.  D is taken as the
    exact rational value of the float passed in, so the compare is exact.
    """
    D = Fraction(width)
    out = []
    for s in range(1, n_shells + 2):
        edge2 = ((2 * s - 1) * D) ** 2          # (2 |q|_edge)^2 = 4 Q_edge
        out.append(math.ceil(edge2 / 4))
    return out


def shell_of_squared_norm(Q: np.ndarray, n_shells: int, width: float) -> np.ndarray:
    """Shell index (1..N_b) of integer squared norms Q, 0 when Q lies in no shell."""
    T = np.asarray(shell_thresholds(n_shells, width), dtype=np.int64)
    Q = np.asarray(Q, dtype=np.int64)
    s = np.searchsorted(T, Q, side="right")     # number of thresholds <= Q
    s = np.where((s >= 1) & (s <= n_shells), s, 0)
    return s.astype(np.int64)


def squared_norm_grid(N: int, half: bool = True) -> np.ndarray:
    """Integer |q|^2 on the rfftn layout [N, N, N//2+1] (or the full [N, N, N])."""
    k = np.fft.fftfreq(N, d=1.0 / N).round().astype(np.int64)   # 0..N/2-1, -N/2..-1
    kz = np.arange(N // 2 + 1, dtype=np.int64) if half else k
    return k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2


def shell_id_grid(N: int, n_shells: int, width: float, half: bool = True) -> np.ndarray:
    return shell_of_squared_norm(squared_norm_grid(N, half), n_shells, width)


def outer_radius(n_shells: int, width: float) -> float:
    """K_e = (N_b + 1/2) D, the outer edge of the last shell in units of k_f."""
    return (n_shells + 0.5) * width


def is_alias_free(N: int, order: int, n_shells: int, width: float) -> bool:
    """n K_e <= N: no sum of n shell vectors can wrap around the periodic grid.

    Sec. 1 and Sec. 4.3 require a grid of at least (n N_max)^3 for the n-point
    function; with the outer edge K_e the exact condition is n K_e <= N.
    """
    return order * Fraction(width) * Fraction(2 * n_shells + 1, 2) <= N


def shell_mode_counts(N: int, n_shells: int, width: float) -> np.ndarray:
    """|S_s| for s = 1..N_b, counted over the full periodic grid."""
    sid = shell_id_grid(N, n_shells, width, half=False)
    return np.bincount(sid.ravel(), minlength=n_shells + 1)[1:]


# ----------------------------------------------------------------------------
# Tuples (Sec. 4.2: k_1 >= ... >= k_n, flattened row-major with k_n fastest;
# stored here in the equivalent ascending form t_1 <= ... <= t_n).
# ----------------------------------------------------------------------------
def sorted_tuples(order: int, n_shells: int) -> np.ndarray:
    """All t_1 <= ... <= t_n over shells 1..N_b, lexicographic, t_n fastest."""
    tl = list(itertools.combinations_with_replacement(range(1, n_shells + 1), order))
    return np.asarray(tl, dtype=np.int64).reshape(-1, order)


def candidate_tuples(order: int, n_shells: int, alias_free: bool = True) -> np.ndarray:
    """Sorted tuples that can close: t_n < t_1 + ... + t_{n-1} + n/2 when alias-free.

    |q_n| = |q_1 + ... + q_{n-1}| <= sum |q_j| < sum (t_j + 1/2) D, while q_n in
    shell t_n needs |q_n| >= (t_n - 1/2) D.  With wrap-around (aliasing) any
    sorted tuple can close modulo N, so every one is a candidate.
    """
    t = sorted_tuples(order, n_shells)
    if not alias_free:
        return t
    lhs = 2 * t[:, -1]
    rhs = 2 * t[:, :-1].sum(axis=1) + order
    return t[lhs < rhs]


def pair_list(n_shells: int) -> np.ndarray:
    """Pairs (i, j), 1 <= i <= j <= N_b, lexicographic."""
    return sorted_tuples(2, n_shells)


# ----------------------------------------------------------------------------
# Shell fields (Sec. 2, I_k(x) as the inverse transform of the shell-filtered
# density; Appendix A: I[x] = (2 pi)^3 / N^3 FFTW(I~[q]); the prefactor is
# pulled out, so the fields here are the raw unnormalised FFTW outputs).
# ----------------------------------------------------------------------------
def shell_fields_from_hat(delta_hat: np.ndarray, N: int, n_shells: int, width: float,
                          shells=None) -> np.ndarray:
    """d_s[x] = sum_q [s(q) = s] delta_hat[q] e^{+2 pi i q.x/N} for the requested shells."""
    sid = shell_id_grid(N, n_shells, width)
    shells = range(1, n_shells + 1) if shells is None else shells
    out = np.empty((len(shells), N, N, N), dtype=np.float64)
    for n, s in enumerate(shells):
        masked = np.where(sid == s, delta_hat, 0.0)
        out[n] = irfftn(masked, s=(N, N, N)) * float(N) ** 3
    return out


def shell_fields(delta: np.ndarray, n_shells: int, width: float, shells=None) -> np.ndarray:
    """Shell fields of a real field delta[x] (float64 [N, N, N])."""
    delta = np.asarray(delta, dtype=np.float64)
    N = delta.shape[0]
    return shell_fields_from_hat(rfftn(delta), N, n_shells, width, shells)


def count_fields(N: int, n_shells: int, width: float, shells=None) -> np.ndarray:
    """c_s[x]: the same transform of the unit shell iota~_s (Appendix A)."""
    sid = shell_id_grid(N, n_shells, width)
    shells = range(1, n_shells + 1) if shells is None else shells
    out = np.empty((len(shells), N, N, N), dtype=np.float64)
    for n, s in enumerate(shells):
        out[n] = irfftn((sid == s).astype(np.float64), s=(N, N, N)) * float(N) ** 3
    return out


def shell_fields_on_planes(delta_hat: np.ndarray, N: int, n_shells: int, width: float,
                           planes, shells=None, unit: bool = False) -> np.ndarray:
    """Shell fields restricted to the x0-planes listed (for grids too large to hold whole).

    The inverse transform along the first axis is evaluated only at the requested
    x0 as an explicit sum, then each plane is the 2-D inverse real transform of the
    remaining (q1, q2) half spectrum.  With unit=True the unit shells are used.
    """
    sid = shell_id_grid(N, n_shells, width)
    planes = np.asarray(planes, dtype=np.int64)
    shells = range(1, n_shells + 1) if shells is None else shells
    q0 = np.fft.fftfreq(N, d=1.0 / N).round().astype(np.int64)
    phase = np.exp(2j * np.pi * np.outer(planes, q0) / N)          # [P, N]
    out = np.empty((len(shells), len(planes), N, N), dtype=np.float64)
    for n, s in enumerate(shells):
        if unit:
            masked = (sid == s).astype(np.complex128)
        else:
            masked = np.where(sid == s, delta_hat, 0.0)
        g = (phase @ masked.reshape(N, -1)).reshape(len(planes), N, N // 2 + 1)
        out[n] = irfft2(g, s=(N, N)) * float(N) ** 2
    return out


# ----------------------------------------------------------------------------
# Product sums (Sec. 2: the grid sum of products of the shell fields;
# Appendix A: sum over [x] of prod_j FFTW(I~_{k_j})).
# ----------------------------------------------------------------------------
def triple_list(n_shells: int) -> np.ndarray:
    """Triples (i, j, k), 1 <= i <= j <= k <= N_b, lexicographic."""
    return sorted_tuples(3, n_shells)


def product_sums(fields: np.ndarray, tuples: np.ndarray, chunk: int = 8192, compensated: bool = False):
    """S_t = sum_x prod_j fields[t_j - 1][x] in FP64, for orders 2 to 6.

    The grid is summed in chunks.  Each tuple is split into a left and a right
    part -- a shell and a shell (order 2), a pair and a shell (3), a pair and a
    pair (4), a pair and a triple (5), a triple and a triple (6) -- whose products
    d_i d_j (d_k) are formed once per chunk and multiplied with a matrix product.
    With compensated=True the chunk results are added with error-free
    transformations and the pair (hi, lo) with S = hi + lo is returned (used for
    polygon counts, which reach 10^12 and must round to the right integer).
    """
    tuples = np.asarray(tuples, dtype=np.int64)
    order = tuples.shape[1]
    if order not in (2, 3, 4, 5, 6):
        raise ValueError("product_sums supports orders 2 to 6")
    nb = fields.shape[0]
    flat = fields.reshape(nb, -1)
    G = flat.shape[1]
    left = {2: 1, 3: 2, 4: 2, 5: 2, 6: 3}[order]     # factors in the left part
    lists = {1: sorted_tuples(1, nb), 2: pair_list(nb), 3: triple_list(nb)}
    lrows, rrows = lists[left], lists[order - left]
    lidx = {tuple(int(v) for v in r): n for n, r in enumerate(lrows)}
    ridx = {tuple(int(v) for v in r): n for n, r in enumerate(rrows)}
    acc = np.zeros((len(lrows), len(rrows)))
    lo = np.zeros_like(acc) if compensated else None

    def products(blk, rows):
        out = blk[rows[:, 0] - 1].copy()
        for c in range(1, rows.shape[1]):
            out *= blk[rows[:, c] - 1]
        return out

    for x0 in range(0, G, chunk):
        blk = flat[:, x0:x0 + chunk]
        L = products(blk, lrows)
        R = L if rrows is lrows else products(blk, rrows)
        part = L @ R.T
        if compensated:      # two-sum: acc + part = s + err exactly
            s_ = acc + part
            bb = s_ - acc
            lo += (acc - (s_ - bb)) + (part - bb)
            acc = s_
        else:
            acc += part
    rows = np.array([lidx[tuple(int(v) for v in t[:left])] for t in tuples], dtype=np.int64)
    cols = np.array([ridx[tuple(int(v) for v in t[left:])] for t in tuples], dtype=np.int64)
    return (acc[rows, cols], lo[rows, cols]) if compensated else acc[rows, cols]


def tuple_product_sums(fields_by_shell: dict, tuples) -> np.ndarray:
    """sum_x prod_j f_{t_j}[x] for each tuple, accumulated in extended precision."""
    out = np.empty(len(tuples), dtype=np.float64)
    for n, t in enumerate(tuples):
        prod = np.array(fields_by_shell[int(t[0])], dtype=np.float64, copy=True)
        for s in t[1:]:
            prod *= fields_by_shell[int(s)]
        out[n] = float(np.sum(prod, dtype=np.longdouble))
    return out


def counts_from_sums(C, N: int, tol: float = 1e-3) -> np.ndarray:
    """n_t = rint(C_t / N^3); the quotient q must be an integer to within max(tol, |q| 2^-46).

    C is an array of sums, or a (hi, lo) pair of arrays with C = hi + lo.  N^3 is a
    power of two for the grids used here, so the division is exact.  The relative
    part of the tolerance covers the FP64 rounding of the count fields, which for
    counts near 10^12 reaches 1e-3 of a unit; counts of 2^44 or more are refused.
    """
    if isinstance(C, tuple):
        hi, lo = (np.asarray(a, dtype=np.float64) for a in C)
    else:
        hi, lo = np.asarray(C, dtype=np.float64), np.zeros(np.shape(C))
    qh, ql = hi / float(N) ** 3, lo / float(N) ** 3
    n = np.rint(qh + ql)
    frac = (qh - n) + ql
    if np.any(np.abs(qh) >= 2.0 ** 44):
        raise ArithmeticError("polygon count of 2^44 or more: beyond exact FP64 recovery")
    lim = np.maximum(tol, np.ldexp(np.abs(qh), -46))
    if np.any(np.abs(frac) >= lim):
        raise ArithmeticError(f"polygon count not integral: worst {np.abs(frac).max():.3e}")
    return n.astype(np.int64)


def polygon_counts(N: int, order: int, n_shells: int, width: float, tuples) -> np.ndarray:
    """Number of closed ordered vector n-tuples per tuple (Appendix A, count on a unit grid)."""
    c = count_fields(N, n_shells, width)
    return counts_from_sums(product_sums(c, tuples, chunk=2048, compensated=True), N)


def pair_counts(c_i: np.ndarray, c_j: np.ndarray) -> np.ndarray:
    """P_ij(q) = #{(q_1, q_2) : q_1 in S_i, q_2 in S_j, q_1 + q_2 = q mod N} on the rfftn layout.

    c_i, c_j are the count fields of the two shells.  The DFT of c_i c_j is N^3 P_ij;
    every value is a small integer (at most min(|S_i|, |S_j|)), so rounding the
    FP64 transform recovers it exactly.
    """
    N = c_i.shape[0]
    P = rfftn(c_i * c_j)
    P /= float(N) ** 3
    R = np.rint(P.real)
    if np.abs(P.real - R).max() >= 1e-3 or np.abs(P.imag).max() >= 1e-3:
        raise ArithmeticError("pair count not integral")
    return R.astype(np.int64)


def triple_counts(c_i: np.ndarray, c_j: np.ndarray, c_k: np.ndarray) -> np.ndarray:
    """T_ijk(q) = #{(q_1, q_2, q_3) in S_i x S_j x S_k : q_1 + q_2 + q_3 = q mod N}, rfftn layout.

    As for pair_counts: the DFT of c_i c_j c_k is N^3 T_ijk, and every value is an
    integer no larger than |S_i| |S_j|, small enough for the FP64 transform to be
    rounded to it exactly.
    """
    N = c_i.shape[0]
    T = rfftn(c_i * c_j * c_k)
    T /= float(N) ** 3
    R = np.rint(T.real)
    if np.abs(T.real - R).max() >= 1e-3 or np.abs(T.imag).max() >= 1e-3:
        raise ArithmeticError("triple count not integral")
    return R.astype(np.int64)


def polygon_counts_exact(N: int, order: int, n_shells: int, width: float, tuples) -> np.ndarray:
    """The counts of polygon_counts, summed in integers from pair and triple counts.

    A closed ordered tuple q_1 + ... + q_n = 0 (mod N) splits into a left part
    with sum q and a right part with sum -q, so n_ijk = sum_{q in S_k} P_ij(q),
    n_ijkl = sum_q P_ij(q) P_kl(q), n_ijklm = sum_q P_ij(q) T_klm(q) and
    n_ijklmn = sum_q T_ijk(q) T_lmn(q) (the partial counts are even because every
    shell is); order 2 is P_ij(0).  Nothing large is ever rounded, so the result is
    exact for any count that fits in int64.
    """
    tuples = np.asarray(tuples, dtype=np.int64)
    order = tuples.shape[1]
    if order not in (2, 3, 4, 5, 6):
        raise ValueError("polygon_counts_exact supports orders 2 to 6")
    wz = np.full(N // 2 + 1, 2, dtype=np.int64)      # half-spectrum multiplicity of q_z
    wz[0] = 1
    wz[N // 2] = 1
    used = sorted({int(s) for s in tuples.ravel()})
    c = dict(zip(used, count_fields(N, n_shells, width, used)))
    sid = shell_id_grid(N, n_shells, width) if order == 3 else None
    cache = {}

    def part(shells):
        key = tuple(sorted(shells))
        if key not in cache:
            cache[key] = (pair_counts(c[key[0]], c[key[1]]) if len(key) == 2
                          else triple_counts(c[key[0]], c[key[1]], c[key[2]]))
        return cache[key]

    out = np.empty(len(tuples), dtype=np.int64)
    for n, t in enumerate(tuples.tolist()):
        if order == 2:
            out[n] = part(t)[0, 0, 0]
        elif order == 3:
            m = sid == t[2]
            out[n] = int(np.sum(part(t[:2])[m] * np.broadcast_to(wz, m.shape)[m]))
        else:
            split = 3 if order == 6 else 2
            out[n] = int(np.sum(part(t[:split]) * part(t[split:]) * wz))
    return out


def physical_factor(order: int, N: int, box_length: float) -> float:
    """V^{n-1} / N^{3n} with V = L^3 (Appendix A); 1 when no box length is given."""
    if not box_length:
        return 1.0
    V = float(box_length) ** 3
    return V ** (order - 1) / float(N) ** (3 * order)


def polyspectrum(delta: np.ndarray, order: int, n_shells: int, width: float,
                 box_length: float = 0.0, allow_aliasing: bool = False,
                 counts=None, return_fields: bool = False) -> dict:
    """The estimator for one real field delta[x] (float64 [N, N, N]).

    Returns the closing tuples, their counts n_t, the raw sums S_t and
    B_t = physical_factor * S_t / (N^3 n_t).
    """
    delta = np.asarray(delta, dtype=np.float64)
    return polyspectrum_from_hat(rfftn(delta), delta.shape[0], order, n_shells, width, box_length,
                                 allow_aliasing, counts, return_fields)


def polyspectrum_from_hat(delta_hat: np.ndarray, N: int, order: int, n_shells: int, width: float,
                          box_length: float = 0.0, allow_aliasing: bool = False,
                          counts=None, return_fields: bool = False) -> dict:
    """The estimator for a field given by its half spectrum delta_hat (rfftn layout [N, N, N//2+1]).

    Appendix A's input delta[q]; the shell fields are the inverse real transforms of the
    masked half spectrum, so in the q2 = 0 plane (where q and -q are both stored) the
    inverse transform keeps the real part of the result, as a real-to-complex pair does.
    """
    if 2 * outer_radius(n_shells, width) > N:
        raise ValueError("outer shell edge beyond the Nyquist wavenumber")
    alias_free = is_alias_free(N, order, n_shells, width)
    if not alias_free and not allow_aliasing:
        raise ValueError("configuration aliases: order * (N_b + 1/2) * width > N")
    cand = candidate_tuples(order, n_shells, alias_free)
    if counts is None:
        n_cand = polygon_counts(N, order, n_shells, width, cand)
    else:
        n_cand = np.asarray(counts, dtype=np.int64)
    keep = n_cand > 0
    tuples = cand[keep]
    n_t = n_cand[keep]
    d = shell_fields_from_hat(np.asarray(delta_hat, dtype=np.complex128), N, n_shells, width)
    S = product_sums(d, tuples)
    B = physical_factor(order, N, box_length) * S / (float(N) ** 3 * n_t)
    out = dict(tuples=tuples, counts=n_t, sums=S, B=B, candidates=cand, candidate_counts=n_cand)
    if return_fields:
        out["fields"] = d
    return out


# ----------------------------------------------------------------------------
# Gradient.  Not in the paper: the adjoint of the estimator, derived here.
# B_t = c_t S_t with c_t = phys / (N^3 n_t) and S_t = sum_x prod_j d_{t_j}[x].
# dS_t / d d_m[x] = sum over positions p with t_p = m of prod_{q != p} d_{t_q}[x].
# Each d_m = C2R(M_m R2C(delta)) with an even real kernel, so its adjoint is the
# same operator: dL/d delta = C2R( sum_m M_m R2C(a_m) ), a_m = dL/d d_m.
# ----------------------------------------------------------------------------
def adjoint_weights(tuples: np.ndarray, weights: np.ndarray, n_shells: int) -> np.ndarray:
    """W[m, rest] for order n: every position p of t adds w_t to W[t_p, t without p].

    `rest` runs over the sorted (n-1)-tuples (pairs for n = 3, triples for n = 4), so
    dS_t / d d_m = sum of the products of the other n - 1 fields over the positions of m.
    """
    tuples = np.asarray(tuples)
    order = tuples.shape[1]
    rests = sorted_tuples(order - 1, n_shells)
    ridx = {tuple(int(v) for v in r): n for n, r in enumerate(rests)}
    W = np.zeros((n_shells, len(rests)))
    for t, w in zip(tuples, np.asarray(weights, dtype=np.float64)):
        for p in range(order):
            rest = tuple(sorted(int(v) for q, v in enumerate(t) if q != p))
            W[int(t[p]) - 1, ridx[rest]] += w
    return W


def gradient_spectrum(N: int, order: int, n_shells: int, width: float, tuples, counts, fields,
                      grad_B, shells=None, box_length: float = 0.0, chunk: int = 8192) -> np.ndarray:
    """g[q] = sum_m [s(q) = m] R2C(a_m)[q] on the rfftn layout, a_m = dL/d d_m (orders 2, 3, 4).

    `fields` holds the shell fields of `shells` (all shells when None), in that order.
    Only those a_m are formed, from products of those fields; so dL/dB_t must vanish on
    every tuple that uses another shell (checked).
    """
    tuples = np.asarray(tuples, dtype=np.int64)
    shells = list(range(1, n_shells + 1)) if shells is None else [int(s) for s in shells]
    pos = {s: n for n, s in enumerate(shells)}
    w = np.asarray(grad_B, dtype=np.float64) * physical_factor(order, N, box_length) \
        / (float(N) ** 3 * np.asarray(counts, dtype=np.float64))
    inside = np.array([all(int(v) in pos for v in t) for t in tuples], dtype=bool)
    if np.any(w[~inside] != 0.0):
        raise ValueError("dL/dB is non-zero on a tuple with a shell whose field is not given")
    flat = np.asarray(fields, dtype=np.float64).reshape(len(shells), -1)
    a = np.zeros_like(flat)
    if order == 2:
        # S_(i,i) = sum d_i^2; only diagonal tuples close.
        for t, wt in zip(tuples[inside], w[inside]):
            i, j = pos[int(t[0])], pos[int(t[1])]
            a[i] += wt * flat[j]
            a[j] += wt * flat[i]
    elif order in (3, 4):
        # a_m = sum over rests r of W[m, r] prod_{s in r} d_s, over the given shells
        W = adjoint_weights(tuples[inside], w[inside], n_shells)
        rests = sorted_tuples(order - 1, n_shells)
        keep_r = np.array([all(int(v) in pos for v in r) for r in rests], dtype=bool)
        rest_pos = np.array([[pos[int(v)] for v in r] for r in rests[keep_r]], dtype=np.int64)
        Wk = W[np.array(shells) - 1][:, keep_r]
        for x0 in range(0, flat.shape[1], chunk):
            blk = flat[:, x0:x0 + chunk]
            prod = blk[rest_pos[:, 0]].copy()
            for c in range(1, order - 1):
                prod *= blk[rest_pos[:, c]]
            a[:, x0:x0 + chunk] = Wk @ prod
    else:
        raise ValueError("gradient supports orders 2, 3 and 4")
    sid = shell_id_grid(N, n_shells, width)
    g_hat = np.zeros((N, N, N // 2 + 1), dtype=np.complex128)
    for n, m in enumerate(shells):
        am_hat = rfftn(a[n].reshape(N, N, N))
        sel = sid == m
        g_hat[sel] += am_hat[sel]
    return g_hat


def gradient(delta: np.ndarray, order: int, n_shells: int, width: float, grad_B: np.ndarray,
             result: dict | None = None, box_length: float = 0.0,
             allow_aliasing: bool = False, chunk: int = 8192) -> np.ndarray:
    """dL/d delta[x] for L with dL/dB_t = grad_B[t] over the closing tuples (orders 2, 3, 4).

    Each d_m is C2R(M_m R2C(delta)) with an even real kernel, so the adjoint of
    delta -> d_m is the same operator and dL/d delta = C2R(g), g = gradient_spectrum.
    """
    delta = np.asarray(delta, dtype=np.float64)
    N = delta.shape[0]
    if result is None or "fields" not in result:
        result = polyspectrum(delta, order, n_shells, width, box_length, allow_aliasing,
                              return_fields=True)
    g_hat = gradient_spectrum(N, order, n_shells, width, result["tuples"], result["counts"],
                              result["fields"], grad_B, box_length=box_length, chunk=chunk)
    return irfftn(g_hat, s=(N, N, N)) * float(N) ** 3


def gradient_half_spectrum(N: int, order: int, n_shells: int, width: float, tuples, counts, fields,
                           grad_B, box_length: float = 0.0) -> np.ndarray:
    """dL/dRe delta_hat + i dL/dIm delta_hat for a half-spectrum input (rfftn layout).

    The inverse real transform reads an entry with q2 = 0 or q2 = N/2 once and any
    other entry twice (itself and, conjugated, its mirror -q), so the derivative of L
    with respect to the real and imaginary parts of that entry is 1 resp. 2 times g[q].
    """
    g_hat = gradient_spectrum(N, order, n_shells, width, tuples, counts, fields, grad_B,
                              box_length=box_length)
    wz = np.full(N // 2 + 1, 2.0)
    wz[0] = 1.0
    wz[N // 2] = 1.0
    return g_hat * wz


# ----------------------------------------------------------------------------
# Redshift-space multipoles.  Sec. 5 notes that the estimator extends to the angular
# multipoles by running it on multipole-weighted fields, after Scoccimarro (2015).
# Reading taken (the paper gives no formula): a fixed line of sight along the third
# grid axis (plane-parallel), the Legendre weight L_ell(mu) with mu = q_los/|q| on one
# leg, w, of each triangle, and
#   B_ell(u, v; w) = (2 ell + 1) phys sum_x d_u d_v d^ell_w / (N^3 n_t),
# d^ell_w the shell field of delta_hat L_ell, n_t the count of the triangle (u, v, w).
# Only even ell: L_ell(-mu) = L_ell(mu) keeps the weighted spectrum Hermitian, so the
# weighted fields are real.
# ----------------------------------------------------------------------------
def legendre(ell: int, mu: np.ndarray) -> np.ndarray:
    """The Legendre polynomial L_ell (numpy's Legendre series with one coefficient)."""
    coef = np.zeros(ell + 1)
    coef[ell] = 1.0
    return np.polynomial.legendre.legval(mu, coef)


def los_cosine_grid(N: int, axis: int = 2) -> np.ndarray:
    """mu = q_axis / |q| on the half-spectrum grid (rfftn layout); 0 at q = 0."""
    f = np.fft.fftfreq(N) * N
    h = np.fft.rfftfreq(N) * N
    q = np.meshgrid(f, f, h, indexing="ij")
    norm = np.sqrt(q[0] ** 2 + q[1] ** 2 + q[2] ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.where(norm > 0, q[axis] / norm, 0.0)
    return mu


def multipole_fields_from_hat(delta_hat: np.ndarray, N: int, n_shells: int, width: float, ell: int,
                              axis: int = 2) -> np.ndarray:
    """d^ell_s[x]: the shell fields of delta_hat[q] L_ell(mu_q) (even ell)."""
    if ell % 2:
        raise ValueError("odd multipoles give imaginary weighted fields; ell must be even")
    if axis == 2:
        weighted = delta_hat * legendre(ell, los_cosine_grid(N, 2))
        return shell_fields_from_hat(weighted, N, n_shells, width)
    # another line of sight: weight the full spectrum, keep its half (the weight is
    # even in q, so the weighted spectrum stays Hermitian)
    full = np.fft.fftn(np.fft.irfftn(delta_hat, s=(N, N, N), axes=(0, 1, 2)))
    f = np.fft.fftfreq(N) * N
    q = np.meshgrid(f, f, f, indexing="ij")
    norm = np.sqrt(q[0] ** 2 + q[1] ** 2 + q[2] ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.where(norm > 0, q[axis] / norm, 0.0)
    half = (full * legendre(ell, mu))[:, :, : N // 2 + 1]
    return shell_fields_from_hat(half, N, n_shells, width)


def multipole_tuples(tuples: np.ndarray, counts: np.ndarray):
    """(u, v, w) with u <= v and w the weighted leg, for every closing sorted triangle and
    every distinct choice of its weighted side, in lexicographic order; with their counts."""
    rows = {}
    for t, n in zip(np.asarray(tuples), np.asarray(counts)):
        a, b, c = (int(x) for x in t)
        for w, rest in ((a, (b, c)), (b, (a, c)), (c, (a, b))):
            rows[(rest[0], rest[1], w)] = int(n)
    keys = sorted(rows)
    return np.array(keys, dtype=np.int64).reshape(-1, 3), np.array([rows[k] for k in keys], dtype=np.int64)


def bispectrum_multipoles(delta: np.ndarray, n_shells: int, width: float, ell: int, axis: int = 2,
                          box_length: float = 0.0, counts=None) -> dict:
    """The multipole-ell bispectrum of a real field delta[x] (float64 [N, N, N]).

    Returns tuples (u, v, w) (1-based shells, w the weighted one), the triangle counts,
    the raw sums S = sum_x d_u d_v d^ell_w and B = (2 ell + 1) phys S / (N^3 n)."""
    delta = np.asarray(delta, dtype=np.float64)
    N = delta.shape[0]
    mono = polyspectrum(delta, 3, n_shells, width, counts=counts, return_fields=True)
    tup, n = multipole_tuples(mono["tuples"], mono["counts"])
    dl = multipole_fields_from_hat(rfftn(delta), N, n_shells, width, ell, axis)
    # the weighted fields follow the shells: (u, v, w) is the plain triple (u, v, n_shells + w)
    stacked = np.concatenate([mono["fields"], dl])
    S = product_sums(stacked, tup + np.array([0, 0, n_shells]))
    B = (2 * ell + 1) * physical_factor(3, N, box_length) * S / (float(N) ** 3 * n)
    return dict(tuples=tup, counts=n, sums=S, B=B)
