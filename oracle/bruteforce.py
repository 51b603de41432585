"""Direct n-gon enumeration: the estimator as it is defined, before the FFT trick.

TEST INFRASTRUCTURE ONLY.  Sec. 2 (label eq:estimateBk and its n-point
extension eq:estimator) defines the angle-averaged polyspectrum as the average
of delta(q_1) ... delta(q_n) over all vector tuples with q_j in shell t_j that
close (q_1 + ... + q_n = 0), normalised by the number of such tuples.  On the
periodic grid closure is taken modulo N.  This module enumerates those tuples
explicitly; it is slow and meant for tiny grids (16^3, 32^3).
"""
from __future__ import annotations

import itertools

import numpy as np

from .polyspec import shell_of_squared_norm


def _wrap(v: np.ndarray, N: int) -> np.ndarray:
    """Representative of each component in [-N/2, N/2)."""
    return (v + N // 2) % N - N // 2


def shell_vectors(N: int, n_shells: int, width: float):
    """For each shell s = 1..N_b: the integer wave vectors (wrapped) that it holds."""
    k = np.arange(N)
    k = _wrap(k, N)
    g = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1).reshape(-1, 3)
    sid = shell_of_squared_norm((g ** 2).sum(axis=1), n_shells, width)
    return [g[sid == s] for s in range(1, n_shells + 1)]


def bruteforce_polyspectrum(delta: np.ndarray, order: int, n_shells: int, width: float,
                            tuples, last_weight=None) -> tuple[np.ndarray, np.ndarray]:
    """(count, sum of prod delta_hat) for each tuple, by explicit enumeration.

    delta_hat is the unnormalised forward DFT of the real field; the returned sums
    are complex (their imaginary parts vanish up to rounding because the set of
    closed tuples is symmetric under q -> -q).  last_weight(q) (an array of wave
    vectors -> weights) multiplies each product by a weight of the last vector.
    """
    delta = np.asarray(delta, dtype=np.float64)
    N = delta.shape[0]
    dhat = np.fft.fftn(delta)
    vecs = shell_vectors(N, n_shells, width)

    def value(v):
        w = v % N
        return dhat[w[..., 0], w[..., 1], w[..., 2]]

    counts = np.zeros(len(tuples), dtype=np.int64)
    sums = np.zeros(len(tuples), dtype=np.complex128)
    for n, t in enumerate(np.asarray(tuples)):
        if len(t) != order or order < 2:
            raise ValueError("tuples must have `order` entries, order >= 2")
        first = [vecs[int(s) - 1] for s in t[:-1]]
        last = int(t[-1])
        # the last two free vectors are enumerated as a grid, any earlier ones one
        # combination at a time; q_n closes the polygon
        head, (a, b) = first[:-2], ([np.zeros((1, 3), dtype=np.int64)] + first)[-2:]
        cnt = 0
        acc = 0j
        for combo in itertools.product(*[range(len(h)) for h in head]):
            base = np.zeros(3, dtype=np.int64)
            w = 1.0 + 0j
            for h, i in zip(head, combo):
                base = base + h[i]
                w *= value(h[i])
            tot = base[None, None, :] + a[:, None, :] + b[None, :, :]
            q_last = _wrap(-tot, N)
            ok = shell_of_squared_norm((q_last ** 2).sum(-1), n_shells, width) == last
            va = value(a) if order > 2 else np.ones(1)
            prod = w * va[:, None] * value(b)[None, :] * value(q_last)
            if last_weight is not None:
                prod = prod * last_weight(q_last)
            cnt += int(ok.sum())
            acc += prod[ok].sum()
        counts[n] = cnt
        sums[n] = acc
    return counts, sums
