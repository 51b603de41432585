"""Direct n-gon enumeration: the estimator as it is defined, before the FFT trick.

TEST INFRASTRUCTURE ONLY.  Sec. 2 (label eq:estimateBk and its n-point
extension eq:estimator) defines the angle-averaged polyspectrum as the average
of delta(q_1) ... delta(q_n) over all vector tuples with q_j in shell t_j that
close (q_1 + ... + q_n = 0), normalised by the number of such tuples.  On the
periodic grid closure is taken modulo N.  This module enumerates those tuples
explicitly; it is slow and meant for tiny grids (16^3, 32^3).
"""
from __future__ import annotations

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
                            tuples) -> tuple[np.ndarray, np.ndarray]:
    """(count, sum of prod delta_hat) for each tuple, by explicit enumeration.

    delta_hat is the unnormalised forward DFT of the real field; the returned sums
    are complex (their imaginary parts vanish up to rounding because the set of
    closed tuples is symmetric under q -> -q).
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
        first = [vecs[int(s) - 1] for s in t[:-1]]
        last = int(t[-1])
        if order == 2:
            q_last = _wrap(-first[0], N)
            ok = shell_of_squared_norm((q_last ** 2).sum(-1), n_shells, width) == last
            counts[n] = ok.sum()
            sums[n] = (value(first[0]) * value(q_last))[ok].sum()
        elif order == 3:
            a, b = first
            tot = a[:, None, :] + b[None, :, :]
            q_last = _wrap(-tot, N)
            ok = shell_of_squared_norm((q_last ** 2).sum(-1), n_shells, width) == last
            prod = value(a)[:, None] * value(b)[None, :] * value(q_last)
            counts[n] = ok.sum()
            sums[n] = prod[ok].sum()
        elif order == 4:
            a, b, c = first
            va, vb, vc = value(a), value(b), value(c)
            cnt = 0
            acc = 0j
            for ia in range(len(a)):
                tot = a[ia][None, None, :] + b[:, None, :] + c[None, :, :]
                q_last = _wrap(-tot, N)
                ok = shell_of_squared_norm((q_last ** 2).sum(-1), n_shells, width) == last
                prod = va[ia] * vb[:, None] * vc[None, :] * value(q_last)
                cnt += int(ok.sum())
                acc += prod[ok].sum()
            counts[n] = cnt
            sums[n] = acc
        else:
            raise ValueError("bruteforce supports orders 2, 3 and 4")
    return counts, sums
