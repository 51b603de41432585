"""Seeded synthetic density fields on a periodic N^3 grid.

These generators supply *inputs* only; they contain none of the estimator's
arithmetic (no shell binning, no products of shell fields, no normalisation by
polygon counts).  Both the HIP library's tests/benchmark and the CPU oracle's
tests draw their fields from here, so the two sides see identical numbers.

Recipe (the paper gives only the field type, so the amplitude and the RNG are
fixed here):

* Gaussian field with power spectrum P(k):
    1. w[x] ~ N(0, 1) i.i.d. on N^3 from ``numpy.random.default_rng(seed)`` (PCG64);
    2. w_hat = rfftn(w);  g_hat = w_hat * sqrt(P(|q|)) with |q| in units of the
       fundamental wavenumber k_f and P(0) = 0;
    3. g = irfftn(g_hat), rescaled to unit sample standard deviation (ddof 0).
* Lognormal field: delta = exp(g - s2/2) - 1 with s2 the sample variance of g
  (equal to 1 after step 3), built on the Gaussian g with
  P_g(k) = k^-1.5 exp(-(k / (N/4))^2)  (N/4 k_f is half the Nyquist wavenumber).

All arrays are float64; callers that feed a float32 kernel cast with
``astype(np.float32)`` and hand the oracle the same float32 values promoted back
to float64.
"""
from __future__ import annotations

import os

import numpy as np

try:  # scipy's pocketfft runs multi-threaded; numpy's is the fallback
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=_workers())

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=_workers())
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def _workers() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def _wavenumber_magnitude(N: int) -> np.ndarray:
    """|q| in units of k_f on the rfftn half-spectrum layout [N, N, N//2+1]."""
    k = np.fft.fftfreq(N, d=1.0 / N)
    kz = np.arange(N // 2 + 1, dtype=np.float64)
    return np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2)


def power_law(alpha: float):
    """P(k) = k^alpha (alpha < 0 for the red spectra used here)."""
    def P(k):
        out = np.zeros_like(k)
        nz = k > 0
        out[nz] = k[nz] ** alpha
        return out
    return P


def lognormal_seed_spectrum(N: int):
    """P_g(k) = k^-1.5 exp(-(k/(N/4))^2)."""
    def P(k):
        out = np.zeros_like(k)
        nz = k > 0
        out[nz] = k[nz] ** -1.5 * np.exp(-(k[nz] / (N / 4.0)) ** 2)
        return out
    return P


def gaussian_field(N: int, seed: int, spectrum=None) -> np.ndarray:
    """Unit-variance Gaussian random field with the given P(k) (default k^-2)."""
    if spectrum is None:
        spectrum = power_law(-2.0)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N, N))
    w_hat = _rfftn(w)
    del w
    w_hat *= np.sqrt(spectrum(_wavenumber_magnitude(N)))
    g = _irfftn(w_hat, s=(N, N, N))
    del w_hat
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_field(N: int, seed: int) -> np.ndarray:
    """delta = exp(g - sigma^2/2) - 1 on the Gaussian g with P_g above."""
    g = gaussian_field(N, seed, lognormal_seed_spectrum(N))
    s2 = g.var()
    np.subtract(g, 0.5 * s2, out=g)
    np.exp(g, out=g)
    g -= 1.0
    return g


def unit_spectrum_field(N: int) -> np.ndarray:
    """delta[x] = 1 at x = 0 and 0 elsewhere, whose unnormalised DFT is 1 at every mode."""
    d = np.zeros((N, N, N))
    d[0, 0, 0] = 1.0
    return d


# The workloads the library is measured and tested on.  Each entry fixes the
# grid, the field recipe and its seed; the estimator parameters live beside it.
WORKLOADS = {
    "bispec_64": dict(N=64, order=3, n_shells=16, width=1.0, batch=1,
                      field="gaussian", seeds=[1]),
    "bispec_256_lognormal": dict(N=256, order=3, n_shells=40, width=2.0, batch=1,
                                 field="lognormal", seeds=[2]),
    "trispec_256_lognormal": dict(N=256, order=4, n_shells=24, width=2.0, batch=1,
                                  field="lognormal", seeds=[2]),
    # the trispectrum with more than 32 shells (alias-free: 4 x 40.5 <= 256), whose adjoint
    # takes four 16-shell chunks of u and two 32-row blocks of m
    "trispec_256_40": dict(N=256, order=4, n_shells=40, width=1.0, batch=1,
                           field="lognormal", seeds=[2]),
    "bispec_grad_128x8": dict(N=128, order=3, n_shells=24, width=1.0, batch=8,
                              field="gaussian", seeds=list(range(40, 48)), target_seed=48),
    "bispec_512_lognormal": dict(N=512, order=3, n_shells=64, width=1.0, batch=1,
                                 field="lognormal", seeds=[5]),
    # orders 5 and 6 (Sec. 4.2): as many unit-width shells as keep every polygon
    # count below 2^44, the limit of exact recovery from float64 count sums
    "quadspec_256_lognormal": dict(N=256, order=5, n_shells=16, width=1.0, batch=1,
                                   field="lognormal", seeds=[2]),
    "pentaspec_256_lognormal": dict(N=256, order=6, n_shells=8, width=1.0, batch=1,
                                    field="lognormal", seeds=[2]),
    # streamed mode: a 1024^3 input, the band-limited interpolation of the 512^3 field
    # above (the inverse transform of zero_padded_half_spectrum)
    "bispec_1024_streamed": dict(N=1024, order=3, n_shells=64, width=1.0, batch=1,
                                 field="lognormal", seeds=[5], spectrum_of="bispec_512_lognormal",
                                 stream=True),
    # 128 unit shells on the same 1024^3 input (alias-free: 3 x 128.5 <= 1024); the
    # contraction stages eight 16-shell blocks; forward only (the adjoint holds 64 shells)
    "bispec_1024_streamed_128": dict(N=1024, order=3, n_shells=128, width=1.0, batch=1,
                                     field="lognormal", seeds=[5], spectrum_of="bispec_512_lognormal",
                                     stream=True),
}


def zero_padded_half_spectrum(field: np.ndarray, N_out: int, K: int) -> np.ndarray:
    """Half spectrum (complex64 [N_out, N_out, N_out/2 + 1]) of the band-limited interpolation
    of a real N^3 field onto N_out^3, kept on the modes whose components are all at most K
    in magnitude (K < N/2) and zero elsewhere.

    The unnormalised DFT of the interpolated field is (N_out/N)^3 times that of the field
    on every mode both grids hold.
    """
    N = field.shape[0]
    hs = np.fft.rfftn(np.asarray(field, dtype=np.float64)) * (N_out / N) ** 3
    out = np.zeros((N_out, N_out, N_out // 2 + 1), dtype=np.complex64)
    for src0, dst0 in ((slice(0, K + 1), slice(0, K + 1)), (slice(N - K, N), slice(N_out - K, N_out))):
        for src1, dst1 in ((slice(0, K + 1), slice(0, K + 1)), (slice(N - K, N), slice(N_out - K, N_out))):
            out[dst0, dst1, :K + 1] = hs[src0, src1, :K + 1]
    return out


def make_field(kind: str, N: int, seed: int) -> np.ndarray:
    if kind == "gaussian":
        return gaussian_field(N, seed)
    if kind == "lognormal":
        return lognormal_field(N, seed)
    raise ValueError(f"unknown field kind {kind!r}")


def workload_fields(name: str, dtype=np.float32) -> np.ndarray:
    """[batch, N, N, N] array of the workload's fields in the requested dtype."""
    w = WORKLOADS[name]
    out = np.empty((len(w["seeds"]), w["N"], w["N"], w["N"]), dtype=dtype)
    for b, seed in enumerate(w["seeds"]):
        out[b] = make_field(w["field"], w["N"], seed)
    return out
