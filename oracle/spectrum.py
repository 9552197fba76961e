"""FP64 oracle of the Welch power spectral density and the adjacent-channel power
ratio of a PA output.

TEST INFRASTRUCTURE ONLY (imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the HIP path).

The paper names ACPR as the out-of-band metric it sets aside (Sec. I) but gives
no estimator.  The reading used here: Welch's method with nfft-point segments,
a periodic Hann window and 50 % overlap, two-sided, no detrending, scaled by
1/sum(w^2).  Main channel = PSD bins k with |k| <= h (h = half the occupied
band in PSD bins, DC included); the upper adjacent channel = bins h < k <= 3h,
the lower = -3h <= k < -h.  ACPR_{L,U} = 10 log10(P_adj / P_main).
"""
from __future__ import annotations

import numpy as np


def hann_periodic(n: int) -> np.ndarray:
    i = np.arange(n)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * i / n)


def welch_psd(y: np.ndarray, nfft: int = 4096) -> np.ndarray:
    """Two-sided PSD in natural FFT bin order (bin k at index k mod nfft)."""
    y = np.asarray(y, dtype=np.complex128)
    hop = nfft // 2
    nseg = (y.size - nfft) // hop + 1
    if nseg < 1:
        raise ValueError("signal shorter than one segment")
    w = hann_periodic(nfft)
    acc = np.zeros(nfft)
    for s in range(nseg):
        X = np.fft.fft(y[s * hop:s * hop + nfft] * w)
        acc += X.real ** 2 + X.imag ** 2
    return acc / nseg / np.sum(w * w)


def band_powers(psd: np.ndarray, half_bins: int):
    """(P_lower, P_main, P_upper) under the channel plan in the module docstring."""
    nfft = psd.size
    h = half_bins
    if 3 * h >= nfft // 2:
        raise ValueError("adjacent channels do not fit below Nyquist")
    k = np.arange(nfft)
    ks = np.where(k < nfft // 2, k, k - nfft)              # signed bin index
    main = psd[np.abs(ks) <= h].sum()
    upper = psd[(ks > h) & (ks <= 3 * h)].sum()
    lower = psd[(ks < -h) & (ks >= -3 * h)].sum()
    return float(lower), float(main), float(upper)


def acpr_db(psd: np.ndarray, half_bins: int):
    """(ACPR_L, ACPR_U, max) in dB."""
    lo, mn, up = band_powers(psd, half_bins)
    aL = 10.0 * np.log10(lo / mn)
    aU = 10.0 * np.log10(up / mn)
    return float(aL), float(aU), float(max(aL, aU))
