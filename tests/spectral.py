"""Partial-frequency estimator used by the tests (same estimator on every output
that is compared, so its bias cancels in GPU-vs-oracle comparisons).

1. Hann window, zero padding x8, FFT; pick the log-magnitude peak near each
   guess and refine it by quadratic interpolation.
2. Refine all partials jointly by a damped-sinusoid least-squares fit
   (variable projection: frequencies and decay rates are the nonlinear
   parameters, amplitudes and phases are solved linearly).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import least_squares


def fft_peaks(y, fs, guesses, pad=8, search_cents=60.0):
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    Y = np.fft.rfft(y * np.hanning(n), n * pad)
    mag = np.log(np.abs(Y) + 1e-300)
    df = fs / (n * pad)
    out = []
    for f in guesses:
        lo = int(np.floor(f * 2 ** (-search_cents / 1200) / df))
        hi = int(np.ceil(f * 2 ** (search_cents / 1200) / df)) + 1
        lo = max(lo, 1)
        hi = min(hi, len(mag) - 1)
        i = lo + int(np.argmax(mag[lo:hi]))
        a, b, c = mag[i - 1], mag[i], mag[i + 1]
        den = a - 2 * b + c
        d = 0.5 * (a - c) / den if den != 0 else 0.0
        out.append((i + d) * df)
    return np.array(out)


def _basis(t, f, d):
    cols = []
    for fk, dk in zip(f, d):
        env = np.exp(-dk * t)
        cols.append(env * np.cos(2 * np.pi * fk * t))
        cols.append(env * np.sin(2 * np.pi * fk * t))
    return np.stack(cols, axis=1)


def fit_partials(y, fs, guesses, decay_guess=1.0, max_samples=None):
    """Return (freqs, decays, amplitudes) of damped sinusoids near `guesses`."""
    y = np.asarray(y, dtype=np.float64)
    if max_samples:
        y = y[:max_samples]
    t = np.arange(len(y)) / fs
    f0 = fft_peaks(y, fs, guesses)
    K = len(f0)
    x0 = np.concatenate([f0, np.full(K, float(decay_guess))])
    scale = np.max(np.abs(y)) or 1.0
    yn = y / scale

    def resid(x):
        Bm = _basis(t, x[:K], x[K:])
        coef, *_ = np.linalg.lstsq(Bm, yn, rcond=None)
        return Bm @ coef - yn

    sol = least_squares(resid, x0, x_scale=np.concatenate([np.full(K, 0.01), np.full(K, 0.1)]),
                        xtol=1e-14, ftol=1e-14, gtol=1e-14, max_nfev=200)
    f, d = sol.x[:K], sol.x[K:]
    Bm = _basis(t, f, d)
    coef, *_ = np.linalg.lstsq(Bm, yn, rcond=None)
    amp = np.hypot(coef[0::2], coef[1::2]) * scale
    return f, d, amp


def cents(f, fref):
    return 1200.0 * np.log2(np.asarray(f) / np.asarray(fref))
