"""Spectral analysis of synthesised notes: fundamental, inharmonicity and
phantom partials (the paper's qualitative plots of Sec. 4, without CREPE).

A stiff string's transverse partials lie at f_n = n f0 sqrt(1 + B n^2)
(Sec. 4.1); the nonlinear coupling with the longitudinal motion adds
"phantom" partials near sums f_i + f_j of transverse ones.  The analysis:

1. magnitude spectrum with a 4-term Blackman-Harris window (sidelobes below
   -92 dB, so weak phantoms are not confused with leakage), zero padded;
   spectral peaks above a floor relative to the largest, refined by a
   parabola through the log magnitudes;
2. f0: harmonic-sum search over a grid of candidates, then a least-squares
   fit of (f_n / n)^2 = f0^2 + f0^2 B n^2 over the peaks matched to n = 1..N;
3. phantoms: peaks that match no transverse partial but lie near a sum
   f_i + f_j.

Plain numpy on the host (post-processing of output samples).
"""
from __future__ import annotations

import numpy as np


def _window(n: int) -> np.ndarray:
    a0, a1, a2, a3 = 0.35875, 0.48829, 0.14128, 0.01168
    x = 2.0 * np.pi * np.arange(n) / (n - 1)
    return a0 - a1 * np.cos(x) + a2 * np.cos(2 * x) - a3 * np.cos(3 * x)


def spectrum(y, fs: float, pad: int = 4):
    """(frequencies, magnitude in dB) of the windowed, zero-padded signal."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    Y = np.abs(np.fft.rfft((y - y.mean()) * _window(n), pad * n))
    f = np.arange(len(Y)) * fs / (pad * n)
    return f, 20.0 * np.log10(Y + 1e-300)


def find_peaks(y, fs: float, floor_db: float = -70.0, pad: int = 4, f_min: float = 20.0):
    """Local maxima of the spectrum within floor_db of the largest: arrays
    (frequency, level in dB), the frequency refined by a parabola."""
    f, m = spectrum(y, fs, pad)
    top = m[f >= f_min].max()
    i = np.nonzero((m[1:-1] > m[:-2]) & (m[1:-1] >= m[2:]) & (m[1:-1] > top + floor_db) & (f[1:-1] >= f_min))[0] + 1
    a, b, c = m[i - 1], m[i], m[i + 1]
    den = a - 2 * b + c
    d = np.where(den != 0, 0.5 * (a - c) / np.where(den != 0, den, 1), 0.0)
    df = f[1] - f[0]
    return f[i] + d * df, b - 0.25 * (a - c) * d


def _cents(a, b):
    return 1200.0 * np.log2(np.asarray(a, dtype=np.float64) / b)


def fit_inharmonic(freqs, levels, f0_guess: float, n_max: int = 12, tol_cents: float = 50.0):
    """Match peaks to n = 1..n_max around n f0 sqrt(1 + B n^2) and fit f0, B;
    returns (f0, B, matched) with matched {n: frequency}.  The match grows
    from the lowest partials (n <= 3 within tol_cents of n f0) to n_max (within
    tol_cents / 2 of the current fit's prediction), taking the strongest peak
    in reach, and the fit is redone at every stage."""
    freqs = np.asarray(freqs, dtype=np.float64)
    levels = np.asarray(levels, dtype=np.float64)
    f0, B = float(f0_guess), 0.0
    matched = {}
    for stage, top in enumerate(sorted({3, 5, 8, n_max})):
        if top > n_max:
            break
        tol = tol_cents if stage == 0 else 0.5 * tol_cents
        cand = {}
        for n in range(1, top + 1):
            target = n * f0 * np.sqrt(1.0 + B * n * n)
            near = np.nonzero(np.abs(_cents(freqs, target)) <= tol)[0] if len(freqs) else []
            if len(near):
                cand[n] = float(freqs[near[int(np.argmax(levels[near]))]])
        if len(cand) < 2:
            break
        ns = np.array(sorted(cand), dtype=np.float64)
        yv = (np.array([cand[int(n)] for n in ns]) / ns) ** 2
        A = np.stack([np.ones_like(ns), ns * ns], axis=1)
        (c0, c1), *_ = np.linalg.lstsq(A, yv, rcond=None)
        if c0 <= 0:
            break
        f0, B, matched = float(np.sqrt(c0)), float(max(c1 / c0, 0.0)), cand
    return f0, B, matched


def f0_estimate(y, fs: float, f_lo: float = 20.0, f_hi: float = 2000.0, harmonics: int = 8):
    """Fundamental and inharmonicity: harmonic-sum search, then the fit."""
    f, m = spectrum(y, fs)
    lin = 10.0 ** (m / 20.0)
    cands = np.exp(np.linspace(np.log(f_lo), np.log(f_hi), 4000))
    df = f[1] - f[0]
    score = np.zeros_like(cands)
    for k in range(1, harmonics + 1):
        idx = np.clip(np.round(k * cands / df).astype(int), 0, len(lin) - 1)
        # the largest bin within +-1 % of k f (inharmonicity moves upper partials)
        w = np.maximum(1, np.round(0.01 * k * cands / df).astype(int))
        best = np.array([lin[max(i - ww, 0):i + ww + 1].max() for i, ww in zip(idx, w)])
        score += best / k
    g = float(cands[int(np.argmax(score))])
    peaks, levels = find_peaks(y, fs)
    return fit_inharmonic(peaks, levels, g)


def phantom_partials(y, fs: float, f0: float, B: float, n_max: int = 12, tol_cents: float = 15.0,
                     floor_db: float = -70.0):
    """Peaks that match no transverse partial n f0 sqrt(1 + B n^2) (n <= 2 n_max)
    but lie within tol_cents of a sum f_i + f_j (1 <= i <= j <= n_max):
    [(frequency, level dB, (i, j))]."""
    freqs, levels = find_peaks(y, fs, floor_db=floor_db)
    ns = np.arange(1, 2 * n_max + 1)
    fn = ns * f0 * np.sqrt(1.0 + B * ns * ns)
    out = []
    for fr, lv in zip(freqs, levels):
        if np.min(np.abs(_cents(fn, fr))) <= tol_cents:
            continue
        best = None
        for i in range(1, n_max + 1):
            for j in range(i, n_max + 1):
                c = abs(float(_cents(fn[i - 1] + fn[j - 1], fr)))
                if c <= tol_cents and (best is None or c < best[0]):
                    best = (c, (i, j))
        if best is not None:
            out.append((float(fr), float(lv), best[1]))
    return out


def analyze(y, fs: float, n_max: int = 12) -> dict:
    f0, B, matched = f0_estimate(y, fs)
    return {"f0": f0, "B": B, "partials": matched, "phantoms": phantom_partials(y, fs, f0, B, n_max)}


def main(argv=None) -> None:
    """Analyse rows of .npy files (one note per row, as the dataset generator
    writes them) and print one JSON line per note: f0, B, the matched
    partials and the phantom partials."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description="f0, inharmonicity and phantom partials of synthesised notes")
    ap.add_argument("files", nargs="+", help=".npy arrays, one note per row (or one 1-D note)")
    ap.add_argument("--fs", type=float, default=48000.0)
    ap.add_argument("--n-max", type=int, default=12)
    ap.add_argument("--labels", help="labels.json of the dataset generator: trims each row to its length")
    args = ap.parse_args(argv)
    lengths = None
    if args.labels:
        with open(args.labels) as f:
            lengths = [int(x["samples"]) for x in json.load(f)]
    k = 0
    for path in args.files:
        rows = np.atleast_2d(np.load(path))
        for row in rows:
            y = row[:lengths[k]] if lengths is not None else row
            r = analyze(np.asarray(y, np.float64), args.fs, args.n_max)
            print(json.dumps({"file": path, "row": k, "f0": r["f0"], "B": r["B"],
                              "partials": {str(n): f for n, f in sorted(r["partials"].items())},
                              "phantoms": [[f, lv, list(ij)] for f, lv, ij in r["phantoms"]]}), flush=True)
            k += 1


if __name__ == "__main__":
    main()
