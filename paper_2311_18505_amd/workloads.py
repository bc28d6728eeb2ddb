"""Seeded synthetic workloads (parameter draws only; no arithmetic of the method).

Every input of the tests, the benchmark and the serving loop comes from here,
and the same dictionaries feed both the GPU library and the CPU oracle.  The
paper publishes no parameter distributions (Sec. 1 names "stochastic
parameterization" only), so the distributions below are this project's
synthetic stand-ins, with the paper's own worked parameters (Sec. 4.2) where
it gives them.

String dictionary keys: fs, f0, B, alpha, theta, sigma0_t, sigma1_t, sigma0_l,
sigma1_l, x_out, n_samples, mod_type (0 none, 1 vibrato, 2 glide),
mod_depth_cents, mod_rate_hz, glide_semitones, grid_t, grid_l, grid_interp
(order of the grid interpolant: 0 or 1 linear, 3 cubic).
Excitation keys: type (0 none, 1 pluck, 2 hammer), x, c0, v_H, M_H, K_H,
alpha_H, rhoA.
"""
from __future__ import annotations

import numpy as np

SEED = 231118505
FS = 48000.0
X_OUT = 0.8

# hammer constants of the single nonlinear string workload (felt force
# K max(0, compression)^alpha_H, 8 g, 4 m/s); rho A is not given anywhere and
# is taken as 0.05 kg/m for a string of length 1 m.
HAMMER = dict(M_H=0.008, K_H=1e8, alpha_H=2.5, rhoA=0.05)


def string(f0, B, alpha, sigma0, sigma1, n_samples, theta=0.0, fs=FS, x_out=X_OUT,
           mod_type=0, mod_depth_cents=0.0, mod_rate_hz=0.0, glide_semitones=0.0,
           grid_t=0, grid_l=0, sigma0_l=None, sigma1_l=None, grid_interp=0) -> dict:
    return dict(fs=float(fs), f0=float(f0), B=float(B), alpha=float(alpha), theta=float(theta),
                grid_interp=int(grid_interp),
                sigma0_t=float(sigma0), sigma1_t=float(sigma1),
                sigma0_l=float(sigma0 if sigma0_l is None else sigma0_l),
                sigma1_l=float(sigma1 if sigma1_l is None else sigma1_l),
                x_out=float(x_out), n_samples=int(n_samples), mod_type=int(mod_type),
                mod_depth_cents=float(mod_depth_cents), mod_rate_hz=float(mod_rate_hz),
                glide_semitones=float(glide_semitones), grid_t=int(grid_t), grid_l=int(grid_l))


def pluck(x, c0) -> dict:
    return dict(type=1, x=float(x), c0=float(c0), v_H=0.0, M_H=0.0, K_H=0.0, alpha_H=0.0, rhoA=0.0)


def hammer(x, v_H, M_H=HAMMER["M_H"], K_H=HAMMER["K_H"], alpha_H=HAMMER["alpha_H"], rhoA=HAMMER["rhoA"]) -> dict:
    return dict(type=2, x=float(x), c0=0.0, v_H=float(v_H), M_H=float(M_H), K_H=float(K_H),
                alpha_H=float(alpha_H), rhoA=float(rhoA))


def bow(x, v_B, F_B, x_end=None, attack=0.02, fric_a=100.0, fric_eps=0.2) -> dict:
    """Bow (eq. 5) at x (moving linearly to x_end over the note), bow speed v_B
    [m/s] and force F_B, both rising over `attack` seconds; friction curve
    parameters a and eps."""
    return dict(type=3, x=float(x), c0=0.0, x_end=float(x if x_end is None else x_end), v_B=float(v_B),
                F_B=float(F_B), attack=float(attack), fric_a=float(fric_a), fric_eps=float(fric_eps))


def single_bowed(seconds: float = 0.5):
    """A linear string of 110 Hz bowed at 0.12 (stick-slip locked to f0)."""
    p = string(110.0, 1e-4, 1.0, 0.5, 1e-4, int(round(seconds * FS)))
    return p, bow(0.12, 0.1, 100.0)


def bowed_batch(n: int, seed: int = SEED + 11, seconds: float = 0.25):
    """Bowed strings with seed-drawn parameters: string draws as in
    random_batch (f0 log-U(40, 1000), alpha U(1, 4), ...), bow at U(0.05, 0.3)
    moving by U(-0.05, 0.05) over the note (a third stay in place), v_B
    U(0.05, 0.2) m/s, F_B log-U(20, 300), attack U(0.005, 0.05) s, friction
    a U(20, 200) s/m and eps U(0.1, 0.5)."""
    rng = np.random.default_rng(seed)
    f0 = _loguniform(rng, 40.0, 1000.0, n)
    B = _loguniform(rng, 1e-5, 1e-2, n)
    sigma0 = rng.uniform(0.5, 3.0, n)
    sigma1 = _loguniform(rng, 1e-5, 1e-3, n)
    alpha = rng.uniform(1.0, 4.0, n)
    pos = rng.uniform(0.05, 0.3, n)
    move = np.where(rng.uniform(0.0, 1.0, n) < 1.0 / 3.0, 0.0, rng.uniform(-0.05, 0.05, n))
    vB = rng.uniform(0.05, 0.2, n)
    FB = _loguniform(rng, 20.0, 300.0, n)
    att = rng.uniform(0.005, 0.05, n)
    fa = rng.uniform(20.0, 200.0, n)
    fe = rng.uniform(0.1, 0.5, n)
    ns = int(round(seconds * FS))
    return [(string(f0[i], B[i], alpha[i], sigma0[i], sigma1[i], ns),
             bow(pos[i], vB[i], FB[i], x_end=pos[i] + move[i], attack=att[i], fric_a=fa[i], fric_eps=fe[i]))
            for i in range(n)]


def single_linear(seconds: float = 1.0, theta: float = 0.0):
    """Single linear stiff string: fs 48 kHz, f0 110 Hz, B 1e-4, sigma0 1, sigma1 5e-4,
    pluck at 0.2 with peak 1e-3, readout at 0.8, fixed ends, alpha = 1."""
    return (string(110.0, 1e-4, 1.0, 1.0, 5e-4, int(round(seconds * FS)), theta=theta),
            pluck(0.2, 1e-3))


def single_nonlinear(seconds: float = 2.0, theta: float = 0.0):
    """Single nonlinear planar string: f0 82.4 Hz, B 2e-4, sigma0 0.8, sigma1 3e-4,
    alpha 3 (the value of the paper's Sec. 4.2 example), hammer at 0.12 L
    (alpha_H 2.5, K_H 1e8, 8 g, 4 m/s)."""
    return (string(82.4, 2e-4, 3.0, 0.8, 3e-4, int(round(seconds * FS)), theta=theta),
            hammer(0.12, 4.0))


def _loguniform(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def random_batch(n: int, seed: int = SEED, seconds=2.0, durations=None, modulation: bool = False,
                 theta: float = 0.0):
    """Batch of nonlinear strings with seed-drawn parameters.

    f0 log-uniform 40-1000 Hz, B log-uniform 1e-5..1e-2, sigma0 U(0.5, 3),
    sigma1 log-uniform 1e-5..1e-3, alpha U(1, 4), pluck/hammer 50/50 at a
    position U(0.05, 0.3), amplitude a U(1e-4, 3e-3): pluck peak c0 = a, hammer
    velocity 2000 a m/s (a = 2e-3 gives the 4 m/s of the single string).
    durations: None -> `seconds` for all; ("uniform", lo, hi) -> U(lo, hi) s.
    modulation: 50/50 vibrato (depth U(0, 50) cents, rate U(4, 7) Hz) or a
    linear glide of U(-2, 2) semitones over the duration.
    """
    rng = np.random.default_rng(seed)
    f0 = _loguniform(rng, 40.0, 1000.0, n)
    B = _loguniform(rng, 1e-5, 1e-2, n)
    sigma0 = rng.uniform(0.5, 3.0, n)
    sigma1 = _loguniform(rng, 1e-5, 1e-3, n)
    alpha = rng.uniform(1.0, 4.0, n)
    is_hammer = rng.uniform(0.0, 1.0, n) < 0.5
    pos = rng.uniform(0.05, 0.3, n)
    amp = rng.uniform(1e-4, 3e-3, n)
    if durations is None:
        dur = np.full(n, float(seconds))
    else:
        _, lo, hi = durations
        dur = rng.uniform(lo, hi, n)
    if modulation:
        is_vib = rng.uniform(0.0, 1.0, n) < 0.5
        depth = rng.uniform(0.0, 50.0, n)
        rate = rng.uniform(4.0, 7.0, n)
        glide = rng.uniform(-2.0, 2.0, n)
    items = []
    for i in range(n):
        kw = {}
        if modulation:
            if is_vib[i]:
                kw = dict(mod_type=1, mod_depth_cents=depth[i], mod_rate_hz=rate[i])
            else:
                kw = dict(mod_type=2, glide_semitones=glide[i])
        s = string(f0[i], B[i], alpha[i], sigma0[i], sigma1[i], int(round(dur[i] * FS)), theta=theta, **kw)
        e = hammer(pos[i], 2000.0 * amp[i]) if is_hammer[i] else pluck(pos[i], amp[i])
        items.append((s, e))
    return items


def uniform_batch_4096(seconds: float = 2.0):
    """4096 nonlinear strings, 2 s each (the oracle checks strings 0..63)."""
    return random_batch(4096, seconds=seconds)


def uneven_batch_16384():
    """16384 nonlinear strings, durations U(0.5, 4) s, vibrato or glide."""
    return random_batch(16384, durations=("uniform", 0.5, 4.0), modulation=True)


def serving_requests(rate_hz: float = 2000.0, seconds: float = 60.0, seed: int = SEED + 5):
    """Poisson arrivals; each request one string with the batch draws and a
    duration U(0.25, 3) s.  Returns (arrival_times, items)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, int(rate_hz * seconds * 1.5) + 100)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    items = random_batch(len(t), seed=seed + 1, durations=("uniform", 0.25, 3.0))
    return t, items
