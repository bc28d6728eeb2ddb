"""Independent dense numpy construction of the scheme (test helper for the
brute-force pin of the oracle on tiny grids, and for the energy pins).

Built from the paper's operator definitions with numpy/scipy routines of its
own (np.interp for every interpolant, dense products, numpy.linalg.solve),
sharing no code with the oracle.  The hammer of eq. (6) is applied in its
eliminated form (lumped-mass update substituted into the string equation),
while the oracle solves the joint system; agreement checks both.
"""
from __future__ import annotations

import numpy as np


def dmin(N, h):
    """D_{x-}: N x (N-1), fixed ends."""
    D = np.zeros((N, N - 1))
    for i in range(1, N + 1):
        if i <= N - 1:
            D[i - 1, i - 1] = 1.0 / h
        if i >= 2:
            D[i - 1, i - 2] = -1.0 / h
    return D


def interp_matrix(x_src, x_dst):
    """Matrix of np.interp (linear, constant beyond the ends)."""
    M = np.zeros((len(x_dst), len(x_src)))
    for j in range(len(x_src)):
        e = np.zeros(len(x_src))
        e[j] = 1.0
        M[:, j] = np.interp(x_dst, x_src, e)
    return M


_CUBIC_HALVES = {}


def interp_matrix_cubic_halves(Nl, x_dst):
    key = (Nl, tuple(np.round(np.asarray(x_dst, dtype=np.float64), 15)))
    if key not in _CUBIC_HALVES:
        _CUBIC_HALVES[key] = _interp_matrix_cubic_halves(Nl, x_dst)
    return _CUBIC_HALVES[key]


def _interp_matrix_cubic_halves(Nl, x_dst):
    """Cubic interpolation from the longitudinal half points (j - 1/2)/Nl,
    j = 1..Nl, to the positions x_dst: for each unit vector, the cubic through
    the four half points around x, those past an end taking the value of their
    mirror image about that end (p_0 = p_1, p_{-1} = p_2, p_{Nl+1} = p_{Nl},
    ...), fitted with numpy and evaluated."""
    h = 1.0 / Nl
    M = np.zeros((len(x_dst), Nl))

    def fold(j):
        if j < 1:
            return 1 - j
        if j > Nl:
            return 2 * Nl + 1 - j
        return j

    for col in range(Nl):
        e = np.zeros(Nl)
        e[col] = 1.0
        for r, x in enumerate(x_dst):
            j0 = int(np.floor(x / h + 0.5))
            js = np.arange(j0 - 1, j0 + 3)
            coef = np.polyfit((js - 0.5) * h, [e[fold(j) - 1] for j in js], 3)
            M[r, col] = np.polyval(coef, x)
    return M


def point_row_cubic(x, N, s):
    """Row of the cubic interpolant at x: for each interior node's unit vector,
    the cubic through the four nodes around x (ghost nodes u_{-1} = s u_1,
    u_{N+1} = s u_{N-1}, end nodes zero), fitted with numpy and evaluated."""
    h = 1.0 / N
    l = int(np.floor(x * N))
    m = np.arange(l - 1, l + 3)
    row = np.zeros(N - 1)
    # only the nodes of the four-point stencil and the two next to the ends
    # (the ghosts' mirrors) can get a weight; every other column fits zeros
    cand = sorted({j for j in range(l - 2, l + 2) if 0 <= j < N - 1} | {0, N - 2})
    for j in cand:
        ext = np.zeros(N + 3)               # nodes -1 .. N+1
        ext[j + 2] = 1.0
        ext[0] = s * ext[2]
        ext[N + 2] = s * ext[N]
        coef = np.polyfit(m * h, ext[m + 1], 3)
        row[j] = np.polyval(coef, x)
    return row


def point_row(x, N):
    """Row interpolating the interior nodes 1..N-1 at x (end nodes are zero)."""
    nodes = np.arange(N + 1) / N
    row = np.zeros(N - 1)
    for j in range(N - 1):
        e = np.zeros(N + 1)
        e[j + 1] = 1.0
        row[j] = np.interp(x, nodes, e)
    return row


def clamped_curvature(N, h):
    """Curvature at the nodes 0..N of a clamped string, (N+1) x (N-1), and the
    trapezoid weights of its energy: with u_0 = u_N = 0 and zero end slope the
    second difference at an end node is 2 u_1 / h^2 (resp. 2 u_{N-1} / h^2).
    The stiffness energy (h/2) sum_i w_i c_i^2 has the gradient h C^T W C u,
    so D_xxxx = C^T W C."""
    C = np.zeros((N + 1, N - 1))
    for i in range(1, N):
        C[i, i - 1] = -2.0
        if i - 2 >= 0:
            C[i, i - 2] = 1.0
        if i <= N - 2:
            C[i, i] = 1.0
    C[0, 0] = 2.0
    C[N, N - 2] = 2.0
    w = np.ones(N + 1)
    w[0] = w[N] = 0.5
    return C / h ** 2, w


class Dense:
    def __init__(self, p, g):
        self.p, self.g = p, g
        Nt, Nl = g["N_t"], g["N_l"]
        ht, k, th = g["h_t"], g["k"], g["theta"]
        self.nt = Nt - 1
        self.nl = Nl - 1 if Nl > 0 else 0
        self.Dm_t = dmin(Nt, ht)
        self.Dp_t = -self.Dm_t.T
        self.Dxx_t = self.Dp_t @ self.Dm_t
        Mx = 0.5 * (np.eye(self.nt, k=1) + np.eye(self.nt, k=-1))
        self.Theta = th * np.eye(self.nt) + (1 - th) * Mx
        if p.get("boundary", 0) == 1:
            C, w = clamped_curvature(Nt, ht)
            self.S = g["kappa"] ** 2 * k ** 2 * (C.T @ (w[:, None] * C))
        else:
            self.S = g["kappa"] ** 2 * k ** 2 * (self.Dxx_t @ self.Dxx_t)
        if Nl > 0:
            hl = g["h_l"]
            self.Dm_l = dmin(Nl, hl)
            self.Dp_l = -self.Dm_l.T
            self.Dxx_l = self.Dp_l @ self.Dm_l
            xt = (np.arange(1, Nt + 1) - 0.5) * ht
            xl = (np.arange(1, Nl + 1) - 0.5) * hl
            if p.get("grid_interp", 0) == 3:
                self.I_lt = interp_matrix_cubic_halves(Nl, xt)
            else:
                self.I_lt = interp_matrix(xl, xt)
            self.I_tl = (ht / hl) * self.I_lt.T

    def blocks(self, u_n, gamma):
        p, g = self.p, self.g
        k = g["k"]
        a2 = p["alpha"] ** 2
        phi2 = gamma ** 2 * k ** 2 * (a2 - 1) / 4
        G = gamma ** 2 * k ** 2
        Lam = np.diag(self.Dm_t @ u_n)
        V = -phi2 * self.Dp_t @ Lam @ Lam @ self.Dm_t
        It = np.eye(self.nt)
        Qp = self.Theta + p["sigma0_t"] * k * It - p["sigma1_t"] * k * self.Dxx_t
        Qm = self.Theta - p["sigma0_t"] * k * It + p["sigma1_t"] * k * self.Dxx_t
        Buu = -2 * self.Theta - G * self.Dxx_t + self.S
        if self.nl == 0:
            return Qp + V, Buu, Qm + V
        Il = np.eye(self.nl)
        Ktl = -phi2 * self.Dp_t @ Lam @ self.I_lt @ self.Dm_l
        Klt = -phi2 * self.Dp_l @ self.I_tl @ Lam @ self.Dm_t
        Qlp = (1 + p["sigma0_l"] * k) * Il - p["sigma1_l"] * k * self.Dxx_l
        Qlm = (1 - p["sigma0_l"] * k) * Il + p["sigma1_l"] * k * self.Dxx_l
        A = np.block([[Qp + V, Ktl], [Klt, Qlp]])
        Bm = np.block([[Buu, 2 * Ktl], [np.zeros((self.nl, self.nt)), -2 * Il - a2 * G * self.Dxx_l]])
        Cm = np.block([[Qm + V, Ktl], [Klt, Qlm]])
        return A, Bm, Cm


def gamma_at(p, n):
    t = n / p["fs"]
    f = p["f0"]
    if p.get("mod_type", 0) == 1:
        f *= 2.0 ** ((p["mod_depth_cents"] / 1200.0) * np.sin(2 * np.pi * p["mod_rate_hz"] * t))
    elif p.get("mod_type", 0) == 2:
        T = p["n_samples"] / p["fs"]
        f *= 2.0 ** ((p["glide_semitones"] / 12.0) * (t / T))
    return 2.0 * f


def run_dense(p, e, g, n_samples, schedule=None):
    """Step eq. (7) with dense solves; returns (traj_u, traj_z, u_H).

    schedule: optional [(m, hammer)] of hammers set on the sounding string
    before the step that computes w^{m+1}: the hammer takes the string's
    displacement at level m-1 under it and moves on with its speed,
    u_H^{m-1} = I_H u^{m-1}, u_H^m = u_H^{m-1} + k v_H."""
    D = Dense(p, g)
    nt, nl = D.nt, D.nl
    Nt, k = g["N_t"], g["k"]
    w0 = np.zeros(nt + nl)
    uH = np.zeros(n_samples)
    if e is not None and e["type"] == 1:
        x = np.arange(1, Nt) / Nt
        tri = np.where(x <= e["x"], e["c0"] * x / e["x"], e["c0"] * (1 - x) / (1 - e["x"]))
        w0[:nt] = tri
    w1 = w0.copy()
    traj = np.zeros((n_samples, nt + nl))
    traj[0], traj[1] = w0, w1
    events = dict(schedule or [])
    hm = None

    def hammer_of(x):
        if x.get("interp_order", 0) == 3:
            Ih = point_row_cubic(x["x"], Nt, 1.0 if p.get("boundary", 0) == 1 else -1.0)
        else:
            Ih = point_row(x["x"], Nt)
        return dict(Ih=Ih, Jh=Ih / g["h_t"], Mr=x["M_H"] / x["rhoA"], wpow=x["K_H"] / x["M_H"], aH=x["alpha_H"])

    if e is not None and e["type"] == 2:
        uH[1] = k * e["v_H"]
        hm = hammer_of(e)
    for n in range(1, n_samples - 1):
        if n in events:
            hm = hammer_of(events[n])
            uH[n - 1] = hm["Ih"] @ w0[:nt]
            uH[n] = uH[n - 1] + k * events[n]["v_H"]
        gam = gamma_at(p, n)
        A, Bm, Cm = D.blocks(w1[:nt], gam)
        rhs = -Bm @ w1 - Cm @ w0
        if hm is not None:
            Ih, Jh = hm["Ih"], hm["Jh"]
            eta_n = uH[n] - Ih @ w1[:nt]
            eta_m = uH[n - 1] - Ih @ w0[:nt]
            c = 0.5 * hm["wpow"] * eta_n ** (hm["aH"] - 1) if eta_n > 0 else 0.0
            beta = k * k * hm["Mr"] * c / (1 + k * k * c)
            A = A.copy()
            A[:nt, :nt] += beta * np.outer(Jh, Ih)
            rhs[:nt] += beta * Jh * (2 * uH[n] - uH[n - 1] + eta_m)
        w2 = np.linalg.solve(A, rhs)
        if hm is not None:
            uH[n + 1] = (2 * uH[n] - uH[n - 1] - k * k * c * (eta_m - Ih @ w2[:nt])) / (1 + k * k * c)
        traj[n + 1] = w2
        w0, w1 = w1, w2
    return traj[:, :nt], traj[:, nt:], uH


def energy(p, g, u1, u0, z1, z0, gamma):
    """H^{n+1/2}: discrete energy of the lossless unforced scheme (string only)."""
    Nt, Nl = g["N_t"], g["N_l"]
    ht, k, th, kap = g["h_t"], g["k"], g["theta"], g["kappa"]

    def half_diff(v, h):
        return np.diff(np.concatenate([[0.0], v, [0.0]])) / h

    def lap(v, h):
        w = np.concatenate([[0.0], v, [0.0]])
        return (w[2:] - 2 * w[1:-1] + w[:-2]) / h ** 2

    du = u1 - u0
    dpad = np.concatenate([[0.0], du, [0.0]])
    theta_du = th * du + (1 - th) * 0.5 * (dpad[2:] + dpad[:-2])
    q1, q0 = half_diff(u1, ht), half_diff(u0, ht)
    if p.get("boundary", 0) == 1:
        C, w = clamped_curvature(Nt, ht)
        stiff = np.dot(w * (C @ u1), C @ u0)
    else:
        stiff = np.dot(lap(u1, ht), lap(u0, ht))
    H = ht / (2 * k * k) * np.dot(du, theta_du) + gamma ** 2 * ht / 2 * np.dot(q1, q0) + kap ** 2 * ht / 2 * stiff
    if Nl > 0:
        hl = g["h_l"]
        a2 = p["alpha"] ** 2
        p1, p0 = half_diff(z1, hl), half_diff(z0, hl)
        xt = (np.arange(1, Nt + 1) - 0.5) * ht
        xl = (np.arange(1, Nl + 1) - 0.5) * hl
        if p.get("grid_interp", 0) == 3:
            I = interp_matrix_cubic_halves(Nl, xt)
            pt1, pt0 = I @ p1, I @ p0
        else:
            pt1, pt0 = np.interp(xt, xl, p1), np.interp(xt, xl, p0)
        qq = q1 * q0
        H += hl / (2 * k * k) * np.dot(z1 - z0, z1 - z0) + gamma ** 2 * a2 * hl / 2 * np.dot(p1, p0) \
            + gamma ** 2 * (a2 - 1) / 2 * ht * np.sum(qq * qq / 4 + qq * (pt1 + pt0) / 2)
    return H
