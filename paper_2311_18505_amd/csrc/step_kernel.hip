// Batched stepping kernel of libstringfdtd for gfx950.
//
// One wavefront owns one string for a whole launch: every lane holds a
// contiguous run of grid points of both grids in registers (lane l owns the
// transverse points l*mt+1 .. l*mt+mt and the longitudinal points
// l*ml+1 .. l*ml+ml), neighbours come from the adjacent lanes, and the two
// grids exchange interpolated values through LDS.  The scheme is eq. (7) of
// the paper written for the acceleration a = w^{n+1} - 2 w^n + w^{n-1}:
//     (A^n + beta J I) a = -(A^n + B^n + C^n) w^n - (A^n - C^n) v + 2 beta J eta^n,
// v = w^n - w^{n-1}, whose right-hand side is O(k^2 force) (the O(1) Theta
// terms cancel), which is what makes FP32 stepping accurate.  The linear
// system is solved by block Gauss-Seidel between the two grids around the
// constant Toeplitz blocks T_u0 = Theta + sigma0 k - sigma1 k D_xx and
// T_z = (1 + sigma0 k) - sigma1 k D_xx, each inverted exactly through its
// factorisation kT (1 + rho S-)(1 + rho S+) on the odd periodic extension of
// the fixed-end grid (two first-order recurrences per lane plus lane scans);
// the hammer's rank-one term is removed exactly by Sherman-Morrison.
#include <hip/hip_runtime.h>

#include "sfd_types.h"

namespace sfd {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Wave-uniform copies (scalar registers) of values every lane holds equally.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ float uni(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint64_t b = (uint64_t)x;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double x) {
  return __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, x)));
}
template <typename P>
__device__ __forceinline__ P *uni(P *x) {
  return (P *)(uintptr_t)uni((int64_t)(uintptr_t)x);
}

template <typename T>
__device__ __forceinline__ T lane_prev(T v) {  // value of lane-1 (0 for lane 0)
  T r = __shfl_up(v, 1, kWave);
  return lane_id() == 0 ? T(0) : r;
}

template <typename T>
__device__ __forceinline__ T lane_next(T v) {  // value of lane+1 (0 for the last lane)
  T r = __shfl_down(v, 1, kWave);
  return lane_id() == kWave - 1 ? T(0) : r;
}

// Deterministic wave sum: butterfly, then lane 0's value for everyone.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
  return __shfl(v, 0, kWave);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return __shfl(v, 0, kWave);
}

// Inclusive scan of x_l = e_l + g x_{l-1} over the lanes (x_{-1} = 0).
template <typename T>
__device__ __forceinline__ T scan_fwd(T e, T g) {
  T t = e, gp = g;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(t, d, kWave);
    if (lane_id() >= d) t = fma(gp, o, t);
    gp = gp * gp;
  }
  return t;
}

// Inclusive scan of x_l = e_l + g x_{l+1} over the lanes (x_64 = 0).
template <typename T>
__device__ __forceinline__ T scan_bwd(T e, T g) {
  T t = e, gp = g;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_down(t, d, kWave);
    if (lane_id() + d < kWave) t = fma(gp, o, t);
    gp = gp * gp;
  }
  return t;
}

// x[m-1] for a wave-uniform m >= 1 (no runtime register indexing).
template <typename T, int MM>
__device__ __forceinline__ T last_of(const T (&x)[MM], int m) {
  T v = x[0];
#pragma unroll
  for (int j = 1; j < MM; ++j)
    if (j < m) v = x[j];
  return v;
}

// Point evaluation w0 x(n0) + w1 x(n1) of a lane-blocked array (m slots per
// lane, nodes 1-based, node 0 = absent), returned to every lane in FP64.
template <typename T, int MM>
__device__ __forceinline__ double point_eval(const T (&x)[MM], const T (&c)[MM], int m, int n0, double w0, int n1,
                                             double w1) {
  const int base = lane_id() * m;
  double part = 0.0;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    if (r >= m) continue;
    const int i = base + r + 1;
    const double v = (double)x[r] - (double)c[r];
    if (i == n0) part += w0 * v;
    if (i == n1) part += w1 * v;
  }
  const int l0 = n0 ? (n0 - 1) / m : 0, l1 = n1 ? (n1 - 1) / m : 0;
  double y = __shfl(part, l0, kWave);
  if (n1 && l1 != l0) y += __shfl(part, l1, kWave);
  return y;
}

template <typename T, int MM>
struct Toep {
  T rho, itk, g;      // factor, 1/kT, (-rho)^m
  T pr[MM];           // (-rho)^{r+1}
  T qr[MM];           // (-rho)^{m-r}
};

template <typename T, int MM>
__device__ __forceinline__ void toep_init(Toep<T, MM> &tp, double rho, double itk, int m) {
  tp.rho = (T)rho;
  tp.itk = (T)itk;
  T pw = T(1);
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    pw = pw * (-tp.rho);
    tp.pr[r] = pw;
  }
  pw = T(1);
#pragma unroll
  for (int r = MM - 1; r >= 0; --r) {
    if (r < m) pw = pw * (-tp.rho);
    tp.qr[r] = pw;
  }
  tp.g = pw;   // (-rho)^m
}

// Exact solve of the fixed-end symmetric Toeplitz tridiagonal system
// kT (1 + rho S-)(1 + rho S+) x = b on nodes 1..n (n = N-1), m slots per lane.
//   forward:  z_i = b_i / kT - rho z_{i-1},  z_0 = sum_m wb_m b_m  (odd extension)
//   backward: x_i = z_i - rho x_{i+1},       x_N = 0
// valid: number of this lane's slots holding nodes <= n.
template <typename T, int MM>
__device__ __forceinline__ void toeplitz_solve(T (&x)[MM], const T (&b)[MM], const T (&wb)[MM], int m, int valid,
                                               const Toep<T, MM> &tp) {
  T part = T(0);
#pragma unroll
  for (int r = 0; r < MM; ++r)
    if (r < m) part = fma(wb[r], b[r], part);
  const T z0 = wave_sum(part);
  T z[MM];
  T prev = T(0);
#pragma unroll
  for (int r = 0; r < MM; ++r)
    if (r < m) {
      z[r] = fma(-tp.rho, prev, b[r] * tp.itk);
      prev = z[r];
    }
  T e = prev;
  if (lane_id() == 0) e = fma(tp.g, z0, e);
  const T Z = scan_fwd(e, tp.g);
  T C = lane_prev(Z);
  if (lane_id() == 0) C = z0;
#pragma unroll
  for (int r = 0; r < MM; ++r)
    if (r < m) {
      z[r] = fma(tp.pr[r], C, z[r]);
      if (r >= valid) z[r] = T(0);
    }
  prev = T(0);
#pragma unroll
  for (int r = MM - 1; r >= 0; --r)
    if (r < m) {
      x[r] = fma(-tp.rho, prev, z[r]);
      prev = x[r];
    }
  const T X = scan_bwd(prev, tp.g);
  const T Dn = lane_next(X);
#pragma unroll
  for (int r = 0; r < MM; ++r)
    if (r < m) {
      x[r] = fma(tp.qr[r], Dn, x[r]);
      if (r >= valid) x[r] = T(0);
    }
}

// x += (v - cv) with compensation: the stored pairs represent x - c and v - cv.
template <typename T, bool KAHAN>
__device__ __forceinline__ void update_pos(T &x, T &c, T v, T cv) {
  if (KAHAN) {
    const T yy = v - (c + cv);
    const T t = x + yy;
    c = (t - x) - yy;
    x = t;
  } else {
    x += v;
  }
}

// s += y with compensation: the stored pair represents s - c.
template <typename T, bool KAHAN>
__device__ __forceinline__ void kahan_add(T &s, T &c, T y) {
  if (KAHAN) {
    const T yy = y - c;
    const T t = s + yy;
    c = (t - s) - yy;
    s = t;
  } else {
    s += y;
  }
}

// (gamma^n k)^2 with gamma^n = 2 f0(nk), f0 modulated by vibrato or glide.
// Out of line: evaluated once per 64 steps (one step per lane), its FP64
// transcendental code stays out of the stepping loop's registers.
__device__ __attribute__((noinline)) double gamma2k2_at(const Desc &D, int64_t n) {
  const double t = (double)n / D.fs;
  double f = D.f0;
  if (D.mod_type == 1)
    f = f * exp2(D.mod_a * sin(2.0 * M_PI * D.mod_b * t));
  else if (D.mod_type == 2)
    f = f * exp2(D.mod_a * (t / D.mod_b));
  const double gam = 2.0 * f;
  return gam * gam * D.k * D.k;
}

// Contact coefficient c = omega^{1+alpha_H} (eta^+)^{alpha_H - 1} / 2 of eq. (6)
// (power factor at time n); out of line, used only while the hammer touches.
__device__ __attribute__((noinline)) double contact_coef(double eta, double omega_pow, double alpha_H) {
  return eta > 0.0 ? 0.5 * omega_pow * pow(eta, alpha_H - 1.0) : 0.0;
}

template <typename T>
__device__ __forceinline__ double to_d(T hi, T c) {
  return (double)hi - (double)c;
}

// Discrete energy H^{n+1/2} (FP64) from w^{n+1} = (u - cu, z - cz) and
// w^n = w^{n+1} - v, read from the string's state block in global memory:
// kinetic and linear potential of both grids plus the nonlinear potential
// (gamma^2 (alpha^2-1)/2)(p q^2/2 + q^4/8) in the time-paired form of the
// scheme.  Not inlined: it runs once per monitor period and keeps its FP64
// temporaries out of the stepping loop's registers.
template <typename T, int MM>
__device__ __attribute__((noinline)) double energy_fp64(const Desc &D, double g2k2, double *sD) {
  const int lane = lane_id();
  const int mt = D.mt, ml = D.ml, nt = D.nt, Nt = D.Nt, Nl = D.Nl, nl = D.nl;
  const double k = D.k, th = D.theta;
  const T *st = (const T *)D.st;
  const T *tf = (const T *)D.tabf;
  double U1[MM], U0[MM], DU[MM];
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    const bool ok = r < mt;
    U1[r] = ok ? to_d(st[(0 * mt + r) * kWave + lane], st[(2 * mt + r) * kWave + lane]) : 0.0;
    DU[r] = ok ? to_d(st[(1 * mt + r) * kWave + lane], st[(3 * mt + r) * kWave + lane]) : 0.0;
    U0[r] = U1[r] - DU[r];
  }
  const double dul = lane_prev(last_of<double, MM>(DU, mt)), dur = lane_next(DU[0]);
  const double u1l = lane_prev(last_of<double, MM>(U1, mt)), u0l = lane_prev(last_of<double, MM>(U0, mt));
  double q1[MM], q0[MM];
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    const double a1 = r == 0 ? u1l : U1[r > 0 ? r - 1 : 0];
    const double a0 = r == 0 ? u0l : U0[r > 0 ? r - 1 : 0];
    q1[r] = (U1[r] - a1) * D.Ntd;
    q0[r] = (U0[r] - a0) * D.Ntd;
  }
  const double q1r = lane_next(q1[0]), q0r = lane_next(q0[0]);
  double kin = 0.0, pot = 0.0, stf = 0.0;
  const int base = lane * mt;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    if (r >= mt) continue;
    const int i = base + r + 1;
    const bool nx = r + 1 < mt && r + 1 < MM;
    const double n1 = nx ? q1[r + 1 < MM ? r + 1 : r] : q1r;
    const double n0 = nx ? q0[r + 1 < MM ? r + 1 : r] : q0r;
    const double c1 = (n1 - q1[r]) * D.Ntd, c0 = (n0 - q0[r]) * D.Ntd;
    const double dl = r == 0 ? dul : DU[r > 0 ? r - 1 : 0];
    const double dr = nx ? DU[r + 1 < MM ? r + 1 : r] : dur;
    if (i <= nt) {
      kin += DU[r] * (th * DU[r] + 0.5 * (1.0 - th) * (dl + dr));
      stf += c1 * c0;
    }
    if (i <= Nt) pot += q1[r] * q0[r];
  }
  const double gam2 = g2k2 / (k * k);
  const double kap2 = D.cS / (k * k * D.Ntd * D.Ntd);
  double H = (1.0 / D.Ntd) / (2.0 * k * k) * kin + gam2 / D.Ntd / 2.0 * pot + kap2 / D.Ntd / 2.0 * stf;
  if (nl > 0) {
    const int zo = 4 * mt * kWave;
    double Z1[MM], Z0[MM], DZ[MM];
#pragma unroll
    for (int r = 0; r < MM; ++r) {
      const bool ok = r < ml;
      Z1[r] = ok ? to_d(st[zo + (0 * ml + r) * kWave + lane], st[zo + (2 * ml + r) * kWave + lane]) : 0.0;
      DZ[r] = ok ? to_d(st[zo + (1 * ml + r) * kWave + lane], st[zo + (3 * ml + r) * kWave + lane]) : 0.0;
      Z0[r] = Z1[r] - DZ[r];
    }
    const double z1l = lane_prev(last_of<double, MM>(Z1, ml)), z0l = lane_prev(last_of<double, MM>(Z0, ml));
    double kz = 0.0, pz = 0.0;
    const int lb = lane * ml;
#pragma unroll
    for (int r = 0; r < MM; ++r) {
      if (r >= ml) continue;
      const double a1 = r == 0 ? z1l : Z1[r > 0 ? r - 1 : 0];
      const double a0 = r == 0 ? z0l : Z0[r > 0 ? r - 1 : 0];
      const double p1 = (Z1[r] - a1) * D.Nld, p0 = (Z0[r] - a0) * D.Nld;
      const int j = lb + r + 1;
      if (j <= nl) kz += DZ[r] * DZ[r];
      if (j <= Nl) pz += p1 * p0;
      sD[2 * (lb + r)] = p1;
      sD[2 * (lb + r) + 1] = p0;
    }
    __syncthreads();
    // p^{n+1}, p^n interpolated to the transverse half points
    double nlt = 0.0;
#pragma unroll
    for (int r = 0; r < MM; ++r) {
      if (r >= mt) continue;
      const int i = base + r + 1;
      if (i > Nt) continue;
      const uint32_t jab = D.tab[r * kWave + lane];
      const int ja = (int)(jab & 0xffffu), jb = (int)(jab >> 16);
      const double w = (double)tf[r * kWave + lane];
      const double pt1 = (1.0 - w) * sD[2 * (ja - 1)] + w * sD[2 * (jb - 1)];
      const double pt0 = (1.0 - w) * sD[2 * (ja - 1) + 1] + w * sD[2 * (jb - 1) + 1];
      const double qq = q1[r] * q0[r];
      nlt += qq * qq / 4.0 + qq * (pt1 + pt0) / 2.0;
    }
    __syncthreads();
    const double a2 = D.a2;
    H += (1.0 / D.Nld) / (2.0 * k * k) * kz + gam2 * a2 / D.Nld / 2.0 * pz + gam2 * (a2 - 1.0) / 2.0 / D.Ntd * nlt;
  }
  return wave_sum(H);
}

template <typename T, int MM>
__device__ __forceinline__ void store_state(T *st, const T (&u)[MM], const T (&vu)[MM], const T (&cu)[MM],
                                            const T (&cvu)[MM], const T (&z)[MM], const T (&vz)[MM],
                                            const T (&cz)[MM], const T (&cvz)[MM], int mt, int ml, int lane) {
  const int zo = 4 * mt * kWave;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    if (r < mt) {
      st[(0 * mt + r) * kWave + lane] = u[r];
      st[(1 * mt + r) * kWave + lane] = vu[r];
      st[(2 * mt + r) * kWave + lane] = cu[r];
      st[(3 * mt + r) * kWave + lane] = cvu[r];
    }
    if (r < ml) {
      st[zo + (0 * ml + r) * kWave + lane] = z[r];
      st[zo + (1 * ml + r) * kWave + lane] = vz[r];
      st[zo + (2 * ml + r) * kWave + lane] = cz[r];
      st[zo + (3 * ml + r) * kWave + lane] = cvz[r];
    }
  }
}

// I_(t)->(l) gather for one longitudinal half point: the sums of the two
// contribution arrays over its ranges [sa, sa+na) and [sb, sb+nb) (packed as
// start | count << 16).  Uniform trip count gmax, predicated per lane.
template <typename T>
__device__ __forceinline__ T range_gather(const T *sA, const T *sB, uint32_t ra, uint32_t rb, int gmax) {
  const int sa = (int)(ra & 0xffffu), na = (int)(ra >> 16);
  const int sb = (int)(rb & 0xffffu), nb = (int)(rb >> 16);
  T acc = T(0);
  for (int c = 0; c < gmax; ++c) {
    const T va = sA[c < na ? sa + c : 0];
    const T vb = sB[c < nb ? sb + c : 0];
    acc += (c < na ? va : T(0)) + (c < nb ? vb : T(0));
  }
  return acc;
}

template <typename T, int MM, bool KAHAN>
__device__ __forceinline__ void run_steps(const LaunchArgs &a, const Desc &D, Status *S, const int64_t done,
                                          const int64_t nsteps, T *sP, T *sA, T *sB);

template <typename T, int MM, bool KAHAN>
__device__ void run_string(const LaunchArgs &a, int s, T *sP, T *sA, T *sB) {
  const Desc &D = a.desc[s];
  Status *S = a.status + s;
  const int64_t n_samples = uni(D.n_samples);
  const int64_t done = uni(S->samples_done);
  const int64_t left = n_samples - done;
  const int64_t nsteps = a.n_steps < left ? a.n_steps : left;
  // one uniform guard, no early return (keeps the persistent loop structured)
  if (uni(S->flags) == 0 && done >= 2 && nsteps > 0) run_steps<T, MM, KAHAN>(a, D, S, done, nsteps, sP, sA, sB);
}

template <typename T, int MM, bool KAHAN>
__device__ __forceinline__ void run_steps(const LaunchArgs &a, const Desc &D, Status *S, const int64_t done,
                                          const int64_t nsteps, T *sP, T *sA, T *sB) {
  const int lane = lane_id();
  const int Nt = uni(D.Nt), Nl = uni(D.Nl), nt = uni(D.nt), nl = uni(D.nl), mt = uni(D.mt), ml = uni(D.ml);
  const bool has_l = nl > 0;
  // uniform coefficients (scalar registers)
  const int mod_type = uni(D.mod_type), ham_on = uni(D.ham_on), mon_check = uni(D.mon_check);
  const int hn0 = uni(D.hn0), hn1 = uni(D.hn1), on0 = uni(D.on0), on1 = uni(D.on1);
  const double hw0 = uni(D.hw0), hw1 = uni(D.hw1), ow0 = uni(D.ow0), ow1 = uni(D.ow1);
  const double omega_pow = uni(D.omega_pow), alpha_H = uni(D.alpha_H), Mr = uni(D.Mr), IHs = uni(D.IHs);
  const double g2k2_0 = uni(D.g2k2_0), a2m1_4 = uni(D.a2m1_4), a2d = uni(D.a2), Ntdd = uni(D.Ntd);
  const int gmax = uni(D.gmax);

  // ---- state and tables into registers ----
  T u[MM], vu[MM], cu[MM], cvu[MM], z[MM], vz[MM], cz[MM], cvz[MM];
  uint32_t jab[MM], rga[MM], rgb[MM];
  T wi[MM], wbu[MM], wbz[MM];
  T *st = (T *)uni(D.st);
  const T *tf = (const T *)uni(D.tabf);
  const uint32_t *tab = uni(D.tab);
  const int zo = 4 * mt * kWave;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    const bool ot = r < mt, ol = r < ml;
    u[r] = ot ? st[(0 * mt + r) * kWave + lane] : T(0);
    vu[r] = ot ? st[(1 * mt + r) * kWave + lane] : T(0);
    cu[r] = ot ? st[(2 * mt + r) * kWave + lane] : T(0);
    cvu[r] = ot ? st[(3 * mt + r) * kWave + lane] : T(0);
    z[r] = ol ? st[zo + (0 * ml + r) * kWave + lane] : T(0);
    vz[r] = ol ? st[zo + (1 * ml + r) * kWave + lane] : T(0);
    cz[r] = ol ? st[zo + (2 * ml + r) * kWave + lane] : T(0);
    cvz[r] = ol ? st[zo + (3 * ml + r) * kWave + lane] : T(0);
    jab[r] = ot ? tab[r * kWave + lane] : 0x00010001u;
    rga[r] = ol ? tab[(mt + r) * kWave + lane] : 0u;
    rgb[r] = ol ? tab[(mt + ml + r) * kWave + lane] : 0u;
    wi[r] = ot ? tf[r * kWave + lane] : T(0);
    wbu[r] = ot ? tf[(mt + r) * kWave + lane] : T(0);
    wbz[r] = ol ? tf[(2 * mt + r) * kWave + lane] : T(0);
  }
  const T *smv = tf + (2 * mt + ml) * kWave;   // Sherman-Morrison vector T_u0^{-1} J_H

  const int tb = lane * mt, lb = lane * ml;
  const int vt_node = max(0, min(mt, nt - tb));   // slots with nodes 1..nt
  const int vt_half = max(0, min(mt, Nt - tb));   // slots with half points 1..Nt
  const int vl_node = max(0, min(ml, nl - lb));
  const int vl_half = max(0, min(ml, Nl - lb));

  Toep<T, MM> Tu, Tz;
  toep_init<T, MM>(Tu, uni(D.rho_t), uni(D.itk_t), mt);
  toep_init<T, MM>(Tz, uni(D.rho_l), uni(D.itk_l), ml);
  const T Ntd = uni((T)D.Ntd), Nld = uni((T)D.Nld);
  const T cS = uni((T)D.cS), s0t2 = uni((T)(2.0 * D.s0k_t)), s1t2 = uni((T)(2.0 * D.s1k_t));
  const T s0l2 = uni((T)(2.0 * D.s0k_l)), s1l2 = uni((T)(2.0 * D.s1k_l));
  const T ratio = uni((T)D.ratio_lt);
  const double kk = uni(D.k * D.k);

  // hammer
  double uH_n = S->uH_n, uH_nm1 = S->uH_nm1, eta_nm1 = S->eta_nm1;
  int touched = S->touched;
  const bool ham = ham_on != 0;
  // monitor
  double H_ref = S->H_ref, H_last = S->H_latest;
  int64_t H_step = S->H_step;
  int flags = 0, max_sw = S->max_sweeps;
  int64_t tot_sw = S->total_sweeps;

  T *out = (T *)uni(D.out);
  const int64_t first_m = done;
  T ring = T(0);
  double g2blk = g2k2_0;
  int64_t blk0 = -1000000;

  int64_t it = 0;
  for (; it < nsteps; ++it) {
    const int64_t n = done - 1 + it;  // time level of this step; produces sample n+1
    // ---- gamma^n (f0 modulation), 64 steps per block, one per lane ----
    double g2k2 = g2k2_0;
    if (mod_type != 0) {
      if (n - blk0 >= kWave) {
        blk0 = n;
        g2blk = gamma2k2_at(D, n + lane);
      }
      g2k2 = __shfl(g2blk, (int)(n - blk0), kWave);
    }
    const T G = (T)g2k2;
    const T phi2 = uni((T)(g2k2 * a2m1_4));
    const T aG = uni((T)(g2k2 * a2d));

    // ---- slopes q (t half points) and p (l half points) ----
    T q[MM], p[MM];
    {
      const T ul = lane_prev(last_of<T, MM>(u, mt)), cl = lane_prev(last_of<T, MM>(cu, mt));
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        const T um = r == 0 ? ul : u[r > 0 ? r - 1 : 0];
        const T cm = r == 0 ? cl : cu[r > 0 ? r - 1 : 0];
        q[r] = (r < vt_half) ? ((u[r] - um) - (cu[r] - cm)) * Ntd : T(0);
      }
    }
    if (has_l) {
      const T zl = lane_prev(last_of<T, MM>(z, ml)), cl = lane_prev(last_of<T, MM>(cz, ml));
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        const T zm = r == 0 ? zl : z[r > 0 ? r - 1 : 0];
        const T cm = r == 0 ? cl : cz[r > 0 ? r - 1 : 0];
        p[r] = (r < vl_half) ? ((z[r] - zm) - (cz[r] - cm)) * Nld : T(0);
      }
    }

    // ---- right-hand side, transverse ----
    T ru[MM], rz[MM];
    T f[MM];
#pragma unroll
    for (int r = 0; r < MM; ++r) f[r] = T(0);
    if (has_l) {
      // p~ = I_(l)->(t) p and the transposed contributions of q^2
#pragma unroll
      for (int r = 0; r < MM; ++r)
        if (r < ml) sP[lb + r] = p[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        if (r >= mt) continue;
        const int ja = (int)(jab[r] & 0xffffu), jb = (int)(jab[r] >> 16);
        const T w = wi[r];
        const T pt = (T(1) - w) * sP[ja - 1] + w * sP[jb - 1];
        const T q2 = q[r] * q[r];
        f[r] = q[r] * (q2 + T(2) * pt);
        sA[tb + r] = (T(1) - w) * q2;
        sB[tb + r] = w * q2;
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int r = 0; r < MM; ++r) f[r] = T(0);
    }
    {
      T c[MM];
      const T qr = lane_next(q[0]);
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        const T qn = (r + 1 < mt && r + 1 < MM) ? q[r + 1 < MM ? r + 1 : r] : qr;
        c[r] = (r < vt_node) ? (qn - q[r]) * Ntd : T(0);
      }
      const T cl = lane_prev(last_of<T, MM>(c, mt)), cr = lane_next(c[0]);
      const T fr = lane_next(f[0]);
      const T vl = lane_prev(last_of<T, MM>(vu, mt)), vr = lane_next(vu[0]);
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        if (r >= mt) continue;
        const T cm = r == 0 ? cl : c[r > 0 ? r - 1 : 0];
        const T cp = (r + 1 < mt && r + 1 < MM) ? c[r + 1 < MM ? r + 1 : r] : cr;
        const T fp = (r + 1 < mt && r + 1 < MM) ? f[r + 1 < MM ? r + 1 : r] : fr;
        const T vm = r == 0 ? vl : vu[r > 0 ? r - 1 : 0];
        const T vp = (r + 1 < mt && r + 1 < MM) ? vu[r + 1 < MM ? r + 1 : r] : vr;
        T acc = G * c[r] - cS * ((cp - T(2) * c[r]) + cm);
        acc = fma(T(2) * phi2 * Ntd, fp - f[r], acc);
        acc = fma(-s0t2, vu[r], acc);
        acc = fma(s1t2, (vp - T(2) * vu[r]) + vm, acc);
        ru[r] = (r < vt_node) ? acc : T(0);
      }
    }
    // ---- right-hand side, longitudinal ----
    if (has_l) {
      T g[MM];
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        g[r] = r < ml ? range_gather<T>(sA, sB, rga[r], rgb[r], gmax) * ratio : T(0);
      }
      const T pr = lane_next(p[0]), gr = lane_next(g[0]);
      const T vl = lane_prev(last_of<T, MM>(vz, ml)), vr = lane_next(vz[0]);
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        if (r >= ml) continue;
        const T pn = (r + 1 < ml && r + 1 < MM) ? p[r + 1 < MM ? r + 1 : r] : pr;
        const T gn = (r + 1 < ml && r + 1 < MM) ? g[r + 1 < MM ? r + 1 : r] : gr;
        const T vm = r == 0 ? vl : vz[r > 0 ? r - 1 : 0];
        const T vp = (r + 1 < ml && r + 1 < MM) ? vz[r + 1 < MM ? r + 1 : r] : vr;
        T acc = aG * ((pn - p[r]) * Nld);
        acc = fma(T(2) * phi2 * Nld, gn - g[r], acc);
        acc = fma(-s0l2, vz[r], acc);
        acc = fma(s1l2, (vp - T(2) * vz[r]) + vm, acc);
        rz[r] = (r < vl_node) ? acc : T(0);
      }
    }

    // ---- hammer: contact coefficient at time n, right-hand side 2 beta J eta^n ----
    double eta_n = 0.0, cH = 0.0, beta = 0.0;
    if (ham) {
      const double Iu = point_eval<T, MM>(u, cu, mt, hn0, hw0, hn1, hw1);
      eta_n = uni(uH_n - Iu);
      if (eta_n > 0.0) {
        cH = uni(contact_coef(eta_n, omega_pow, alpha_H));
        touched = 1;
      }
      beta = uni(kk * Mr * cH / (1.0 + kk * cH));
      if (beta != 0.0) {
        const T add0 = (T)(2.0 * beta * hw0 * Ntdd * eta_n), add1 = (T)(2.0 * beta * hw1 * Ntdd * eta_n);
#pragma unroll
        for (int r = 0; r < MM; ++r) {
          const int i = tb + r + 1;
          if (r < mt && i == hn0) ru[r] += add0;
          if (r < mt && i == hn1) ru[r] += add1;
        }
      }
    }

    // ---- coupled solve: block Gauss-Seidel around T_u0 (+ hammer) and T_z ----
    T au[MM], az[MM];
#pragma unroll
    for (int r = 0; r < MM; ++r) {
      au[r] = T(0);
      az[r] = T(0);
    }
    T smr[MM];
    const bool sm_on = beta != 0.0;
    if (sm_on) {
#pragma unroll
      for (int r = 0; r < MM; ++r) smr[r] = r < mt ? smv[r * kWave + lane] : T(0);
    }
    const T smfac = (T)(beta / (1.0 + beta * IHs));
    T zero[MM];
#pragma unroll
    for (int r = 0; r < MM; ++r) zero[r] = T(0);
    int sweep = 0;
    bool conv = !has_l;
    for (; sweep < a.max_sweeps; ++sweep) {
      // transverse right-hand side with the current coupling terms
      T bu[MM];
      if (sweep == 0 || !has_l) {
#pragma unroll
        for (int r = 0; r < MM; ++r) bu[r] = ru[r];
      } else {
        // d = D_x- a_u (t half), dz = D_x- a_z (l half), e = q (q d + I dz)
        const T al = lane_prev(last_of<T, MM>(au, mt));
        const T zl = lane_prev(last_of<T, MM>(az, ml));
#pragma unroll
        for (int r = 0; r < MM; ++r)
          if (r < ml) {
            const T zm = r == 0 ? zl : az[r > 0 ? r - 1 : 0];
            sP[lb + r] = (r < vl_half) ? (az[r] - zm) * Nld : T(0);
          }
        __syncthreads();
        T e[MM];
#pragma unroll
        for (int r = 0; r < MM; ++r) {
          e[r] = T(0);
          if (r >= mt) continue;
          const T am = r == 0 ? al : au[r > 0 ? r - 1 : 0];
          const T d = (au[r] - am) * Ntd;
          const int ja = (int)(jab[r] & 0xffffu), jb = (int)(jab[r] >> 16);
          const T w = wi[r];
          const T idz = (T(1) - w) * sP[ja - 1] + w * sP[jb - 1];
          e[r] = (r < vt_half) ? q[r] * fma(q[r], d, idz) : T(0);
        }
        __syncthreads();
        const T er = lane_next(e[0]);
#pragma unroll
        for (int r = 0; r < MM; ++r) {
          const T en = (r + 1 < mt && r + 1 < MM) ? e[r + 1 < MM ? r + 1 : r] : er;
          bu[r] = (r < vt_node) ? fma(phi2 * Ntd, en - e[r], ru[r]) : T(0);
        }
      }
      T nu[MM];
      toeplitz_solve<T, MM>(nu, bu, wbu, mt, vt_node, Tu);
      if (sm_on) {
        // Sherman-Morrison for the rank-one hammer term beta J I
        const T Iy = (T)point_eval<T, MM>(nu, zero, mt, hn0, hw0, hn1, hw1);
        const T fac = smfac * Iy;
#pragma unroll
        for (int r = 0; r < MM; ++r)
          if (r < mt) nu[r] = fma(-fac, smr[r], nu[r]);
      }
      T delta = T(0), amax = T(0);
#pragma unroll
      for (int r = 0; r < MM; ++r)
        if (r < mt) {
          delta = fmax(delta, fabs(nu[r] - au[r]));
          amax = fmax(amax, fabs(nu[r]));
          au[r] = nu[r];
        }
      if (has_l) {
        // longitudinal right-hand side: r_z + phi^2 D_x+ I_(t)->(l) (q D_x- a_u)
        const T al = lane_prev(last_of<T, MM>(au, mt));
#pragma unroll
        for (int r = 0; r < MM; ++r) {
          if (r >= mt) continue;
          const T am = r == 0 ? al : au[r > 0 ? r - 1 : 0];
          const T fq = (r < vt_half) ? q[r] * ((au[r] - am) * Ntd) : T(0);
          const T w = wi[r];
          sA[tb + r] = (T(1) - w) * fq;
          sB[tb + r] = w * fq;
        }
        __syncthreads();
        T gg[MM];
#pragma unroll
        for (int r = 0; r < MM; ++r) {
          gg[r] = r < ml ? range_gather<T>(sA, sB, rga[r], rgb[r], gmax) * ratio : T(0);
        }
        __syncthreads();
        const T gr = lane_next(gg[0]);
        T bz[MM];
#pragma unroll
        for (int r = 0; r < MM; ++r) {
          const T gn = (r + 1 < ml && r + 1 < MM) ? gg[r + 1 < MM ? r + 1 : r] : gr;
          bz[r] = (r < vl_node) ? fma(phi2 * Nld, gn - gg[r], rz[r]) : T(0);
        }
        T nz[MM];
        toeplitz_solve<T, MM>(nz, bz, wbz, ml, vl_node, Tz);
#pragma unroll
        for (int r = 0; r < MM; ++r)
          if (r < ml) {
            delta = fmax(delta, fabs(nz[r] - az[r]));
            amax = fmax(amax, fabs(nz[r]));
            az[r] = nz[r];
          }
        delta = wave_max(delta);
        amax = wave_max(amax);
        const int done_now = uni((int)((sweep > 0 && delta <= (T)a.tol * amax) || amax == T(0)));
        if (done_now) {
          conv = true;
          ++sweep;
          break;
        }
      } else {
        ++sweep;
        break;
      }
    }
    if (!conv) flags |= kFlagNoConverge;
    tot_sw += sweep;
    max_sw = sweep > max_sw ? sweep : max_sw;

    // ---- state update: v^{n+1/2} = v^{n-1/2} + a, w^{n+1} = w^n + v^{n+1/2} ----
#pragma unroll
    for (int r = 0; r < MM; ++r) {
      if (r < mt) {
        kahan_add<T, KAHAN>(vu[r], cvu[r], au[r]);
        update_pos<T, KAHAN>(u[r], cu[r], vu[r], cvu[r]);
      }
      if (r < ml) {
        kahan_add<T, KAHAN>(vz[r], cvz[r], az[r]);
        update_pos<T, KAHAN>(z[r], cz[r], vz[r], cvz[r]);
      }
    }

    // ---- hammer lumped mass (eq. 6) ----
    if (ham) {
      const double Iu1 = point_eval<T, MM>(u, cu, mt, hn0, hw0, hn1, hw1);
      const double uH_np1 = uni((2.0 * uH_n - uH_nm1 - kk * cH * (eta_nm1 - Iu1)) / (1.0 + kk * cH));
      uH_nm1 = uH_n;
      uH_n = uH_np1;
      eta_nm1 = eta_n;
    }

    // ---- readout y^{n+1} = I(x_out) u^{n+1} into the 64-sample ring ----
    const int64_t m = n + 1;
    {
      const double y = point_eval<T, MM>(u, cu, mt, on0, ow0, on1, ow1);
      if (lane == (int)((m - first_m) & (kWave - 1))) ring = (T)y;
    }

    // ---- FP64 energy monitor ----
    bool bad = false;
    if (a.mon_period > 0 && ((n + 1) % a.mon_period) == 0) {
      store_state<T, MM>(st, u, vu, cu, cvu, z, vz, cz, cvz, mt, ml, lane);
      __syncthreads();
      const double H = uni(energy_fp64<T, MM>(D, g2k2, (double *)sA));
      H_last = H;
      H_step = n;
      bad = !isfinite(H);
      if (!bad && mon_check && !touched && H_ref > 0.0 && H > H_ref * (1.0 + a.mon_tol)) bad = true;
      H_ref = H;
      touched = 0;
      if (bad) flags |= kFlagUnstable;
    }
    // coalesced burst of 64 samples from first_m + 64 j: every lane stores;
    // lanes past m write slots that a later step overwrites (or the 64-sample
    // padding after n_samples), never a sample before first_m
    if (((m - first_m) & (kWave - 1)) == kWave - 1 || it == nsteps - 1 || bad)
      out[first_m + ((m - first_m) & ~(int64_t)(kWave - 1)) + lane] = ring;
    if (bad) {
      ++it;
      break;
    }
  }

  // ---- write back ----
  store_state<T, MM>(st, u, vu, cu, cvu, z, vz, cz, cvz, mt, ml, lane);
  {  // every lane stores the same values (no lane-0-only region)
    S->samples_done = done + it;
    S->flags = flags;
    S->max_sweeps = max_sw;
    S->total_sweeps = tot_sw;
    S->H_latest = H_last;
    S->H_step = H_step;
    S->H_ref = H_ref;
    S->touched = touched;
    S->uH_n = uH_n;
    S->uH_nm1 = uH_nm1;
    S->eta_nm1 = eta_nm1;
  }
}

template <typename T, int MM, bool KAHAN>
__global__ __launch_bounds__(64) void step_kernel(LaunchArgs a) {
  // exchange buffers: longitudinal half points; transverse contributions (2 x)
  __shared__ T sP[MM * kWave];
  __shared__ T sAB[2 * MM * kWave + 2 * MM * kWave * (sizeof(T) == 4 ? 1 : 0)];
  T *sA = sAB, *sB = sAB + MM * kWave;
  for (;;) {
    // every lane takes part; only lane 0 adds, so the wave draws one ticket
    int w = atomicAdd(a.counter, lane_id() == 0 ? 1 : 0);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= a.n_work) break;
    const int s = __builtin_amdgcn_readfirstlane(a.work[w]);
    run_string<T, MM, KAHAN>(a, s, sP, sA, sB);
  }
}

// Restores slots first..first+count-1 to their state right after excitation:
// one block per slot copies the saved state block and the saved status.
template <typename T>
__global__ void rewind_kernel(const Desc *desc, Status *status, const Status *status0, int first, int count) {
  const int s = first + (int)blockIdx.x;
  if ((int)blockIdx.x >= count) return;
  const Desc &D = desc[s];
  if (!D.st0) return;
  T *dst = (T *)D.st;
  const T *src = (const T *)D.st0;
  for (int i = (int)threadIdx.x; i < D.st_elems; i += (int)blockDim.x) dst[i] = src[i];
  if (threadIdx.x == 0) status[s] = status0[s];
}

hipError_t launch_rewind(int precision, const Desc *desc, Status *status, const Status *status0, int first, int count,
                         hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(rewind_kernel<float>, dim3(count), dim3(256), 0, st, desc, status, status0, first, count);
  else
    hipLaunchKernelGGL(rewind_kernel<double>, dim3(count), dim3(256), 0, st, desc, status, status0, first, count);
  return hipGetLastError();
}

__global__ void zero_counters(int32_t *c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0;
}

template <typename T, bool KAHAN>
static hipError_t launch_class(int cls, const LaunchArgs &a, int blocks, hipStream_t st) {
  switch (cls) {
    case 0: hipLaunchKernelGGL((step_kernel<T, 2, KAHAN>), dim3(blocks), dim3(64), 0, st, a); break;
    case 1: hipLaunchKernelGGL((step_kernel<T, 4, KAHAN>), dim3(blocks), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((step_kernel<T, 8, KAHAN>), dim3(blocks), dim3(64), 0, st, a); break;
    default: hipLaunchKernelGGL((step_kernel<T, 16, KAHAN>), dim3(blocks), dim3(64), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_step(int precision, int cls, const LaunchArgs &a, int blocks, hipStream_t st) {
  if (precision == 1) return launch_class<float, true>(cls, a, blocks, st);
  return launch_class<double, false>(cls, a, blocks, st);
}

hipError_t launch_zero(int32_t *c, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_counters, dim3((n + 255) / 256), dim3(256), 0, st, c, n);
  return hipGetLastError();
}

}  // namespace sfd

namespace sfd {

template <typename T, bool KAHAN>
static int blocks_per_cu(int cls) {
  int n = 0;
  hipError_t e;
  switch (cls) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<T, 2, KAHAN>, 64, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<T, 4, KAHAN>, 64, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<T, 8, KAHAN>, 64, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<T, 16, KAHAN>, 64, 0); break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n;
}

int max_blocks_per_cu(int precision, int cls) {
  return precision == 1 ? blocks_per_cu<float, true>(cls) : blocks_per_cu<double, false>(cls);
}

}  // namespace sfd
