// Host planner of libstringfdtd: grid sizing, coefficients and per-string
// tables for the GPU stepping kernel (FP64 on the host, rounded once to the
// kernel precision on upload).
#include "planner.h"
#include "interp.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace sfd {

static bool finite_all(std::initializer_list<double> xs) {
  for (double x : xs)
    if (!std::isfinite(x)) return false;
  return true;
}

double theta_of(const sb_string_params &p) {
  // Sec. 3.2: theta = (1 + 4/pi^2)/2 unless given
  return p.theta > 0.0 ? p.theta : 0.5 * (1.0 + 4.0 / (M_PI * M_PI));
}

// Positive definiteness of the pentadiagonal 4 Theta - (gk)^2 (-D_xx) -
// (kk)^2 D_xxxx (clamped D_xxxx) on N-1 nodes, by the pivots of its LDL^T
// factorisation.
static bool clamped_energy_positive(int N, double th, double gk, double kk) {
  const int n = N - 1;
  const double h2 = 1.0 / ((double)N * N), g2 = gk * gk / h2, s2 = kk * kk / (h2 * h2);
  const double off1 = 2.0 * (1.0 - th) + g2 + 4.0 * s2, off2 = -s2;
  double d1 = 0.0, d2 = 0.0, l1p = 0.0;   // pivots of rows i-1, i-2; L(i-1, i-2)
  for (int i = 0; i < n; ++i) {
    // each end node adds its mirrored ghost to the diagonal of D_xxxx
    const double diag = 4.0 * th - 2.0 * g2 - (6.0 + (i == 0) + (i == n - 1)) * s2;
    const double a2 = i >= 2 ? off2 / d2 : 0.0;
    const double a1 = i >= 1 ? (off1 - (i >= 2 ? a2 * l1p * d2 : 0.0)) / d1 : 0.0;
    const double d = diag - (i >= 1 ? a1 * a1 * d1 : 0.0) - (i >= 2 ? a2 * a2 * d2 : 0.0);
    if (!(d > 0.0)) return false;
    d2 = d1;
    d1 = d;
    l1p = a1;
  }
  return true;
}

int plan_grid(const sb_string_params &p, GridPlan &g, std::string &err) {
  if (!finite_all({p.fs, p.f0, p.B, p.alpha, p.theta, p.sigma0_t, p.sigma1_t, p.sigma0_l, p.sigma1_l,
                   p.x_out, p.mod_depth_cents, p.mod_rate_hz, p.glide_semitones})) {
    err = "non-finite parameter";
    return SB_EINVAL;
  }
  if (!(p.fs > 0) || !(p.f0 > 0) || !(p.B >= 0) || !(p.alpha >= 1)) {
    err = "need fs > 0, f0 > 0, B >= 0, alpha >= 1";
    return SB_EINVAL;
  }
  const double th = theta_of(p);
  if (!(th > 0.5) || !(th <= 1.0)) {
    err = "need 1/2 < theta <= 1";
    return SB_EINVAL;
  }
  if (!(p.sigma0_t >= 0) || !(p.sigma1_t >= 0) || !(p.sigma0_l >= 0) || !(p.sigma1_l >= 0)) {
    err = "losses must be >= 0";
    return SB_EINVAL;
  }
  if (!(p.x_out > 0 && p.x_out < 1)) {
    err = "x_out must lie in (0,1)";
    return SB_EINVAL;
  }
  if (p.n_samples < 2) {
    err = "n_samples must be >= 2";
    return SB_EINVAL;
  }
  if (p.mod_type < 0 || p.mod_type > 2 || p.grid_t < 0 || p.grid_l < 0) {
    err = "bad mod_type or grid override";
    return SB_EINVAL;
  }
  if (p.readout_zeta != 0 && p.readout_zeta != 1) {
    err = "readout_zeta must be 0 or 1";
    return SB_EINVAL;
  }
  if (p.boundary != SB_BOUNDARY_SIMPLE && p.boundary != SB_BOUNDARY_CLAMPED) {
    err = "boundary must be SB_BOUNDARY_SIMPLE or SB_BOUNDARY_CLAMPED";
    return SB_EINVAL;
  }
  if (p.grid_interp != 0 && p.grid_interp != 1 && p.grid_interp != 3) {
    err = "grid_interp must be 0, 1 or 3";
    return SB_EINVAL;
  }
  const double k = 1.0 / p.fs;
  const double gamma0 = 2.0 * p.f0;                      // Sec. 4.1: f0 = gamma/2
  const double kappa = gamma0 * std::sqrt(p.B) / M_PI;    // Sec. 4.1: K = (pi kappa/gamma)^2, K := B
  double gmax = gamma0;                                   // largest gamma the modulation reaches
  if (p.mod_type == 1) gmax = gamma0 * std::exp2(std::fabs(p.mod_depth_cents) / 1200.0);
  if (p.mod_type == 2) gmax = gamma0 * std::exp2((p.glide_semitones > 0.0 ? p.glide_semitones : 0.0) / 12.0);
  // Transverse spacing: stability of the theta-scheme requires
  // lambda^2 + 4 nu^2 <= 2 theta - 1 (Von Neumann), which gives Sec. 3.2's
  // h^(t) at theta = 1.
  const double gk2 = gmax * gmax * k * k;
  const double h2 = (gk2 + std::sqrt(gk2 * gk2 + 16.0 * (2.0 * th - 1.0) * kappa * kappa * k * k)) /
                    (2.0 * (2.0 * th - 1.0));
  int Nt = p.grid_t > 0 ? p.grid_t : (int)std::floor(1.0 / std::sqrt(h2));
  // The bound above comes from the sine modes of simply supported ends.  With
  // clamped ends the scheme's energy (eq. (4a) without loss and
  // nonlinearity) stays non-negative exactly when 4 Theta - k^2 (gamma^2
  // (-D_xx) + kappa^2 D_xxxx) is positive semi-definite; lower N_t until it
  // is positive definite.
  if (p.boundary == SB_BOUNDARY_CLAMPED && p.grid_t <= 0)
    while (Nt >= 2 && !clamped_energy_positive(Nt, th, gmax * k, kappa * k)) --Nt;
  int Nl = 0;
  if (p.alpha != 1.0) Nl = p.grid_l > 0 ? p.grid_l : (int)std::floor(1.0 / (gmax * p.alpha * k));
  if (Nt < 2 || (p.alpha != 1.0 && Nl < 2)) {
    err = "grid has fewer than 2 intervals";
    return SB_EINVAL;
  }
  if (p.grid_interp == 3 && Nl > 0 && Nl < 4) {
    err = "the cubic grid interpolant needs N_l >= 4";
    return SB_EINVAL;
  }
  g.Nt = Nt;
  g.Nl = Nl;
  g.k = k;
  g.theta = th;
  g.gamma0 = gamma0;
  g.gamma_max = gmax;
  g.kappa = kappa;
  return SB_OK;
}

// Factor of the symmetric Toeplitz tridiagonal (c, d, c) = kT (1 + rho S-)(1 + rho S+)
static void toeplitz_factor(double d, double c, double &rho, double &kT) {
  if (c == 0.0) {
    rho = 0.0;
    kT = d;
    return;
  }
  rho = 2.0 * c / (d + std::sqrt(d * d - 4.0 * c * c));
  kT = d / (1.0 + rho * rho);
}

// Weights of the boundary value z_0 = sum_m w_m b_m of the forward
// recurrence on the odd 2N-periodic extension of a Dirichlet system.
static void boundary_weights(double rho, double kT, int N, std::vector<double> &w) {
  w.assign(N + 1, 0.0);
  if (rho == 0.0) return;
  const double mr = -rho;
  const double r2N = std::pow(rho, 2.0 * N);
  const double scale = 1.0 / (kT * (1.0 - r2N));
  for (int m = 1; m <= N - 1; ++m) {
    double a = std::pow(mr, (double)m);
    double b = std::pow(mr, (double)(2 * N - m));
    w[m] = (-a + b) * scale;
  }
}

// Linear interpolation row on the nodes 1..N-1 at x (end nodes are fixed).
static void point_interp(double x, int N, int &n0, int &n1, double &w0, double &w1) {
  int l = (int)std::floor(x * N);
  double w = x * N - l;
  n0 = (l >= 1 && l <= N - 1) ? l : 0;
  n1 = (l + 1 >= 1 && l + 1 <= N - 1) ? l + 1 : 0;
  w0 = n0 ? 1.0 - w : 0.0;
  w1 = n1 ? w : 0.0;
}

int plan_string(const sb_string_params &p, Plan &P, std::string &err, bool shapes) {
  GridPlan g;
  int st = plan_grid(p, g, err);
  if (st) return st;
  if (g.Nt > kMaxN || g.Nl > kMaxN) {
    err = "grid larger than 1024 intervals";
    return SB_EBUDGET;
  }
  P = Plan();
  P.grid = g;
  Desc &D = P.desc;
  const int Nt = g.Nt, Nl = g.Nl;
  D.Nt = Nt;
  D.Nl = Nl;
  D.nt = Nt - 1;
  D.nl = Nl > 0 ? Nl - 1 : 0;
  const int need = std::max(Nt, Nl);   // slots must cover the half points 1..N of both grids
  D.cls = -1;
  for (int c = 0; c < kNumClasses; ++c)
    if (need <= kClassLanes[c] * kClassSlots[c]) {
      D.cls = c;
      break;
    }
  if (D.cls < 0) {
    err = "string exceeds the largest size class";
    return SB_EBUDGET;
  }
  // a string of a class is laid out with the class's MM slots per lane on
  // both grids (nodes past a grid's end hold zeros), or, where the kernels
  // step narrower layouts (shapes), with the fewest slots per lane each grid
  // fits in: the stepping loops run over a grid's slots, so the work follows
  // the slot counts (the fewest in total; a string without a longitudinal
  // grid takes the narrowest level there)
  const int G = kClassLanes[D.cls];
  D.shape = 0;
  if (shapes) {
    int best = 2 * kClassSlots[D.cls] + 1;
    for (int s = 0; s < kNumShapes; ++s) {
      if (!shape_ok(D.cls, s)) continue;
      const int mt = shape_mt(D.cls, s), ml = shape_ml(D.cls, s);
      if (Nt <= G * mt && Nl <= G * ml && mt + ml < best) {
        best = mt + ml;
        D.shape = s;
      }
    }
  }
  D.mt = shape_mt(D.cls, D.shape);
  D.ml = shape_ml(D.cls, D.shape);
  D.mon_check = p.mod_type == 0 ? 1 : 0;
  D.n_samples = p.n_samples;
  const double k = g.k, th = g.theta;
  D.k = k;
  D.Ntd = Nt;
  D.Nld = Nl;
  D.theta = th;
  D.g2k2_0 = g.gamma0 * g.gamma0 * k * k;
  D.a2 = p.alpha * p.alpha;
  D.a2m1_4 = (p.alpha * p.alpha - 1.0) / 4.0;
  D.cS = g.kappa * g.kappa * k * k * (double)Nt * (double)Nt;
  D.s0k_t = p.sigma0_t * k;
  D.s1k_t = p.sigma1_t * k * (double)Nt * (double)Nt;
  D.s0k_l = p.sigma0_l * k;
  D.s1k_l = Nl > 0 ? p.sigma1_l * k * (double)Nl * (double)Nl : 0.0;
  D.ratio_lt = Nl > 0 ? (double)Nl / (double)Nt : 0.0;

  // T_u0 = Theta + sigma0 k I - sigma1 k D_xx (constant part of the
  // transverse block of A); T_z = (1 + sigma0 k) I - sigma1 k D_xx.
  const double dt = th + D.s0k_t + 2.0 * D.s1k_t, ct = 0.5 * (1.0 - th) - D.s1k_t;
  double kTt;
  toeplitz_factor(dt, ct, D.rho_t, kTt);
  D.itk_t = 1.0 / kTt;
  std::vector<double> wbt, wbl;
  boundary_weights(D.rho_t, kTt, Nt, wbt);
  double kTl = 1.0;
  if (Nl > 0) {
    const double dl = 1.0 + D.s0k_l + 2.0 * D.s1k_l, cl = -D.s1k_l;
    toeplitz_factor(dl, cl, D.rho_l, kTl);
    D.itk_l = 1.0 / kTl;
    boundary_weights(D.rho_l, kTl, Nl, wbl);
  }

  D.mod_type = p.mod_type;
  D.clamped = p.boundary == SB_BOUNDARY_CLAMPED ? 1 : 0;
  D.zeta_out = p.readout_zeta ? 1 : 0;
  if (Nl > 0) {
    double w0, w1;
    point_interp(p.x_out, Nl, D.zon0, D.zon1, w0, w1);
    D.zw = D.zon1 ? w1 : 1.0 - w0;
  }
  D.f0 = p.f0;
  D.fs = p.fs;
  if (p.mod_type == 1) {
    D.mod_a = p.mod_depth_cents / 1200.0;
    D.mod_b = p.mod_rate_hz;
  } else if (p.mod_type == 2) {
    D.mod_a = p.glide_semitones / 12.0;
    D.mod_b = (double)p.n_samples / p.fs;   // duration T
  }
  point_interp(p.x_out, Nt, D.on0, D.on1, D.ow0, D.ow1);

  // tables, lane-major [slot][lane]; the cubic grid interpolant (p = 3)
  // appends two more range tables and three more weights per t-slot
  const bool cubic = p.grid_interp == 3 && Nl > 0;
  D.grid_interp = cubic ? 3 : 1;
  const int mt = D.mt, ml = D.ml;
  P.tab.assign((size_t)G * (mt + 2 * ml + (cubic ? 2 * ml : 0)), 0u);
  P.tabf.assign((size_t)G * (3 * mt + ml + (cubic ? 3 * mt : 0)), 0.0);
  uint32_t *jab = P.tab.data();
  uint32_t *rga = jab + (size_t)G * mt;
  uint32_t *rgb = rga + (size_t)G * ml;
  uint32_t *rgc = rgb + (size_t)G * ml;   // cubic only
  uint32_t *rgd = rgc + (size_t)G * ml;
  double *wi = P.tabf.data();
  double *wbu = wi + (size_t)G * mt;
  double *wbz = wbu + (size_t)G * mt;
  double *sm = wbz + (size_t)G * ml;
  double *wc = sm + (size_t)G * mt;       // cubic only: weights 1..3 of each t-half point
  P.ja.assign(Nt + 1, 1);
  P.jb.assign(Nt + 1, 1);
  P.w.assign(Nt + 1, 0.0);
  // cubic: base l-half point b of each t-half point (its four taps sit at
  // b .. b+3) and their weights, half points past an end folded onto their
  // mirror images (p_0 = p_1, p_{-1} = p_2, ...), as the scheme reads it
  std::vector<int> base(Nt + 1, 1);
  std::vector<double> cw((size_t)4 * (Nt + 1), 0.0);
  for (int lane = 0; lane < G; ++lane)
    for (int r = 0; r < mt; ++r) {
      const int i = lane * mt + r + 1;   // half point i / node i
      uint32_t a = 1, b = 1;
      double w = 0.0;
      if (i <= Nt && Nl > 0) {
        // I_(l)->(t): half point (i-1/2) h_t in units of l-half points:
        // xi = ((2i-1) Nl + Nt) / (2 Nt), linear weights, ends held constant
        const long long num = (long long)(2 * i - 1) * Nl + Nt, den = 2LL * Nt;
        const int j0 = (int)(num / den);
        w = (double)(num % den) / (double)den;
        a = (uint32_t)std::min(std::max(j0, 1), Nl);
        b = (uint32_t)std::min(std::max(j0 + 1, 1), Nl);
        P.ja[i] = (int)a;
        P.jb[i] = (int)b;
        P.w[i] = w;
        if (cubic) {
          const double t = w;
          const double lw[4] = {-t * (t - 1.0) * (t - 2.0) / 6.0, (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
                                -(t + 1.0) * t * (t - 2.0) / 2.0, (t + 1.0) * t * (t - 1.0) / 6.0};
          const int bb = std::min(std::max(j0 - 1, 1), Nl - 3);
          base[i] = bb;
          for (int k = 0; k < 4; ++k) {
            int j = j0 - 1 + k;
            if (j < 1) j = 1 - j;
            if (j > Nl) j = 2 * Nl + 1 - j;
            cw[(size_t)4 * i + (j - bb)] += lw[k];
          }
        }
      }
      if (cubic) {
        jab[(size_t)r * G + lane] = (uint32_t)base[std::min(i, Nt)] | ((uint32_t)base[std::min(i, Nt)] << 16);
        wi[(size_t)r * G + lane] = i <= Nt ? cw[(size_t)4 * i] : 0.0;
        for (int k = 1; k < 4; ++k) wc[(size_t)(k - 1) * G * mt + (size_t)r * G + lane] = i <= Nt ? cw[(size_t)4 * i + k] : 0.0;
      } else {
        jab[(size_t)r * G + lane] = a | (b << 16);
        wi[(size_t)r * G + lane] = w;
      }
      if (i <= Nt - 1) wbu[(size_t)r * G + lane] = wbt[i];
    }
  if (Nl > 0) {
    // ranges of t-half points whose taps land on l-half j: linear, first
    // (second) tap; cubic, tap k of the t-half points with base j - k
    std::vector<int> s0(Nl + 2, 0), n0(Nl + 2, 0), s1(Nl + 2, 0), n1(Nl + 2, 0);
    std::vector<int> sbase(Nl + 2, 0), nbase(Nl + 2, 0);
    for (int i = Nt; i >= 1; --i) {
      s0[P.ja[i]] = i - 1;
      n0[P.ja[i]]++;
      s1[P.jb[i]] = i - 1;
      n1[P.jb[i]]++;
      sbase[base[i]] = i - 1;
      nbase[base[i]]++;
    }
    auto packed = [&](int j, int k) -> uint32_t {   // cubic: t-half points with base j - k
      const int b = j - k;
      return (b >= 1 && b <= Nl) ? ((uint32_t)sbase[b] | ((uint32_t)nbase[b] << 16)) : 0u;
    };
    D.gmax = 0;
    for (int j = 1; j <= Nl; ++j) {
      if (cubic)
        for (int k = 0; k < 4; ++k) D.gmax = std::max(D.gmax, (int)(packed(j, k) >> 16));
      else
        D.gmax = std::max(D.gmax, std::max(n0[j], n1[j]));
    }
    for (int lane = 0; lane < G; ++lane)
      for (int r = 0; r < ml; ++r) {
        const int j = lane * ml + r + 1;
        if (j <= Nl) {
          if (cubic) {
            rga[(size_t)r * G + lane] = packed(j, 0);
            rgb[(size_t)r * G + lane] = packed(j, 1);
            rgc[(size_t)r * G + lane] = packed(j, 2);
            rgd[(size_t)r * G + lane] = packed(j, 3);
          } else {
            rga[(size_t)r * G + lane] = (uint32_t)s0[j] | ((uint32_t)n0[j] << 16);
            rgb[(size_t)r * G + lane] = (uint32_t)s1[j] | ((uint32_t)n1[j] << 16);
          }
        }
        if (j <= Nl - 1) wbz[(size_t)r * G + lane] = wbl[j];
      }
  }
  (void)sm;
  return SB_OK;
}

int plan_excitation(const sb_excitation &e, Plan &P, std::string &err) {
  Desc &D = P.desc;
  if (e.type < 0 || e.type > 3) {
    err = "bad excitation type";
    return SB_EINVAL;
  }
  if (e.interp_order != 0 && e.interp_order != 1 && e.interp_order != 3) {
    err = "interp_order must be 0, 1 or 3";
    return SB_EINVAL;
  }
  if (!finite_all({e.x, e.c0, e.v_H, e.M_H, e.K_H, e.alpha_H}) ||
      (e.type == 3 && !finite_all({e.x_end, e.v_B, e.F_B, e.attack, e.fric_a, e.fric_eps}))) {
    err = "non-finite excitation parameter";
    return SB_EINVAL;
  }
  if (e.type != 0 && !(e.x > 0 && e.x < 1)) {
    err = "excitation position must lie in (0,1)";
    return SB_EINVAL;
  }
  if (e.type == 2 && (!(e.M_H > 0) || !(e.K_H > 0) || !(e.alpha_H >= 1) || !(e.rhoA > 0))) {
    err = "hammer needs M_H, K_H, rhoA > 0 and alpha_H >= 1";
    return SB_EINVAL;
  }
  if (e.type == 3 && (!(e.x_end > 0 && e.x_end < 1) || !(e.F_B >= 0) || !(e.attack >= 0) || !(e.fric_a >= 0) ||
                      !(e.fric_eps >= 0 && e.fric_eps <= 1))) {
    err = "bow needs x_end in (0,1), F_B >= 0, attack >= 0, fric_a >= 0 and fric_eps in [0,1]";
    return SB_EINVAL;
  }
  const int Nt = D.Nt, mt = D.mt, ml = D.ml, nt = D.nt;
  const int G = kClassLanes[D.cls];
  D.bow_on = e.type == 3;
  D.bow_cubic = e.type == 3 && e.interp_order == 3;
  D.bx0 = D.bx1 = D.bT = D.bvB = D.bFB = D.bta = D.ba = D.beps = D.bt0 = 0.0;
  if (e.type == 3) {
    D.bx0 = e.x;
    D.bx1 = e.x_end;
    D.bT = (double)D.n_samples / D.fs;
    D.bvB = e.v_B;
    D.bFB = e.F_B;
    D.bta = e.attack;
    D.ba = e.fric_a;
    D.beps = e.fric_eps;
  }
  // the energy may grow under modulation or a bow (forced)
  D.mon_check = (D.mod_type == 0 && e.type != 3) ? 1 : 0;
  D.ham_on = e.type == 2;
  D.hn0 = D.hn1 = 0;
  D.hw0 = D.hw1 = 0.0;
  if (e.type == 2) {
    D.hn2 = D.hn3 = 0;
    D.hw2 = D.hw3 = 0.0;
  }
  D.omega_pow = D.alpha_H = D.Mr = D.IHs = 0.0;
  double *sm = P.tabf.data() + (size_t)G * (2 * mt + ml);
  std::fill(sm, sm + (size_t)G * mt, 0.0);
  if (e.type == 2) {
    if (e.interp_order == 3) {
      int n[4];
      double w[4];
      cubic_interp(e.x, Nt, D.clamped ? 1.0 : -1.0, n, w);
      D.hn0 = n[0];
      D.hn1 = n[1];
      D.hn2 = n[2];
      D.hn3 = n[3];
      D.hw0 = w[0];
      D.hw1 = w[1];
      D.hw2 = w[2];
      D.hw3 = w[3];
    } else {
      point_interp(e.x, Nt, D.hn0, D.hn1, D.hw0, D.hw1);
    }
    D.omega_pow = e.K_H / e.M_H;       // omega_H^{1 + alpha_H}
    D.alpha_H = e.alpha_H;
    D.Mr = e.M_H / e.rhoA;             // mass ratio for a string of length 1
    // s = T_u0^{-1} J_H, J_H = I_H^T / h_t (Thomas algorithm, FP64)
    const double th = D.theta;
    const double d = th + D.s0k_t + 2.0 * D.s1k_t, c = 0.5 * (1.0 - th) - D.s1k_t;
    std::vector<double> rhs(nt + 1, 0.0), cp(nt + 1, 0.0), x(nt + 2, 0.0);
    if (D.hn0) rhs[D.hn0] += D.hw0 * Nt;
    if (D.hn1) rhs[D.hn1] += D.hw1 * Nt;
    if (D.hn2) rhs[D.hn2] += D.hw2 * Nt;
    if (D.hn3) rhs[D.hn3] += D.hw3 * Nt;
    double den = d;
    std::vector<double> dp(nt + 1, 0.0);
    cp[1] = c / d;
    dp[1] = rhs[1] / d;
    for (int i = 2; i <= nt; ++i) {
      den = d - c * cp[i - 1];
      cp[i] = c / den;
      dp[i] = (rhs[i] - c * dp[i - 1]) / den;
    }
    x[nt] = dp[nt];
    for (int i = nt - 1; i >= 1; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    D.IHs = (D.hn0 ? D.hw0 * x[D.hn0] : 0.0) + (D.hn1 ? D.hw1 * x[D.hn1] : 0.0) +
            (D.hn2 ? D.hw2 * x[D.hn2] : 0.0) + (D.hn3 ? D.hw3 * x[D.hn3] : 0.0);
    for (int lane = 0; lane < G; ++lane)
      for (int r = 0; r < mt; ++r) {
        const int i = lane * mt + r + 1;
        if (i <= nt) sm[(size_t)r * G + lane] = x[i];
      }
  }
  return SB_OK;
}

// Initial state (Sec. 3.3): pluck = triangle of peak c0 at x released from
// rest; hammer = string at rest, hammer touching it with velocity v_H.
void initial_state(const sb_excitation &e, const Plan &P, std::vector<double> &u0, double &uH0, double &uH1) {
  const Desc &D = P.desc;
  u0.assign(D.nt + 1, 0.0);
  uH0 = uH1 = 0.0;
  if (e.type == 1) {
    for (int i = 1; i <= D.nt; ++i) {
      const double x = (double)i / D.Nt;
      u0[i] = x <= e.x ? e.c0 * x / e.x : e.c0 * (1.0 - x) / (1.0 - e.x);
    }
  } else if (e.type == 2) {
    uH1 = D.k * e.v_H;
  }
}

// Plain path (eq. (7) solved as one banded system): the unknowns of both
// grids and the hammer are merged by position along the string, which makes
// every coupling local; the half bandwidth follows from the couplings of
// eq. (8) with the interpolants of the scheme and the hammer's rank-one block.
int plan_plain(Plan &P, std::string &err) {
  Desc &D = P.desc;
  const int Nt = D.Nt, Nl = D.Nl, nt = D.nt, nl = D.nl;
  const bool ham = D.ham_on != 0;
  if (ham && (D.hn2 || D.hn3)) {
    err = "the plain path takes the hammer's linear interpolant only";
    return SB_EINVAL;
  }
  if (D.bow_cubic) {
    err = "the plain path takes the bow's linear interpolant only";
    return SB_EINVAL;
  }
  if (D.grid_interp == 3) {
    err = "the plain path takes the linear grid interpolant only";
    return SB_EINVAL;
  }
  struct Item {
    double x;
    int kind, idx;
  };
  std::vector<Item> it;
  for (int i = 1; i <= nt; ++i) it.push_back({(double)i / Nt, 0, i});
  for (int j = 1; j <= nl; ++j) it.push_back({(double)j / Nl, 1, j});
  // the hammer unknown sits at the position of its first node
  if (ham) it.push_back({D.hn0 ? (double)D.hn0 / Nt : (double)D.hn1 / Nt, 2, 0});
  std::stable_sort(it.begin(), it.end(), [](const Item &a, const Item &b) {
    return a.x < b.x || (a.x == b.x && a.kind < b.kind);
  });
  std::vector<int> pt(nt + 1, -1), pl(nl + 1, -1);
  int ph = -1;
  for (int r = 0; r < (int)it.size(); ++r) {
    if (it[r].kind == 0) pt[it[r].idx] = r;
    else if (it[r].kind == 1) pl[it[r].idx] = r;
    else ph = r;
  }
  const int n = (int)it.size();
  // l-half ranges of t-half points per tap (1-based first half, count)
  std::vector<int> sa(Nl + 2, 0), na(Nl + 2, 0), sb(Nl + 2, 0), nb(Nl + 2, 0);
  if (nl > 0)
    for (int h = Nt; h >= 1; --h) {
      sa[P.ja[h]] = h;
      na[P.ja[h]]++;
      sb[P.jb[h]] = h;
      nb[P.jb[h]]++;
    }
  int bw = 0;
  auto see = [&](int r, int c) {
    if (r >= 0 && c >= 0) bw = std::max(bw, std::abs(r - c));
  };
  for (int i = 1; i <= nt; ++i) {
    const int r = pt[i];
    if (i > 1) see(r, pt[i - 1]);
    if (i < nt) see(r, pt[i + 1]);
    if (nl > 0)
      for (int h = i; h <= i + 1; ++h) {
        if (h < 1 || h > Nt) continue;
        for (int j : {P.ja[h], P.ja[h] - 1, P.jb[h], P.jb[h] - 1})
          if (j >= 1 && j <= nl) see(r, pl[j]);
      }
    if (ham && (i == D.hn0 || i == D.hn1)) {
      see(r, ph);
      if (D.hn0) see(r, pt[D.hn0]);
      if (D.hn1) see(r, pt[D.hn1]);
    }
  }
  for (int j = 1; j <= nl; ++j) {
    const int r = pl[j];
    if (j > 1) see(r, pl[j - 1]);
    if (j < nl) see(r, pl[j + 1]);
    for (int m = j; m <= j + 1; ++m) {
      for (int h = sa[m]; h < sa[m] + na[m]; ++h)
        for (int i : {h - 1, h})
          if (i >= 1 && i <= nt) see(r, pt[i]);
      for (int h = sb[m]; h < sb[m] + nb[m]; ++h)
        for (int i : {h - 1, h})
          if (i >= 1 && i <= nt) see(r, pt[i]);
    }
  }
  if (ham) {
    if (D.hn0) see(ph, pt[D.hn0]);
    if (D.hn1) see(ph, pt[D.hn1]);
  }
  D.pn = n;
  D.pbw = bw;
  D.ph = ph;
  if (bw > kPlainMaxBw) {
    err = "plain path: half bandwidth " + std::to_string(bw) + " exceeds " + std::to_string(kPlainMaxBw);
    return SB_EBUDGET;
  }
  if (plain_lds_bytes(D) > (size_t)kPlainMaxLdsBytes) {
    err = "plain path: banded system does not fit in LDS";
    return SB_EBUDGET;
  }
  P.ptab.assign((size_t)nt + nl + Nt + 2 * (size_t)Nl, 0);
  int32_t *q = P.ptab.data();
  for (int i = 1; i <= nt; ++i) *q++ = pt[i];
  for (int j = 1; j <= nl; ++j) *q++ = pl[j];
  for (int h = 1; h <= Nt; ++h) *q++ = nl > 0 ? (P.ja[h] | (P.jb[h] << 16)) : 0;
  for (int m = 1; m <= Nl; ++m) *q++ = sa[m] | (na[m] << 16);
  for (int m = 1; m <= Nl; ++m) *q++ = sb[m] | (nb[m] << 16);
  P.pw.assign(Nt, 0.0);
  for (int h = 1; h <= Nt; ++h) P.pw[h - 1] = nl > 0 ? P.w[h] : 0.0;
  return SB_OK;
}

// LDS of the plain kernel: band (2 bw + 1 per row) and right-hand side of the
// n unknowns, the two time levels of both grids with their end points, and
// per-step half-point and node scratch.
size_t plain_lds_bytes(const Desc &D) {
  const size_t n = (size_t)D.pn, W = 2 * (size_t)D.pbw + 1;
  const size_t words = n * W + n + 1 + W + 2 * ((size_t)D.Nt + 1) + 2 * ((size_t)D.Nl + 1) + 4 * ((size_t)D.Nt + 2) +
                       2 * ((size_t)D.Nl + 2) + (D.bow_on ? n + 1 : 0) + 64;
  return words * sizeof(double);
}

}  // namespace sfd

extern "C" int string_plan_grid(const sb_string_params *p, int32_t *N_t, int32_t *N_l) {
  if (!p) return SB_EINVAL;
  sfd::GridPlan g;
  std::string err;
  int st = sfd::plan_grid(*p, g, err);
  if (st) return st;
  if (N_t) *N_t = g.Nt;
  if (N_l) *N_l = g.Nl;
  return SB_OK;
}
