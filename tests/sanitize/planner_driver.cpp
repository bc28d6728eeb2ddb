// The library's host planner (grid sizing, coefficient tables, excitation
// tables, the plain path's position tables) under AddressSanitizer and
// UndefinedBehaviorSanitizer: a seeded sweep of valid and invalid string
// parameters and excitations goes through every planning entry point, and
// one summary line is printed.  Built and run by tests/test_sanitizers.py.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <string>
#include <vector>

#include "planner.h"

namespace {

uint64_t g_state = 0x2311185055ull;

double urand() {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

double loguni(double lo, double hi) { return lo * std::exp(std::log(hi / lo) * urand()); }

sb_string_params draw_string(int i) {
  sb_string_params p{};
  p.fs = 48000.0;
  p.f0 = loguni(15.0, 2000.0);
  p.B = urand() < 0.1 ? 0.0 : loguni(1e-8, 2e-2);
  p.alpha = urand() < 0.2 ? 1.0 : 1.0 + 3.0 * urand();
  p.theta = urand() < 0.8 ? 0.0 : 0.501 + 0.499 * urand();
  p.sigma0_t = loguni(0.05, 3.0);
  p.sigma1_t = loguni(1e-5, 1e-3);
  p.sigma0_l = loguni(0.05, 3.0);
  p.sigma1_l = loguni(1e-5, 1e-3);
  p.x_out = 0.01 + 0.98 * urand();
  p.n_samples = 2 + (int64_t)(urand() * 2000.0);
  p.mod_type = i % 3;
  p.mod_depth_cents = 30.0 * urand();
  p.mod_rate_hz = 8.0 * urand();
  p.glide_semitones = 6.0 * urand() - 3.0;
  p.boundary = i % 5 == 0 ? 1 : 0;
  p.readout_zeta = i % 7 == 0 ? 1 : 0;
  p.grid_interp = i % 4 == 1 ? 3 : (i % 4 == 2 ? 1 : 0);
  if (i % 11 == 3) p.grid_t = 4 + (int)(urand() * 60.0);
  if (i % 13 == 4) p.grid_l = 2 + (int)(urand() * 60.0);
  // invalid draws: every entry point must refuse them without touching memory
  const double nan = std::numeric_limits<double>::quiet_NaN();
  switch (i % 17) {
    case 5: p.f0 = nan; break;
    case 6: p.alpha = 0.5; break;
    case 7: p.x_out = 1.0; break;
    case 8: p.theta = 0.4; break;
    case 9: p.B = -1e-4; break;
    case 10: p.sigma1_l = std::numeric_limits<double>::infinity(); break;
    case 11: p.n_samples = 1; break;
    case 12: p.grid_interp = 2; break;
    default: break;
  }
  return p;
}

sb_excitation draw_excitation(int i) {
  sb_excitation e{};
  e.type = 1 + i % 3;
  e.interp_order = (i / 3) % 2 ? 3 : 1;
  // positions near the ends exercise the mirrored nodes of the cubic rows
  const double xs[] = {0.003, 0.02, 0.5 * urand() + 0.1, 0.97, 0.999};
  e.x = xs[i % 5];
  e.c0 = 1e-3;
  e.v_H = 0.5 + 3.0 * urand();
  e.M_H = 4.9e-3;
  e.K_H = 4.5e9;
  e.alpha_H = 2.5;
  e.rhoA = 6.3e-3;
  e.x_end = 0.05 + 0.9 * urand();
  e.v_B = 0.05 + 0.2 * urand();
  e.F_B = 100.0 * urand();
  e.attack = 0.02;
  e.fric_a = 100.0;
  e.fric_eps = 0.2;
  if (i % 19 == 7) e.x = 0.0;                                   // invalid
  if (i % 23 == 9) e.type = 7;                                  // invalid
  if (i % 29 == 11) e.fric_eps = 1.5;                           // invalid
  return e;
}

}  // namespace

int main(int argc, char **argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 600;
  int ok = 0, refused = 0, budget = 0, exc_ok = 0, exc_refused = 0, plain_ok = 0, plain_refused = 0, shaped = 0;
  double checksum = 0.0;
  for (int i = 0; i < n; ++i) {
    const sb_string_params p = draw_string(i);
    int32_t nt = -1, nl = -1;
    const int gst = string_plan_grid(&p, &nt, &nl);
    sfd::Plan P;
    std::string err;
    // every other string is planned for an FP32 batch, with the narrow layouts
    const bool shapes = i % 2 == 1;
    const int st = sfd::plan_string(p, P, err, shapes);
    // string_plan_grid sizes the grid only; the per-string budget is the planner's
    if ((st == SB_EINVAL) != (gst == SB_EINVAL)) {
      std::printf("MISMATCH string %d: plan_string %d, string_plan_grid %d (%s)\n", i, st, gst, err.c_str());
      return 2;
    }
    if (st == SB_EBUDGET) {
      ++budget;
      continue;
    }
    if (st != SB_OK) {
      ++refused;
      continue;
    }
    ++ok;
    checksum += nt + nl;
    {
      // the layout: each grid on MM, an intermediate count (3 of 4, 6 of 8,
      // 4 of 6 slots) or MM/2 slots per lane, covering its points, the fewest
      // in total, its wider grid beyond what the next smaller class holds and
      // not both at MM/2; MM on both grids without shapes
      const sfd::Desc &D = P.desc;
      const int G = sfd::kClassLanes[D.cls], mm = sfd::kClassSlots[D.cls];
      std::vector<int> levels = {mm, mm / 2};
      if (mm == 4) levels.push_back(3);
      if (mm == 8) levels.push_back(6);
      if (mm == 6) levels.push_back(4);
      const int below = D.cls > 0 ? sfd::kClassLanes[D.cls - 1] * sfd::kClassSlots[D.cls - 1] : 0;
      int best = 1 << 30;
      for (int mt : levels)
        for (int ml : levels) {
          if (mt == mm / 2 && ml == mm / 2) continue;
          if (G * (mt > ml ? mt : ml) <= below) continue;
          if (D.Nt <= G * mt && D.Nl <= G * ml && mt + ml < best) best = mt + ml;
        }
      const bool cover = D.Nt <= G * D.mt && D.Nl <= G * D.ml;
      if (!cover || (shapes ? D.mt + D.ml != best : (D.mt != mm || D.ml != mm))) {
        std::printf("LAYOUT string %d: class %d Nt %d Nl %d -> mt %d ml %d (fewest %d)\n", i, D.cls, D.Nt, D.Nl,
                    D.mt, D.ml, best);
        return 3;
      }
      shaped += (D.mt + D.ml < 2 * mm) ? 1 : 0;
    }
    for (double v : P.tabf) checksum += std::isfinite(v) ? 1e-9 * v : 0.0;
    for (int k = 0; k < 2; ++k) {
      sfd::Plan Q = P;
      const sb_excitation e = draw_excitation(3 * i + k);
      std::string e_err;
      if (sfd::plan_excitation(e, Q, e_err) != SB_OK) {
        ++exc_refused;
        continue;
      }
      ++exc_ok;
      std::vector<double> u0;
      double uH0 = 0.0, uH1 = 0.0;
      sfd::initial_state(e, Q, u0, uH0, uH1);
      for (double v : u0) checksum += 1e-3 * v;
      checksum += uH0 + uH1;
      sfd::Plan R = Q;
      std::string p_err;
      if (sfd::plan_plain(R, p_err) == SB_OK) {
        ++plain_ok;
        checksum += (double)sfd::plain_lds_bytes(R.desc) * 1e-9;
      } else {
        ++plain_refused;
      }
    }
  }
  std::printf("strings %d ok %d refused %d budget %d excitations ok %d refused %d plain ok %d refused %d "
              "narrow layouts %d checksum %.6e\n",
              n, ok, refused, budget, exc_ok, exc_refused, plain_ok, plain_refused, shaped, checksum);
  return 0;
}
