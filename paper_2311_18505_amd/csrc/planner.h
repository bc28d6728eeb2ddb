// Host planner of libstringfdtd (private header).
#pragma once
#include <string>
#include <vector>

#include "../../include/stringfdtd.h"
#include "sfd_types.h"

namespace sfd {

struct GridPlan {
  int Nt = 0, Nl = 0;
  double k = 0, theta = 0, gamma0 = 0, gamma_max = 0, kappa = 0;
};

// Everything the kernel needs for one string, in FP64.
struct Plan {
  GridPlan grid;
  Desc desc{};
  std::vector<uint32_t> tab;     // lane-major integer tables
  std::vector<double> tabf;      // lane-major real tables (rounded to the kernel precision on upload)
  std::vector<int> ja, jb;       // I_(l)->(t) taps per t-half point (1-based)
  std::vector<double> w;
  std::vector<int32_t> ptab;     // plain path tables (natural order), see Desc::ptab
  std::vector<double> pw;
};

double theta_of(const sb_string_params &p);
int plan_grid(const sb_string_params &p, GridPlan &g, std::string &err);
// shapes: lay each grid out with the fewest slots per lane of its class's
// width levels (MM, 3MM/4, MM/2) that it fits in (the FP32 kernels step those
// layouts)
int plan_string(const sb_string_params &p, Plan &P, std::string &err, bool shapes = false);
int plan_excitation(const sb_excitation &e, Plan &P, std::string &err);
void initial_state(const sb_excitation &e, const Plan &P, std::vector<double> &u0, double &uH0, double &uH1);
int plan_plain(Plan &P, std::string &err);
size_t plain_lds_bytes(const Desc &D);

}  // namespace sfd
