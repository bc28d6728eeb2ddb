// Bow of eq. (5): controls, the interpolant at the bow and the step's scalar
// stick/slip problem, shared by the batched kernels and the plain FP64
// kernel (device code of libstringfdtd, private to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfd {

// Per-group bow record in LDS (doubles): the controls (set at the start of a
// task), then the step's values that the bow's correction after the solve
// reads.  Kept out of registers through the sweeps.
constexpr int kBowX0 = 0, kBowX1 = 1, kBowT = 2, kBowVB = 3, kBowFB = 4, kBowTa = 5, kBowA = 6, kBowEps = 7;
constexpr int kBowStepVB = 8, kBowStepK2F = 9, kBowStepIv = 10, kBowStepW0 = 11, kBowStepW1 = 12, kBowStepN0 = 13,
              kBowStepN1 = 14, kBowT0 = 15;
// the cubic I_p's two further nodes and weights (zero for the linear one)
constexpr int kBowStepW2 = 16, kBowStepW3 = 17, kBowStepN2 = 18, kBowStepN3 = 19;
constexpr int kBowRec = 20;

// Bow of eq. (5).  Controls at time t from the record: kBowX0 the start
// position, kBowX1 its rate of change (zero when it stays) until kBowT
// seconds after the bow was set (kBowT0), kBowTa the rate at which force and
// bow speed ramp up to kBowFB and kBowVB (zero: no attack).
__device__ __forceinline__ void bow_controls(const double *R, double t, double &x, double &vB, double &FB) {
  const double s = t - R[kBowT0];
  const double ramp = R[kBowTa] > 0.0 ? fmin(s * R[kBowTa], 1.0) : 1.0;
  x = fma(R[kBowX1], fmin(s, R[kBowT]), R[kBowX0]);
  vB = R[kBowVB] * ramp;
  FB = R[kBowFB] * ramp;
}

// Record entries kBowX1 and kBowTa from a descriptor's end position x1 after
// T seconds and attack time ta.
__device__ __forceinline__ double bow_x_rate(double x0, double x1, double T) { return T > 0.0 ? (x1 - x0) / T : 0.0; }
__device__ __forceinline__ double bow_ramp_rate(double ta) { return ta > 0.0 ? 1.0 / ta : 0.0; }

// Nodes (1-based, 0 = absent) and weights of the linear interpolant at x.
__device__ __forceinline__ void bow_interp(double x, int N, int &n0, int &n1, double &w0, double &w1) {
  const int l = (int)floor(x * N);
  const double w = x * N - l;
  n0 = (l >= 1 && l <= N - 1) ? l : 0;
  n1 = (l + 1 >= 1 && l + 1 <= N - 1) ? l + 1 : 0;
  w0 = n0 ? 1.0 - w : 0.0;
  w1 = n1 ? w : 0.0;
}

// The step's scalar problem v_rel = b - c phi (c >= 0): stick (v_rel = 0,
// phi = b/c) when |b| <= c, else slip at the root x in (0, |b|) of
// x + c (eps + (1-eps) e^{-a x}) = |b| (convex left side, below |b| at 0):
// Newton's method inside a shrinking bracket.  Every lane of the wavefront
// takes part; the loop ends when all have converged.  Returns phi.
__device__ __forceinline__ double bow_phi(double b, double c, double a, double eps) {
  const bool slip = c > 0.0 && fabs(b) > c;
  const double ab = fabs(b), sg = b > 0.0 ? 1.0 : -1.0;
  double lo = 0.0, hi = ab, x = ab;
  bool done = !slip;
  for (int it = 0; it < 100; ++it) {
    if (__ballot(!done) == 0) break;
    const double ex = exp(-a * x);
    const double h = x + c * (eps + (1.0 - eps) * ex) - ab;
    hi = (!done && h > 0.0) ? x : hi;
    lo = (!done && h < 0.0) ? x : lo;
    const double dh = 1.0 - c * (1.0 - eps) * a * ex;
    double xn = dh > 0.0 ? x - h / dh : 0.5 * (lo + hi);
    xn = (xn > lo && xn < hi) ? xn : 0.5 * (lo + hi);
    const bool fin = h == 0.0 || fabs(xn - x) <= 4e-16 * ab || hi - lo <= 4e-16 * ab;
    x = (done || h == 0.0) ? x : xn;
    done = done || fin;
  }
  if (!(c > 0.0)) return 0.0;
  if (!slip) return b / c;
  return sg * (eps + (1.0 - eps) * exp(-a * x));
}

}  // namespace sfd
