// Internal types shared by the host planner, the C ABI and the HIP kernels of
// libstringfdtd (private to the library).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace sfd {

constexpr int kWave = 64;          // lanes per wavefront on CDNA4
constexpr int kMaxSlots = 16;      // grid points per lane per grid
constexpr int kMaxN = kWave * kMaxSlots;   // N_t, N_l <= 1024

// Size classes of the stepping kernel.  A string occupies a group of G lanes
// (a wavefront holds 64/G strings) and every lane owns up to MM consecutive
// points of each grid; a string runs in the smallest class with
// G * MM >= max(N_t, N_l).
constexpr int kNumClasses = 8;
constexpr int kClassLanes[kNumClasses] = {16, 16, 32, 64, 64, 64, 64, 64};
constexpr int kClassSlots[kNumClasses] = {2, 4, 4, 4, 6, 8, 10, 16};
constexpr int class_points(int c) { return kClassLanes[c] * kClassSlots[c]; }
// the class of G lanes and MM slots per lane (-1 if none)
constexpr int class_of(int G, int MM) {
  for (int c = 0; c < kNumClasses; ++c)
    if (kClassLanes[c] == G && kClassSlots[c] == MM) return c;
  return -1;
}

// Launches of one step.  The classes up to 384 points share one occupancy
// profile (two wavefronts per SIMD) and run as one persistent launch with one
// work queue (unit 0); class 5 runs as a launch of its own (unit 1) and
// classes 6 and 7 one after the other on a third stream (unit 2; no string of
// the benchmark workloads needs class 7), so the three units run
// concurrently.
constexpr int kNumSmall = 5;        // classes 0..4
constexpr int kNumUnits = 3;
constexpr int unit_of_class(int c) { return c < kNumSmall ? 0 : (c == kNumSmall ? 1 : 2); }
// kernel of a class: 0 the merged classes, then one per large class
constexpr int kernel_of_class(int c) { return c < kNumSmall ? 0 : c - kNumSmall + 1; }
constexpr int kNumKernels = kNumClasses - kNumSmall + 1;

// Kernel instantiations by the code a string needs: plain (plucks and
// two-node hammers), the bow family (bowed strings, clamped ends, the zeta
// channel, cubic hammers) and the bow family with the cubic grid
// interpolant.  Each carries only its own code, so a task pays only for the
// registers of what its strings use.
enum : int { kVarPlain = 0, kVarBow = 1, kVarCubic = 2, kNumVariants = 3 };

// Layouts ("shapes") of a string in its class: each grid gets MM, an
// intermediate count or MM/2 slots per lane (width levels 0, 1, 2), the
// fewest its points fit in; shape = 3 * (transverse level) + (longitudinal
// level).  The stepping loops run over a grid's slots, so a narrower grid
// does proportionally less work.  Level 1 is 3MM/4 in the classes of 4 and 8
// slots and 4 in the class of 6; the others have none.  A shape is kept only
// where its wider grid needs more points than the next smaller class holds
// (otherwise the string would be in that class; this also drops both grids
// at MM/2, shape 8).  FP32 batches; FP64 batches use shape 0.
constexpr int kNumShapes = 9;
constexpr int level1_slots(int mm) { return mm == 4 || mm == 8 ? 3 * mm / 4 : (mm == 6 ? 4 : 0); }
constexpr int level_slots(int mm, int level) { return level == 0 ? mm : level == 1 ? level1_slots(mm) : mm / 2; }
constexpr int shape_mt(int c, int s) { return level_slots(kClassSlots[c], s / 3); }
constexpr int shape_ml(int c, int s) { return level_slots(kClassSlots[c], s % 3); }
constexpr bool shape_ok(int c, int s) {
  if (c < 0 || c >= kNumClasses || s < 0 || s >= kNumShapes || s == 8) return false;
  const int mt = shape_mt(c, s), ml = shape_ml(c, s);
  if (mt == 0 || ml == 0) return false;
  const int wide = mt > ml ? mt : ml;
  return c == 0 || kClassLanes[c] * wide > class_points(c - 1);
}
// work lists are kept per part = class * kNumShapes + shape
constexpr int kNumParts = kNumClasses * kNumShapes;

enum : int32_t {
  kFlagUnstable = 1,      // energy monitor: non-finite or growing energy
  kFlagNoConverge = 2,    // coupled solve did not converge within the sweep cap
};

// Per-string plan, computed once on the host in FP64 and uploaded.  All
// offsets are in elements of the respective arena.
struct Desc {
  int32_t Nt, Nl;             // intervals of the transverse / longitudinal grids (Nl = 0: no zeta)
  int32_t nt, nl;             // unknowns: Nt-1, Nl-1 (0)
  int32_t mt, ml;             // slots per lane of each grid (from the shape; FP64: the class's MM)
  int32_t cls;                // size class index
  int32_t shape;              // layout in the class (kNumShapes): mt, ml follow from it
  int32_t shape_pad;
  int32_t mon_check;          // 1: energy must not grow (unforced, constant f0)
  int64_t n_samples;          // samples to produce
  void *st;                   // state block, kernel precision, lane-major [array][slot][lane]
  void *out;                  // output samples, kernel precision
  const uint32_t *tab;        // integer tables: ja|jb<<16 per t-slot, sa|na<<16 and sb|nb<<16 per l-slot
  const void *tabf;           // real tables (kernel precision): w per t-slot, boundary weights, SM vector
  double k;                   // time step
  double Ntd, Nld;            // 1/h_t, 1/h_l
  double theta;
  double g2k2_0;              // (gamma0 k)^2
  double a2;                  // alpha^2
  double a2m1_4;              // (alpha^2 - 1) / 4
  double cS;                  // kappa^2 k^2 Nt^2
  double s0k_t, s1k_t;        // sigma0_t k, sigma1_t k Nt^2
  double s0k_l, s1k_l;        // sigma0_l k, sigma1_l k Nl^2
  double ratio_lt;            // h_t / h_l = Nl / Nt
  double rho_t, itk_t;        // Toeplitz factor of T_u0: rho, 1/kappa_T
  double rho_l, itk_l;        // same for T_z
  // f0 modulation
  int32_t mod_type;           // 0 none, 1 vibrato, 2 glide
  int32_t clamped;            // 1: clamped transverse ends (mirrored ghost nodes in D_xxxx)
  double f0, fs, mod_a, mod_b;   // vibrato: a = depth/1200, b = rate; glide: a = semis/12, b = 1/T
  // hammer
  int32_t ham_on;             // 1 if the excitation is a hammer
  int32_t hn0, hn1;           // nodes of I_H (1-based; 0 = absent)
  int32_t zeta_out;           // 1: the string also records zeta at x_out (batched paths)
  double hw0, hw1;            // weights of I_H
  double omega_pow, alpha_H, Mr, IHs;   // K_H/M_H, exponent, M_H/(rho A), I_H T_u0^{-1} J_H
  // bow (eq. 5), set on the string at time bt0: position bx0 -> bx1 over bT
  // seconds, bow speed and force rising over bta seconds, friction curve
  // sign(v) (beps + (1-beps) e^{-ba|v|})
  int32_t bow_on;             // 1 if the excitation is a bow
  int32_t zon0;               // zeta channel: first l-grid node of I(x_out) (0 = absent)
  int32_t bow_cubic;          // 1: the bow's I_p is the cubic interpolant (four nodes)
  int32_t grid_interp;        // order of I_(l)->(t): 1 linear, 3 cubic (extra tables, see the planner)
  union {
    struct {
      double bx0, bx1, bT, bvB, bFB, bta, ba, beps, bt0;
    };
    // a hammer's cubic interpolant (p = 3) has two more nodes and weights
    // (0 = absent); a string has either a hammer or a bow, never both
    struct {
      int32_t hn2, hn3;
      double hw2, hw3;
    };
  };
  // readout
  int32_t on0, on1;           // nodes of I(x_out)
  double ow0, ow1;
  int32_t gmax;               // longest t-half range gathered by one l-half point
  int32_t st_elems;           // elements of the state block
  void *st0;                  // copy of the state block right after excitation
  // plain FP64 path (eq. (7), merged-order banded LU): unknowns, half
  // bandwidth, position of the hammer unknown (-1: none), and its tables
  int32_t pn, pbw, ph;
  int32_t zon1;               // zeta channel: second l-grid node of I(x_out) (0 = absent)
  // the plain path's tables, or (batched paths, which never read them) the
  // zeta channel's output and interpolation weight: zon0 takes 1 - zw, zon1 zw
  union {
    const int32_t *ptab;      // pos_t[nt] | pos_l[nl] | ja|jb<<16 per t-half [Nt] | sa|na<<16, sb|nb<<16 per l-half [Nl] each
    void *out_z;              // zeta samples, kernel precision (null without the channel)
  };
  union {
    const double *pw;         // interpolation weight w per t-half [Nt]
    double zw;
  };
};

constexpr int kPlainMaxBw = 16;             // half bandwidth the plain kernel accepts
constexpr int kPlainMaxLdsBytes = 64 * 1024;    // LDS the plain kernel may use (no opt-in needed)

// Per-string dynamic status (device memory, updated by the kernel).
struct Status {
  int64_t samples_done;       // samples y^0..y^{samples_done-1} are valid
  int32_t flags;              // kFlag*
  int32_t max_sweeps;         // largest number of solver sweeps taken in one step
  int64_t total_sweeps;       // sum of sweeps (for statistics)
  double H_latest;            // energy H^{n+1/2} of the last monitor check
  int64_t H_step;             // n of that check (-1: none)
  double H_ref;               // reference for the growth check
  int32_t touched;            // hammer in contact since the last check
  int32_t pad0;
  double uH_n, uH_nm1, eta_nm1;  // hammer lumped state (FP64)
};

// Arguments of one launch of the stepping kernel.
struct LaunchArgs {
  const Desc *desc;
  Status *status;
  const int32_t *work;        // 64/G string indices per wavefront task (-1: empty group)
  int32_t n_work;             // number of wavefront tasks (tickets)
  // ticket w runs task tickets[w] & 0xffffff of part tickets[w] >> 24,
  // whose tasks are listed at part_work[part] (the merged launch: the parts
  // of classes 0..4; a large class: its shapes)
  const int32_t *part_work[kNumSmall * kNumShapes];
  const int32_t *tickets;
  int32_t *counter;           // work-queue head (zeroed before the launch)
  int64_t n_steps;            // steps to advance each string (clamped at n_samples)
  int32_t mon_period;         // steps between energy checks (0: off)
  int32_t max_sweeps;         // cap of solver sweeps per step
  double tol;                 // relative convergence tolerance of the coupled solve
  double mon_tol;             // relative growth tolerance of the energy check
  void *trash_st;             // write target of empty groups (kMaxTrash bytes)
  Status *trash_status;
};

constexpr int kMaxTrash = 4 * 2 * kMaxSlots * kWave * 8;   // largest state block in FP64

// Fixed device scratch of the allocation-free gather: per row a slot index,
// an offset, and the slot's progress and flags, for at most kNoAllocMaxRows
// rows (each region starts on a 256-byte boundary).
constexpr int kNoAllocMaxRows = 16384;
constexpr size_t kScratchSlotsOff = 0;
constexpr size_t kScratchOffsOff = kScratchSlotsOff + ((sizeof(int32_t) * kNoAllocMaxRows + 255) & ~size_t(255));
constexpr size_t kScratchDoneOff = kScratchOffsOff + ((sizeof(int64_t) * kNoAllocMaxRows + 255) & ~size_t(255));
constexpr size_t kScratchFlagsOff = kScratchDoneOff + ((sizeof(int64_t) * kNoAllocMaxRows + 255) & ~size_t(255));
constexpr size_t kStaticScratchBytes = kScratchFlagsOff + ((sizeof(int32_t) * kNoAllocMaxRows + 255) & ~size_t(255));

// One segment of a bulk upload (excitation): bytes (a multiple of 4) from
// offset src_off of the staging buffer to dst.
struct UploadSeg {
  uint64_t src_off;
  void *dst;
  uint64_t bytes;
};

}  // namespace sfd
