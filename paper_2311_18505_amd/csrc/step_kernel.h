// Batched stepping kernels of libstringfdtd for gfx950 (device code; each
// instantiation family is compiled by a translation unit of its own).
//
// A wavefront steps 64/G strings at once: each string owns a group of G
// lanes, and lane l of a group holds the transverse points l*mt+1 .. l*mt+mt
// and the longitudinal points l*ml+1 .. l*ml+ml of its string in registers
// for a whole launch.  Neighbours come from the adjacent lanes through DPP
// moves, the two grids exchange interpolated values through LDS, and every
// loop has a wave-uniform trip count with per-group differences expressed as
// selects (writes that a group must not make go to a trash slot), so the
// control flow of the persistent loop never diverges.
//
// The scheme is eq. (7) of the paper written for the acceleration
// a = w^{n+1} - 2 w^n + w^{n-1}:
//     (A^n + beta J I) a = -(A^n + B^n + C^n) w^n - (A^n - C^n) v + 2 beta J eta^n,
// v = w^n - w^{n-1}; its right-hand side is O(k^2 force) (the O(1) Theta
// terms cancel), which is what makes FP32 stepping accurate.  The system is
// solved by block Gauss-Seidel between the two grids around the constant
// Toeplitz blocks T_u0 = Theta + sigma0 k - sigma1 k D_xx and
// T_z = (1 + sigma0 k) - sigma1 k D_xx, each inverted exactly through its
// factorisation kT (1 + rho S-)(1 + rho S+) on the odd periodic extension of
// the fixed-end grid (two first-order recurrences per lane plus group scans);
// the hammer's rank-one term is removed exactly by Sherman-Morrison.
#pragma once
#include <hip/hip_runtime.h>

#include "sfd_types.h"
#include "bow.h"
#include "interp.h"

namespace sfd {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// ---------------------------------------------------------------------------
// Wave-uniform values and cross-lane moves
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint64_t b = (uint64_t)x;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// DPP move of a 32-bit value; lanes whose source lies outside the row / wave read 0.
template <int CTRL>
__device__ __forceinline__ int dpp32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __builtin_bit_cast(float, dpp32<CTRL>(__builtin_bit_cast(int, x)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)dpp32<CTRL>((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)dpp32<CTRL>((int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// DPP move restricted to the rows of ROWS (bit r: row r of 16 lanes); the
// other rows read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// value of lane l (a constant) for every lane
__device__ __forceinline__ float lane_read(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ double lane_read(double x, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl4 = 0x104, kRowShl8 = 0x108;
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kWaveShl1 = 0x130, kWaveShr1 = 0x138;
// lane 15 of each row to the next row; lane 31 to rows 2 and 3; lane 15 of
// each row to its own row
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kRowNewBcast0 = 0x150, kRowNewBcast15 = 0x15F;

// Each odd row's values in both rows of its pair (rows 0 and 1 read row 1,
// rows 2 and 3 read row 3): the second result of v_permlane16_swap with both
// operands x.
__device__ __forceinline__ float odd_rows(float x) {
  const unsigned b = __builtin_bit_cast(unsigned, x);
  return __builtin_bit_cast(float, (unsigned)__builtin_amdgcn_permlane16_swap(b, b, false, false)[1]);
}
__device__ __forceinline__ double odd_rows(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const unsigned nlo = __builtin_amdgcn_permlane16_swap(lo, lo, false, false)[1];
  const unsigned nhi = __builtin_amdgcn_permlane16_swap(hi, hi, false, false)[1];
  return __builtin_bit_cast(double, ((uint64_t)nhi << 32) | nlo);
}

// value of the previous / next lane of the same group (0 at the group edge;
// a group of 64 lanes has its edges at the wave's, where the move reads 0)
template <int G, typename T>
__device__ __forceinline__ T grp_prev(T x) {
  const T v = dpp<kWaveShr1>(x);
  if (G == 64) return v;
  return (lane_id() & (G - 1)) == 0 ? T(0) : v;
}
template <int G, typename T>
__device__ __forceinline__ T grp_next(T x) {
  const T v = dpp<kWaveShl1>(x);
  if (G == 64) return v;
  return (lane_id() & (G - 1)) == G - 1 ? T(0) : v;
}

// Sum (or max, of non-negative inputs) over the lanes of each group, returned
// to every lane of the group, in a fixed association order.
template <int G, bool MAX, typename T>
__device__ __forceinline__ T grp_reduce(T x) {
  auto op = [](T a, T b) { return MAX ? fmax(a, b) : a + b; };
  x = op(x, dpp<kRowShr1>(x));
  x = op(x, dpp<kRowShr2>(x));
  x = op(x, dpp<kRowShr4>(x));
  x = op(x, dpp<kRowShr8>(x));
  // lane 15 of a row now holds the row total
  if (G == 16) return dpp_rows<kRowNewBcast15, 0xf>(x);
  // rows 1 and 3 add the totals of rows 0 and 2: lanes 31 and 63 hold the
  // totals of the two halves (rows 0 and 2 take values no later step reads,
  // so the moves need no row mask)
  x = op(x, dpp<kRowBcast15>(x));
  // (groups of 32: each odd row spreads its lane 15 and lends it to its pair)
  if (G == 32) return odd_rows(dpp<kRowNewBcast15>(x));
  // rows 2 and 3 add the first half's total: lane 63 holds the wave's
  x = op(x, dpp<kRowBcast31>(x));
  return lane_read(x, 63);
}

// Powers of the lane-to-lane carry factor g used by the group scans of G
// lanes.  The cross-row carries move whole rows; a row that must not take a
// carry (one of its own group: a value of another group is never scaled in)
// has the factor 0 there.
template <typename T>
struct ScanPow {
  T g1, g2, g4, g8, g16;
  T gl;   // g^{(lane & 15) + 1} (G = 64: 0 in rows 0 and 2)
  T gl2;  // g^{(lane & 31) + 1} (0 in rows 0 and 1)
  T gr;   // g^{16 - (lane & 15)}, 0 in rows 1 and 3
  T gr2;  // g^{32 - (lane & 31)}, 0 in rows 2 and 3
};

template <typename T>
__device__ __forceinline__ T ipow(T g, int e) {   // 0 <= e <= 31
  T r = T(1), b = g;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    r = (e & (1 << k)) ? r * b : r;
    b = b * b;
  }
  return r;
}

template <int G, typename T>
__device__ __forceinline__ ScanPow<T> scan_pow(T g) {
  ScanPow<T> p;
  p.g1 = g;
  p.g2 = g * g;
  p.g4 = p.g2 * p.g2;
  p.g8 = p.g4 * p.g4;
  p.g16 = p.g8 * p.g8;
  const int j = lane_id() & 15, row = lane_id() >> 4;
  const T gl = ipow(g, j + 1), gr = ipow(g, 16 - j);
  p.gl = (G == 64 && !(row & 1)) ? T(0) : gl;
  p.gl2 = row < 2 ? T(0) : ((row & 1) ? gl * p.g16 : gl);
  p.gr = (row & 1) ? T(0) : gr;
  p.gr2 = row >= 2 ? T(0) : ((row & 1) ? gr : gr * p.g16);
  return p;
}

// Inclusive scan x_l = e_l + g x_{l-1} over the lanes of each group (x_{-1} = 0):
// Kogge-Stone inside rows of 16 lanes, then carries across rows.
template <int G, typename T>
__device__ __forceinline__ T grp_scan_fwd(T e, const ScanPow<T> &p) {
  T t = e;
  t = fma(p.g1, dpp<kRowShr1>(t), t);
  t = fma(p.g2, dpp<kRowShr2>(t), t);
  t = fma(p.g4, dpp<kRowShr4>(t), t);
  t = fma(p.g8, dpp<kRowShr8>(t), t);
  if (G == 32) {
    // rows 1 and 3 carry in the last lane of rows 0 and 2 (rows 0 and 2, the
    // first rows of the groups, take nothing)
    t = fma(p.gl, dpp_rows<kRowBcast15, 0xa>(t), t);
  }
  if (G == 64) {
    // the same within the one group (rows 0 and 2 scale what they read by 0),
    // then rows 2 and 3 carry in lane 31, the scan of the first half
    t = fma(p.gl, dpp<kRowBcast15>(t), t);
    t = fma(p.gl2, dpp<kRowBcast31>(t), t);
  }
  return t;
}

// The same with g = 1 (running sums).
template <int G, typename T>
__device__ __forceinline__ T grp_sum_fwd(T e) {
  T t = e;
  t += dpp<kRowShr1>(t);
  t += dpp<kRowShr2>(t);
  t += dpp<kRowShr4>(t);
  t += dpp<kRowShr8>(t);
  if (G >= 32) t += dpp_rows<kRowBcast15, 0xa>(t);
  if (G == 64) t += dpp_rows<kRowBcast31, 0xc>(t);
  return t;
}

// Inclusive scan x_l = e_l + g x_{l+1} over the lanes of each group (x_G = 0).
template <int G, typename T>
__device__ __forceinline__ T grp_scan_bwd(T e, const ScanPow<T> &p) {
  T t = e;
  t = fma(p.g1, dpp<kRowShl1>(t), t);
  t = fma(p.g2, dpp<kRowShl2>(t), t);
  t = fma(p.g4, dpp<kRowShl4>(t), t);
  t = fma(p.g8, dpp<kRowShl8>(t), t);
  if (G >= 32) {
    // rows 0 and 2 carry in the first lane of rows 1 and 3 (rows 1 and 3 read
    // their own first lane and scale it by 0)
    t = fma(p.gr, dpp<kRowNewBcast0>(odd_rows(t)), t);
  }
  if (G == 64) {
    // rows 0 and 1 carry in lane 32, now the scan of the second half (rows 2
    // and 3 scale it by 0)
    t = fma(p.gr2, lane_read(t, 32), t);
  }
  return t;
}

// p[idx] where ok, else 0; the load itself is unconditional (p[0] is valid).
template <typename T, typename P>
__device__ __forceinline__ T ld_if(const P *p, int idx, bool ok) {
  const P v = p[ok ? idx : 0];
  return ok ? (T)v : T(0);
}

// x[m-1] for a per-lane m >= 1 (no runtime register indexing).
template <typename T, int MM>
__device__ __forceinline__ T last_of(const T (&x)[MM], int m) {
  T v = x[0];
#pragma unroll
  for (int j = 1; j < MM; ++j) v = (j < m) ? x[j] : v;
  return v;
}

// Point evaluation w0 x(n0) + w1 x(n1) (FP64) of a lane-blocked array of the
// calling lane's group (MM slots per lane, nodes 1-based, 0 = absent).
template <int G, typename T, int MM>
__device__ __forceinline__ double point_eval(const T (&x)[MM], const T (&c)[MM], int n0, double w0, int n1,
                                             double w1) {
  constexpr int m = MM;
  const int li = lane_id() & (G - 1), base = lane_id() & ~(G - 1);
  double part = 0.0;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    const int i = li * m + r + 1;
    const double v = (double)x[r] - (double)c[r];
    part += (i == n0) ? w0 * v : 0.0;
    part += (i == n1) ? w1 * v : 0.0;
  }
  const int l0 = n0 ? (n0 - 1) / m : 0, l1 = n1 ? (n1 - 1) / m : 0;
  const double y0 = __shfl(part, base + l0, kWave);
  const double y1 = __shfl(part, base + l1, kWave);
  return (n1 && l1 != l0) ? y0 + y1 : y0;
}

// Point interpolant held as per-slot weights w[0..MM) of the calling lane
// (zero on slots without one of its nodes): sum over the group of
// w (x - c), returned to every lane of the group.
template <int G, int MM, typename T>
__device__ __forceinline__ T slot_dot(const T *w, const T (&x)[MM], const T (&c)[MM]) {
  T wv[MM];
#pragma unroll
  for (int r = 0; r < MM; ++r) wv[r] = w[r];
  T part = T(0);
#pragma unroll
  for (int r = 0; r < MM; ++r) part = fma(wv[r], x[r] - c[r], part);
  return grp_reduce<G, false>(part);
}

// ---------------------------------------------------------------------------
// Exact Toeplitz solve (per group)
// ---------------------------------------------------------------------------

// kT (1 + rho S-)(1 + rho S+) x = b on nodes 1..n of each group's string
// (MM slots per lane; mask[r] is 1 on this lane's nodes <= n, else 0; wb[r]
// are the lane's weights of z_0):
//   forward:  z_i = b_i / kT - rho z_{i-1},  z_0 = sum_i wb_i b_i  (odd extension)
//   backward: x_i = z_i - rho x_{i+1},       x_N = 0
// Lane-local recurrences, then group scans carry the lane boundary values.
template <int G, typename T, int MM, typename WB, typename MK>
__device__ __forceinline__ void toeplitz_solve(T (&x)[MM], const T (&b)[MM], const WB &wb, const MK &mask, T rho,
                                               T itk, const ScanPow<T> &sp) {
  T part = T(0);
#pragma unroll
  for (int r = 0; r < MM; ++r) part = fma(wb[r], b[r], part);
  const T z0 = grp_reduce<G, false>(part);
  T z[MM];
  z[0] = b[0] * itk;
#pragma unroll
  for (int r = 1; r < MM; ++r) z[r] = fma(-rho, z[r - 1], b[r] * itk);
  T prev = z[MM - 1];
  const bool first = (lane_id() & (G - 1)) == 0;
  const T e = first ? fma(sp.g1, z0, prev) : prev;
  const T Z = grp_scan_fwd<G>(e, sp);
  const T Zp = grp_prev<G>(Z);   // every lane takes part in the move
  const T C = first ? z0 : Zp;
  T pw = -rho;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    z[r] = fma(pw, C, z[r]) * mask[r];
    pw = pw * (-rho);
  }
  x[MM - 1] = z[MM - 1];
#pragma unroll
  for (int r = MM - 2; r >= 0; --r) x[r] = fma(-rho, x[r + 1], z[r]);
  const T X = grp_scan_bwd<G>(x[0], sp);
  const T Dn = grp_next<G>(X);
  pw = T(1);
#pragma unroll
  for (int r = MM - 1; r >= 0; --r) {
    pw = pw * (-rho);
    x[r] = fma(pw, Dn, x[r]) * mask[r];
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

// (gamma^n k)^2 with gamma^n = 2 f0(nk), f0 modulated by vibrato or glide
// (evaluated once per G steps, one step per lane).
__device__ __forceinline__ double gamma2k2_at(const Desc &D, int64_t n) {
  const double t = (double)n / D.fs;
  double f = D.f0;
  if (D.mod_type == 1)
    f = f * exp2(D.mod_a * sin(2.0 * M_PI * D.mod_b * t));
  else if (D.mod_type == 2)
    f = f * exp2(D.mod_a * (t / D.mod_b));
  const double gam = 2.0 * f;
  return gam * gam * D.k * D.k;
}

// The same in FP32 for the FP32 kernels: the phase (or the glide's fraction
// of the note) is reduced in FP64, the factor 2^{2 a sin(2 pi r t)} (or
// 2^{2 a t/T}) of (gamma_0 k)^2 evaluated in FP32, where the result is
// rounded anyway.
__device__ __forceinline__ float gamma2k2_at_f(const Desc &D, int64_t n) {
  const double t = (double)n / D.fs;
  float e = 0.f;
  if (D.mod_type == 1) {
    const double cyc = D.mod_b * t;
    e = (float)(2.0 * D.mod_a) * sinf(6.28318530717958647692f * (float)(cyc - floor(cyc)));
  } else if (D.mod_type == 2) {
    e = (float)(2.0 * D.mod_a * (t / D.mod_b));
  }
  return (float)D.g2k2_0 * exp2f(e);
}

// Contact coefficient c = omega^{1+alpha_H} (eta^+)^{alpha_H - 1} / 2 of eq. (6)
// (power factor at time n), used only while a hammer touches.
__device__ __forceinline__ double contact_coef(double eta, double omega_pow, double alpha_H) {
  return eta > 0.0 ? 0.5 * omega_pow * pow(eta > 0.0 ? eta : 1.0, alpha_H - 1.0) : 0.0;
}

template <typename T>
__device__ __forceinline__ double to_d(T hi, T c) {
  return (double)hi - (double)c;
}

// LDS layout per group: the l-half slopes p (for I_(l)->(t)) and the two
// t-half contribution arrays of I_(t)->(l), each MM*G values plus one trash
// entry per lane (writes a lane must not make go there, without bank
// conflicts).
template <int G, int MM, int NARR = 3>
struct Lds {
  static constexpr int kArr = MM * G + G;
  static constexpr int kTrash = MM * G;   // + lane in group
  static constexpr int kStride = NARR * kArr;
};

// Arrays per group: p and two tap arrays; the instantiation that carries the
// cubic grid interpolant holds its two further tap arrays.
template <bool CUB>
constexpr int kLdsArrays = CUB ? 5 : 3;

// MM per-lane values of a group: in registers, or (largest class) in LDS at
// [r G] from the lane's entry, read where they are used.  With 16 slots per
// lane the tables would otherwise take a third of the register file.
template <int MM>
constexpr bool kTabLds = MM >= 10;

template <int G, int MM, typename V, bool IN_LDS>
struct LaneTab {
  V v[MM];
  __device__ V operator[](int r) const { return v[r]; }
  __device__ void put(int r, V x) { v[r] = x; }
};
template <int G, int MM, typename V>
struct LaneTab<G, MM, V, true> {
  V *p;
  __device__ V operator[](int r) const { return p[r * G]; }
  __device__ void put(int r, V x) { p[r * G] = x; }
};

// Node mask of a lane (1 on its nodes <= n, else 0), as an array or computed.
template <int MM, typename T, bool COMPUTED>
struct NodeMask {
  T v[MM];
  __device__ void init(int nb, int n) {
#pragma unroll
    for (int r = 0; r < MM; ++r) v[r] = (nb + r + 1 <= n) ? T(1) : T(0);
  }
  __device__ T operator[](int r) const { return v[r]; }
};
template <int MM, typename T>
struct NodeMask<MM, T, true> {
  int nb, n;
  __device__ void init(int nb_, int n_) {
    nb = nb_;
    n = n_;
  }
  __device__ T operator[](int r) const { return (nb + r + 1 <= n) ? T(1) : T(0); }
};

// LDS of the tables per group (where kTabLds): the index pair of
// I_(l)->(t) and the two ranges of I_(t)->(l) (32-bit words), then the
// interpolation weight, the z_0 weights of both grids and the
// Sherman-Morrison vector (T), each MM*G values.
template <int G, int MM, typename T>
struct TabLds {
  static constexpr int kWordsU = kTabLds<MM> ? 3 * MM * G : 0;
  static constexpr int kWordsT = kTabLds<MM> ? 4 * MM * G : 0;
  static constexpr int kBytes = kWordsU * 4 + kWordsT * (int)sizeof(T);
};

// The compensation arrays of the largest class live in LDS between their
// uses (4 MM G values per group) instead of in registers: with 16 slots per
// lane they would otherwise crowd the register file and spill the state.
template <int MM, typename T, bool KAHAN>
constexpr bool kSideComp = KAHAN && MM >= 16;

// array k of a group's side region holds S slots per lane (S = the larger
// grid's slot count); x has the slots of its own grid
template <int G, int S, typename T, int M>
__device__ __forceinline__ void side_load(T (&x)[M], const T *side, int k, int li) {
#pragma unroll
  for (int r = 0; r < M; ++r) x[r] = side[(k * S + r) * G + li];
}
template <int G, int S, typename T, int M>
__device__ __forceinline__ void side_save(const T (&x)[M], T *side, int k, int li) {
#pragma unroll
  for (int r = 0; r < M; ++r) side[(k * S + r) * G + li] = x[r];
}

// I_(t)->(l) up to the factor h_t/h_l at one l-half point by direct sums (the
// instantiation that carries the bow; the other uses prefix sums below): the sums of the
// two contribution arrays over its t-half ranges [sa, sa+na) and [sb, sb+nb)
// (packed as start | count << 16), with KG >= na, nb: every load is issued
// before the first is used.
template <int KG, typename T>
__device__ __forceinline__ T range_gather(const T *sA, const T *sB, uint32_t ra, uint32_t rb) {
  const int sa = (int)(ra & 0xffffu), na = (int)(ra >> 16);
  const int sb = (int)(rb & 0xffffu), nb = (int)(rb >> 16);
  T va[KG], vb[KG];
#pragma unroll
  for (int c = 0; c < KG; ++c) {
    va[c] = sA[c < na ? sa + c : 0];
    vb[c] = sB[c < nb ? sb + c : 0];
  }
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < KG; ++c) acc += (c < na ? va[c] : T(0)) + (c < nb ? vb[c] : T(0));
  return acc;
}

// The same with a run-time bound (ranges longer than the unrolled cases).
template <typename T>
__device__ __forceinline__ T range_gather_n(const T *sA, const T *sB, uint32_t ra, uint32_t rb, int kg) {
  const int sa = (int)(ra & 0xffffu), na = (int)(ra >> 16);
  const int sb = (int)(rb & 0xffffu), nb = (int)(rb >> 16);
  T acc = T(0);
  for (int c = 0; c < kg; ++c) {
    const T va = sA[c < na ? sa + c : 0];
    const T vb = sB[c < nb ? sb + c : 0];
    acc += (c < na ? va : T(0)) + (c < nb ? vb : T(0));
  }
  return acc;
}

// g[r] = I_(t)->(l) contributions at this lane's l-half points (0 past ml:
// their ranges are empty); kg is the wave's longest range.
template <int MM, typename T, typename RG>
__device__ __forceinline__ void gather_lt(T (&g)[MM], const T *sA, const T *sB, const RG &rga, const RG &rgb,
                                          int kg) {
  if (MM > 8) {
    // the unrolled forms would hold 2 KG MM loads in flight: too many registers
#pragma unroll
    for (int r = 0; r < MM; ++r) g[r] = range_gather_n<T>(sA, sB, rga[r], rgb[r], kg);
  } else if (kg <= 2) {
#pragma unroll
    for (int r = 0; r < MM; ++r) g[r] = range_gather<2, T>(sA, sB, rga[r], rgb[r]);
  } else if (kg <= 4) {
#pragma unroll
    for (int r = 0; r < MM; ++r) g[r] = range_gather<4, T>(sA, sB, rga[r], rgb[r]);
  } else if (kg <= 6) {
#pragma unroll
    for (int r = 0; r < MM; ++r) g[r] = range_gather<6, T>(sA, sB, rga[r], rgb[r]);
  } else {
#pragma unroll
    for (int r = 0; r < MM; ++r) g[r] = range_gather_n<T>(sA, sB, rga[r], rgb[r], kg);
  }
}

// I_(t)->(l) up to the factor h_t/h_l through prefix sums along the t-half
// points: with PA[i] (PB[i]) the sum of the first-tap (second-tap)
// contributions (1-w) x (w x) of t-half points 0 .. i-1, an l-half point
// whose first-tap range is [sa, sa+na) and second-tap range [sb, sb+nb)
// receives PA[sa+na] - PA[sa] + PB[sb+nb] - PB[sb]: four LDS reads, however
// long the ranges.  prefix_store writes PA[1..MM G] and PB[1..MM G] of the
// group (a lane-local running sum plus the group's exclusive scan of the
// lanes' totals) and PA[0] = PB[0] = 0; lanes other than the first write
// that zero to their own entry past the arrays (trash + lane).
template <int G, int MM, typename T, typename WI>
__device__ __forceinline__ void prefix_store(T *PA, T *PB, const T (&x)[MM], const WI &wi, int tb, int li,
                                             int trash) {
  T pa[MM], pb[MM];
  T ca = T(0), cb = T(0);
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    const T b = wi[r] * x[r];
    cb += b;
    ca += x[r] - b;
    pa[r] = ca;
    pb[r] = cb;
  }
  const T oa = grp_sum_fwd<G>(grp_prev<G>(ca)), ob = grp_sum_fwd<G>(grp_prev<G>(cb));
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    PA[tb + r + 1] = oa + pa[r];
    PB[tb + r + 1] = ob + pb[r];
  }
  const int z = li == 0 ? 0 : trash + li;
  PA[z] = T(0);
  PB[z] = T(0);
}

// g[r] = I_(t)->(l) contributions (up to h_t/h_l) at this lane's l-half
// points (0 past ml: their ranges are empty).
template <int MM, typename T, typename RG>
__device__ __forceinline__ void prefix_gather(T (&g)[MM], const T *PA, const T *PB, const RG &rga, const RG &rgb) {
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    const uint32_t ra = rga[r], rb = rgb[r];
    const int sa = (int)(ra & 0xffffu), ea = sa + (int)(ra >> 16);
    const int sb = (int)(rb & 0xffffu), eb = sb + (int)(rb >> 16);
    g[r] = (PA[ea] - PA[sa]) + (PB[eb] - PB[sb]);
  }
}

// LDS scratch of the energy monitor per group: u^{n+1}, u^n, zeta^{n+1},
// zeta^n (FP64) on nodes 0 .. MM*G, each followed by a trash entry.
template <int G, int MM>
struct EnergyLds {
  static constexpr int kArr = MM * G + 2;
  static constexpr int kTrash = MM * G + 1;
  static constexpr int kStride = 4 * kArr;
};

// Writes this lane's part of w^{n+1} = (u - cu, z - cz) and w^n = w^{n+1} - v
// into the group's energy scratch; node 0 and the unused slots hold 0.
template <int G, int MT, int ML, typename T>
__device__ __forceinline__ void energy_fill(double *sD, const T (&u)[MT], const T (&vu)[MT], const T (&cu)[MT],
                                            const T (&cvu)[MT], const T (&z)[ML], const T (&vz)[ML],
                                            const T (&cz)[ML], const T (&cvz)[ML], int li) {
  using E = EnergyLds<G, (MT > ML ? MT : ML)>;
  double *U1 = sD, *U0 = sD + E::kArr, *Z1 = sD + 2 * E::kArr, *Z0 = sD + 3 * E::kArr;
  const int zero_at = li == 0 ? 0 : E::kTrash;
  U1[zero_at] = 0.0;
  U0[zero_at] = 0.0;
  Z1[zero_at] = 0.0;
  Z0[zero_at] = 0.0;
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    const int it = li * MT + r + 1;
    const double a1 = (double)u[r] - (double)cu[r];
    U1[it] = a1;
    U0[it] = a1 - ((double)vu[r] - (double)cvu[r]);
  }
#pragma unroll
  for (int r = 0; r < ML; ++r) {
    const int il = li * ML + r + 1;
    const double b1 = (double)z[r] - (double)cz[r];
    Z1[il] = b1;
    Z0[il] = b1 - ((double)vz[r] - (double)cvz[r]);
  }
}

// Discrete energy H^{n+1/2} (FP64) of the calling lane's group from the
// scratch filled by energy_fill: kinetic and linear potential of both grids
// plus the nonlinear potential (gamma^2 (alpha^2-1)/2)(p q^2/2 + q^4/8) in
// the time-paired form of the scheme.  Streams over the lane's points
// (runs once per monitor period).
template <int G, int MM, typename T, bool CLAMP, bool CUB>
__device__ __forceinline__ double energy_fp64(const Desc &D, double g2k2, const double *sD, int li) {
  using E = EnergyLds<G, MM>;
  const double *U1 = sD, *U0 = sD + E::kArr, *Z1 = sD + 2 * E::kArr, *Z0 = sD + 3 * E::kArr;
  const int mt = D.mt, ml = D.ml, nt = D.nt, Nt = D.Nt, Nl = D.Nl, nl = D.nl;
  const double k = D.k, th = D.theta, Ntd = D.Ntd, Nld = D.Nld;
  const T *tf = (const T *)D.tabf;
  double kin = 0.0, pot = 0.0, stf = 0.0, nlt = 0.0;
#pragma unroll 1
  for (int r = 0; r < MM; ++r) {
    const int i = li * mt + r + 1;
    const bool half = r < mt && i <= Nt, node = r < mt && i <= nt;
    const int ic = half ? i : 1;                       // a valid node for the loads
    const int im = ic - 1, ip = ic + 1 <= MM * G ? ic + 1 : ic;
    const double du = U1[ic] - U0[ic], dm = U1[im] - U0[im], dp = U1[ip] - U0[ip];
    const double q1 = (U1[ic] - U1[im]) * Ntd, q0 = (U0[ic] - U0[im]) * Ntd;
    const double q1p = (U1[ip] - U1[ic]) * Ntd, q0p = (U0[ip] - U0[ic]) * Ntd;
    const double c1 = (q1p - q1) * Ntd, c0 = (q0p - q0) * Ntd;
    kin += node ? du * (th * du + 0.5 * (1.0 - th) * (dm + dp)) : 0.0;
    stf += node ? c1 * c0 : 0.0;
    // clamped ends: the end nodes' curvatures 2 q_1 Nt and -2 q_Nt Nt enter
    // with trapezoid weight 1/2
    if constexpr (CLAMP) stf += (D.clamped != 0 && half && (i == 1 || i == Nt)) ? 2.0 * Ntd * Ntd * q1 * q0 : 0.0;
    pot += half ? q1 * q0 : 0.0;
    const bool on = half && nl > 0;
    const uint32_t jab = ld_if<uint32_t>(D.tab, r * G + li, on);
    const int ja = on ? (int)(jab & 0xffffu) : 1, jb = on ? (int)(jab >> 16) : 1;
    const double w = ld_if<double>(tf, r * G + li, on);
    const double pa1 = (Z1[ja] - Z1[ja - 1]) * Nld, pa0 = (Z0[ja] - Z0[ja - 1]) * Nld;
    const double pb1 = (Z1[jb] - Z1[jb - 1]) * Nld, pb0 = (Z0[jb] - Z0[jb - 1]) * Nld;
    double pt1 = (1.0 - w) * pa1 + w * pb1, pt0 = (1.0 - w) * pa0 + w * pb0;
    if constexpr (CUB) {
      // the cubic grid interpolant: taps ja .. ja+3
      if (D.grid_interp == 3 && on) {
        const T *tfc = tf + (3 * mt + ml) * G;
        const double wc[4] = {w, (double)tfc[r * G + li], (double)tfc[(mt + r) * G + li],
                              (double)tfc[(2 * mt + r) * G + li]};
        double s1 = 0.0, s0 = 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          s1 += wc[x] * ((Z1[ja + x] - Z1[ja + x - 1]) * Nld);
          s0 += wc[x] * ((Z0[ja + x] - Z0[ja + x - 1]) * Nld);
        }
        pt1 = s1;
        pt0 = s0;
      }
    }
    const double qq = q1 * q0;
    nlt += on ? qq * qq / 4.0 + qq * (pt1 + pt0) / 2.0 : 0.0;
  }
  double kz = 0.0, pz = 0.0;
#pragma unroll 1
  for (int r = 0; r < MM; ++r) {
    const int j = li * ml + r + 1;
    const bool half = r < ml && j <= Nl, node = r < ml && j <= nl;
    const int jc = half ? j : 1;
    const double dz = Z1[jc] - Z0[jc];
    const double p1 = (Z1[jc] - Z1[jc - 1]) * Nld, p0 = (Z0[jc] - Z0[jc - 1]) * Nld;
    kz += node ? dz * dz : 0.0;
    pz += half ? p1 * p0 : 0.0;
  }
  const double gam2 = g2k2 / (k * k);
  const double kap2 = D.cS / (k * k * Ntd * Ntd);
  double H = (1.0 / Ntd) / (2.0 * k * k) * kin + gam2 / Ntd / 2.0 * pot + kap2 / Ntd / 2.0 * stf;
  const double a2 = D.a2;
  H += (nl > 0) ? (1.0 / Nld) / (2.0 * k * k) * kz + gam2 * a2 / Nld / 2.0 * pz + gam2 * (a2 - 1.0) / 2.0 / Ntd * nlt
                : 0.0;
  return grp_reduce<G, false>(H);
}

// Stores the register state into the string's state block, laid out
// [array][slot][lane] with MT slots per lane for u and ML for zeta.
template <int G, typename T, int MT, int ML>
__device__ __forceinline__ void store_state(T *st, const T (&u)[MT], const T (&vu)[MT], const T (&cu)[MT],
                                            const T (&cvu)[MT], const T (&z)[ML], const T (&vz)[ML],
                                            const T (&cz)[ML], const T (&cvz)[ML], int li) {
  constexpr int zo = 4 * MT * G;
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    st[(0 * MT + r) * G + li] = u[r];
    st[(1 * MT + r) * G + li] = vu[r];
    st[(2 * MT + r) * G + li] = cu[r];
    st[(3 * MT + r) * G + li] = cvu[r];
  }
#pragma unroll
  for (int r = 0; r < ML; ++r) {
    st[zo + (0 * ML + r) * G + li] = z[r];
    st[zo + (1 * ML + r) * G + li] = vz[r];
    st[zo + (2 * ML + r) * G + li] = cz[r];
    st[zo + (3 * ML + r) * G + li] = cvz[r];
  }
}

// Debug builds (SFD_POISON_LDS=1) fill the LDS that a task or a step must
// write before it reads with NaN: all of a group's LDS at the start of every
// task, and the arrays every step rebuilds (slopes, taps, prefix sums, the
// energy scratch that overlays them) at the end of every step.  A read of a
// stale or never-written entry then makes the output NaN or trips the energy
// monitor.  Regular builds compile none of it.
#ifndef SFD_POISON_LDS
#define SFD_POISON_LDS 0
#endif
constexpr bool kPoisonLds = SFD_POISON_LDS != 0;

template <int G, typename V>
__device__ __forceinline__ void poison_lds(V *p, int n, int li) {
  const V nan = (V)__builtin_nan("");
  for (int i = li; i < n; i += G) p[i] = nan;
}

// ---------------------------------------------------------------------------
// One wavefront task: up to 64/G strings stepped together
// ---------------------------------------------------------------------------

template <int G, int MT, int ML, typename T, bool KAHAN, bool BOW, bool CUB>
__device__ __forceinline__ void run_task(const LaunchArgs &a, const int32_t *work, int task, T *sS, double *sE, T *sC,
                                         uint32_t *sTu, T *sTf, double *sB, T *sW) {
  // MT and ML slots per lane on the transverse and longitudinal grids; LDS
  // regions are laid out for the larger, MM
  constexpr int MM = MT > ML ? MT : ML;
  const int lane = lane_id();
  const int li = lane & (G - 1), gi = lane / G;
  const int sidx = work[task * (kWave / G) + gi];
  const bool present = sidx >= 0;
  // an empty group mirrors the task's first string but never steps or writes it
  const int s = present ? sidx : work[task * (kWave / G)];
  const Desc &D = a.desc[s];
  Status *S = a.status + s;

  // ---- per-group constants (lane registers) ----
  const int nt = D.nt, nl = D.nl;
  constexpr int mt = MT, ml = ML;   // slots per lane of the string's layout
  const int64_t n_samples = D.n_samples;
  const int64_t done = S->samples_done;
  const int64_t left = n_samples - done;
  int64_t nsteps = a.n_steps < left ? a.n_steps : left;
  if (!present || S->flags != 0 || done < 2 || nsteps < 0) nsteps = 0;
  // the wave runs as many steps as its longest group
  int64_t wsteps = nsteps;
#pragma unroll
  for (int o = G; o < kWave; o <<= 1) {
    const int64_t other = __shfl_xor(wsteps, o, kWave);
    wsteps = other > wsteps ? other : wsteps;
  }
  wsteps = uni(wsteps);

  const bool any_mod = __ballot(D.mod_type != 0) != 0;
  // clamped ends and the zeta channel, like the bow, exist only in the BOW
  // instantiation
  const bool clamped = BOW && D.clamped != 0;
  const bool any_clamp = BOW && __ballot(clamped) != 0;
  const bool zout = BOW && D.zeta_out != 0;
  const bool any_zout = BOW && __ballot(zout) != 0;
  const double omega_pow = D.omega_pow, alpha_H = D.alpha_H, Mr = D.Mr, IHs = D.IHs;
  const bool ham = D.ham_on != 0;
  const bool any_ham = __ballot(ham) != 0;
  // The hammer's interpolant I_H (two nodes, four with the cubic one) and
  // the readout's I(x_out) as per-slot weights of this lane, in LDS at
  // [lane][slot]: one multiply-add per slot and one group sum per use.
  T *wH = sW + lane * MT, *wO = sW + kWave * MM + lane * MT;
  using L = Lds<G, MM, kLdsArrays<CUB>>;
  if constexpr (kPoisonLds) {
    poison_lds<G>(sS + gi * L::kStride, L::kStride, li);
    poison_lds<G>(sE + gi * EnergyLds<G, MM>::kStride, EnergyLds<G, MM>::kStride, li);
    poison_lds<1>(wH, MT, 0);
    poison_lds<1>(wO, MT, 0);
    if constexpr (BOW) poison_lds<G>(sB + gi * kBowRec, kBowRec, li);
    if constexpr (kSideComp<MM, T, KAHAN>) poison_lds<G>(sC + gi * 4 * MM * G, 4 * MM * G, li);
    if constexpr (kTabLds<MM>) poison_lds<G>(sTf + gi * TabLds<G, MM, T>::kWordsT, TabLds<G, MM, T>::kWordsT, li);
    __syncthreads();
  }
  {
    // (a cubic hammer's extra nodes share their storage with a bow's fields)
    const int h0 = ham ? D.hn0 : 0, h1 = ham ? D.hn1 : 0, h2 = ham ? D.hn2 : 0, h3 = ham ? D.hn3 : 0;
    const double w0 = h0 ? D.hw0 : 0.0, w1 = h1 ? D.hw1 : 0.0, w2 = h2 ? D.hw2 : 0.0, w3 = h3 ? D.hw3 : 0.0;
    const int o0 = D.on0, o1 = D.on1;
    const double v0 = o0 ? D.ow0 : 0.0, v1 = o1 ? D.ow1 : 0.0;
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      const int node = li * MT + r + 1;
      wH[r] = (T)((node == h0 ? w0 : 0.0) + (node == h1 ? w1 : 0.0) + (node == h2 ? w2 : 0.0) + (node == h3 ? w3 : 0.0));
      wO[r] = (T)((node == o0 ? v0 : 0.0) + (node == o1 ? v1 : 0.0));
    }
  }
  const bool bowed = BOW && D.bow_on != 0;
  // the stopping rule of the coupled solve for bowed strings (the other
  // strings of the bow family's instantiation keep the usual one)
  const bool bow_stop = bowed;
  // the bow's code exists only in the BOW instantiation (its registers would
  // crowd every other task's)
  const bool any_bow = BOW && __ballot(bowed) != 0;
  double *bR = sB + gi * kBowRec;   // this group's bow record
  if (any_bow) {
    // groups without a bow get zeros (their descriptor's bow fields may hold
    // a cubic hammer's nodes)
    bR[kBowX0] = bowed ? D.bx0 : 0.0;
    bR[kBowX1] = bowed ? bow_x_rate(D.bx0, D.bx1, D.bT) : 0.0;
    bR[kBowT] = bowed ? D.bT : 0.0;
    bR[kBowVB] = bowed ? D.bvB : 0.0;
    bR[kBowFB] = bowed ? D.bFB : 0.0;
    bR[kBowTa] = bowed ? bow_ramp_rate(D.bta) : 0.0;
    bR[kBowA] = bowed ? D.ba : 0.0;
    bR[kBowEps] = bowed ? D.beps : 0.0;
    bR[kBowT0] = bowed ? D.bt0 : 0.0;
  }
  const bool any_l = __ballot(D.nl > 0) != 0;
  // the instantiation that carries the bow sums I_(t)->(l) directly over the
  // ranges (chaotic bowed strings are sensitive to the rounding of prefix
  // differences); gmax is the wave's longest range
  int gmax = 0;
  if constexpr (BOW) {
    gmax = D.gmax;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int x = __shfl_xor(gmax, o, kWave);
      gmax = x > gmax ? x : gmax;
    }
    gmax = __builtin_amdgcn_readfirstlane(gmax);
  }
  // cubic grid interpolant (p = 3), only in its own instantiation (one that
  // also carries the bow's code): a string's jab holds the base l-half point b of each t-half point
  // (taps b .. b+3) and wi the first tap's weight; the other three weights and
  // the ranges of taps 2 and 3 follow the linear tables and are read from
  // memory where used
  const bool cub = CUB && D.grid_interp == 3;
  const bool any_cub = CUB && __ballot(cub) != 0;
  const double g2k2_0 = D.g2k2_0, a2m1_4 = D.a2m1_4, a2d = D.a2, Ntdd = D.Ntd, kk = D.k * D.k;
  const int mon_check = D.mon_check;

  // ---- state and tables into registers ----
  T u[MT], vu[MT], cu[MT], cvu[MT], z[ML], vz[ML], cz[ML], cvz[ML];
  constexpr bool kTL = kTabLds<MM>;
  LaneTab<G, MT, uint32_t, kTL> jab;
  LaneTab<G, ML, uint32_t, kTL> rga, rgb;
  LaneTab<G, MT, T, kTL> wi, wbu, smt;
  LaneTab<G, ML, T, kTL> wbz;
  if constexpr (kTL) {
    jab.p = sTu + gi * TabLds<G, MM, T>::kWordsU + li;
    rga.p = jab.p + MM * G;
    rgb.p = rga.p + MM * G;
    wi.p = sTf + gi * TabLds<G, MM, T>::kWordsT + li;
    wbu.p = wi.p + MM * G;
    wbz.p = wbu.p + MM * G;
    smt.p = wbz.p + MM * G;
  }
  T *st = (T *)D.st;
  const T *tf = (const T *)D.tabf;
  const uint32_t *tab = D.tab;
  const int zo = 4 * mt * G;
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    // without compensation the c arrays stay zero (constants the compiler folds)
    u[r] = st[(0 * mt + r) * G + li];
    vu[r] = st[(1 * mt + r) * G + li];
    cu[r] = KAHAN ? st[(2 * mt + r) * G + li] : T(0);
    cvu[r] = KAHAN ? st[(3 * mt + r) * G + li] : T(0);
    jab.put(r, tab[r * G + li]);
    wi.put(r, tf[r * G + li]);
    wbu.put(r, tf[(mt + r) * G + li]);
    // Sherman-Morrison vector (zero without a hammer), kept in LDS
    if constexpr (kTL) smt.put(r, tf[(2 * mt + ml + r) * G + li]);
  }
#pragma unroll
  for (int r = 0; r < ML; ++r) {
    z[r] = st[zo + (0 * ml + r) * G + li];
    vz[r] = st[zo + (1 * ml + r) * G + li];
    cz[r] = KAHAN ? st[zo + (2 * ml + r) * G + li] : T(0);
    cvz[r] = KAHAN ? st[zo + (3 * ml + r) * G + li] : T(0);
    rga.put(r, tab[(mt + r) * G + li]);
    rgb.put(r, tab[(mt + ml + r) * G + li]);
    wbz.put(r, tf[(2 * mt + r) * G + li]);
  }
  const T *smv = tf + (2 * mt + ml) * G;   // Sherman-Morrison vector T_u0^{-1} J_H
  constexpr bool kSide = kSideComp<MM, T, KAHAN>;
  T *side = sC + gi * 4 * MM * G;
  if constexpr (kSide) {
    side_save<G, MM>(cu, side, 0, li);
    side_save<G, MM>(cvu, side, 1, li);
    side_save<G, MM>(cz, side, 2, li);
    side_save<G, MM>(cvz, side, 3, li);
  }

  // Nodes past the string's end hold zero state, which the solves keep
  // (node masks); slopes, couplings and LDS contributions there vanish by
  // themselves, so no other predicate is needed.
  const int tb = li * mt, lb = li * ml;
  NodeMask<MT, T, kTL> mask_t;
  NodeMask<ML, T, kTL> mask_l;
  mask_t.init(tb, nt);
  mask_l.init(lb, nl);

  const T rho_t = (T)D.rho_t, itk_t = (T)D.itk_t, rho_l = (T)D.rho_l, itk_l = (T)D.itk_l;
  const ScanPow<T> spt = scan_pow<G, T>(ipow<T>(-rho_t, mt));
  const ScanPow<T> spl = scan_pow<G, T>(ipow<T>(-rho_l, ml));
  const T Ntd = (T)D.Ntd, Nld = (T)D.Nld;
  const T cS = (T)D.cS, s0t2 = (T)(2.0 * D.s0k_t), s1t2 = (T)(2.0 * D.s1k_t);
  const T s0l2 = (T)(2.0 * D.s0k_l), s1l2 = (T)(2.0 * D.s1k_l);
  const T ratio = (T)D.ratio_lt;

  // hammer and monitor state
  double uH_n = S->uH_n, uH_nm1 = S->uH_nm1, eta_nm1 = S->eta_nm1;
  int touched = S->touched;
  double H_ref = S->H_ref, H_last = S->H_latest;
  int64_t H_step = S->H_step;
  int flags = 0, max_sw = S->max_sweeps;
  int64_t tot_sw = S->total_sweeps;
  int64_t steps_done = 0;

  // output: a ring of G samples per group, anchored at the first sample of
  // this launch; a lane with nothing to write stores into the padding after n_samples
  T *out = (T *)D.out;
  const int64_t first_m = done;
  T ring = T(0), ring_z = T(0);
  // per-step coefficients of an unmodulated string (and a modulated string's
  // block of G values of (gamma^n k)^2, one per lane, in the kernel precision)
  const bool modg = D.mod_type != 0;
  const T G2_0 = (T)g2k2_0, phi2_0 = (T)(g2k2_0 * a2m1_4), aG_0 = (T)(g2k2_0 * a2d);
  const T a2m1_4t = (T)a2m1_4, a2t = (T)a2d;
  T g2blk = G2_0;
  T *trash = (T *)a.trash_st;
  // (n + 1) mod mon_period of the current step
  int mon_ctr = a.mon_period > 0 ? (int)(done % a.mon_period) : 1;

  T *gP = sS + gi * L::kStride, *gA = gP + L::kArr, *gB = gA + L::kArr;
  T *gC = CUB ? gB + L::kArr : gB, *gD = CUB ? gC + L::kArr : gB;   // cubic taps 2 and 3
  const T *tfc = tf + (3 * mt + ml) * G;          // cubic grid interpolant: weights 1..3 per t-slot
  const uint32_t *tabc = tab + (mt + 2 * ml) * G; // and the ranges of taps 2 and 3 per l-slot
  // weight k (1..3) of the cubic grid interpolant at t-slot r (0 elsewhere)
  auto cw = [&](int k, int r) -> T { return ld_if<T>(tfc, ((k - 1) * mt + r) * G + li, cub && r < mt); };
  // I_(l)->(t) at this lane's t-half point r of the group's l-half values sX
  auto interp_lt = [&](const T *sX, int r) -> T {
    const int ja = (int)(jab[r] & 0xffffu), jb = (int)(jab[r] >> 16);
    const T w = wi[r];
    T v = (T(1) - w) * sX[ja - 1] + w * sX[jb - 1];
    if constexpr (CUB) {
      if (any_cub) {
        // taps b .. b+3 from the base b = ja; index ja + 2 stays inside the
        // group's array for every group
        const T vc = ((w * sX[ja - 1] + cw(1, r) * sX[ja]) + cw(2, r) * sX[ja + 1]) + cw(3, r) * sX[ja + 2];
        v = cub ? vc : v;
      }
    }
    return v;
  };
  // the tap contributions of x at this lane's t-half points (the
  // instantiation that carries the bow sums them directly over the ranges)
  auto tap_store = [&](const T (&x)[MT]) {
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      const T w = wi[r];
      if (CUB && any_cub) {
        gA[tb + r] = (cub ? w : T(1) - w) * x[r];
        gB[tb + r] = (cub ? cw(1, r) : w) * x[r];
        gC[tb + r] = cw(2, r) * x[r];
        gD[tb + r] = cw(3, r) * x[r];
      } else {
        gA[tb + r] = (T(1) - w) * x[r];
        gB[tb + r] = w * x[r];
      }
    }
  };
  // I_(t)->(l) up to h_t/h_l at this lane's l-half points, summed directly
  auto tap_gather = [&](T (&g)[ML]) {
    gather_lt<ML, T>(g, gA, gB, rga, rgb, gmax);
    if (CUB && any_cub) {
      uint32_t rc[ML], rd[ML];
#pragma unroll
      for (int r = 0; r < ML; ++r) {
        rc[r] = ld_if<uint32_t>(tabc, r * G + li, cub && r < ml);
        rd[r] = ld_if<uint32_t>(tabc, (ml + r) * G + li, cub && r < ml);
      }
      T g2[ML];
      gather_lt<ML, T>(g2, gC, gD, rc, rd, gmax);
#pragma unroll
      for (int r = 0; r < ML; ++r) g[r] += g2[r];
    }
  };
  double *gE = sE + gi * EnergyLds<G, MM>::kStride;

  for (int64_t it = 0; it < wsteps; ++it) {
    const bool act = it < nsteps;                  // this group still steps
    const int64_t n = done - 1 + it;               // time level; the step produces sample n+1
    // ---- gamma^n (f0 modulation): one block of G steps per lane ----
    double g2k2 = g2k2_0;
    T G2 = G2_0, phi2 = phi2_0, aG = aG_0;
    if (any_mod) {
      if ((it & (G - 1)) == 0) {
        if constexpr (sizeof(T) == 4)
          g2blk = gamma2k2_at_f(D, n + li);
        else
          g2blk = gamma2k2_at(D, n + li);
      }
      const T gm = __shfl(g2blk, (lane & ~(G - 1)) + (int)(it & (G - 1)), kWave);
      G2 = modg ? gm : G2_0;
      phi2 = modg ? gm * a2m1_4t : phi2_0;
      aG = modg ? gm * a2t : aG_0;
      g2k2 = modg ? (double)gm : g2k2_0;
    }

    // ---- slopes q (t half points) and p (l half points) ----
    T q[MT], p[ML];
    if constexpr (kSide) {
      side_load<G, MM>(cu, side, 0, li);
      side_load<G, MM>(cz, side, 2, li);
    }
    {
      const T ul = grp_prev<G>(last_of<T, MT>(u, mt)), cl = grp_prev<G>(last_of<T, MT>(cu, mt));
      const T zl = grp_prev<G>(last_of<T, ML>(z, ml)), czl = grp_prev<G>(last_of<T, ML>(cz, ml));
#pragma unroll
      for (int r = 0; r < MT; ++r) {
        const T um = r == 0 ? ul : u[r > 0 ? r - 1 : 0];
        const T cm = r == 0 ? cl : cu[r > 0 ? r - 1 : 0];
        q[r] = ((u[r] - um) - (cu[r] - cm)) * Ntd;
      }
#pragma unroll
      for (int r = 0; r < ML; ++r) {
        const T zm = r == 0 ? zl : z[r > 0 ? r - 1 : 0];
        const T czm = r == 0 ? czl : cz[r > 0 ? r - 1 : 0];
        p[r] = ((z[r] - zm) - (cz[r] - czm)) * Nld;
      }
    }

    // ---- p~ = I_(l)->(t) p, and the transposed contributions of q^2 ----
    T f[MT], q2[MT];
#pragma unroll
    for (int r = 0; r < ML; ++r) gP[lb + r] = p[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      const T pt = interp_lt(gP, r);
      q2[r] = q[r] * q[r];
      f[r] = q[r] * (q2[r] + T(2) * pt);
    }
    if constexpr (BOW)
      tap_store(q2);
    else
      prefix_store<G, MT, T>(gA, gB, q2, wi, tb, li, L::kTrash);
    __syncthreads();

    // ---- right-hand side, transverse ----
    T ru[MT], rz[ML];
    {
      T c[MT];
      const T qr = grp_next<G>(q[0]);
#pragma unroll
      for (int r = 0; r < MT; ++r) {
        const T qn = (r + 1 < MT) ? q[r + 1 < MT ? r + 1 : r] : qr;
        c[r] = (qn - q[r]) * Ntd * mask_t[r];
      }
      // Curvature at the end nodes 0 and Nt: zero for simply supported ends;
      // for clamped ends the mirrored ghost slopes (q_0 = -q_1, q_{Nt+1} =
      // -q_Nt) give 2 q_1 Nt and -2 q_Nt Nt.  Slot nt holds q_Nt and stands
      // for node Nt; slots past it only feed rows the solve keeps at zero.
      T cl = grp_prev<G>(last_of<T, MT>(c, mt));
      if constexpr (BOW) {
        if (any_clamp) {
          const T e = clamped ? T(2) * Ntd : T(0);
#pragma unroll
          for (int r = 0; r < MT; ++r) c[r] = tb + r == nt ? -e * q[r] : c[r];
          cl = li == 0 ? e * q[0] : cl;
        }
      }
      const T cr = grp_next<G>(c[0]);
      const T fr = grp_next<G>(f[0]);
      const T vl = grp_prev<G>(last_of<T, MT>(vu, mt)), vr = grp_next<G>(vu[0]);
#pragma unroll
      for (int r = 0; r < MT; ++r) {
        const bool nx = r + 1 < MT;
        const T cm = r == 0 ? cl : c[r > 0 ? r - 1 : 0];
        const T cp = nx ? c[r + 1 < MT ? r + 1 : r] : cr;
        const T fp = nx ? f[r + 1 < MT ? r + 1 : r] : fr;
        const T vm = r == 0 ? vl : vu[r > 0 ? r - 1 : 0];
        const T vp = nx ? vu[r + 1 < MT ? r + 1 : r] : vr;
        T acc = G2 * c[r] - cS * ((cp - T(2) * c[r]) + cm);
        acc = fma(T(2) * phi2 * Ntd, fp - f[r], acc);
        acc = fma(-s0t2, vu[r], acc);
        acc = fma(s1t2, (vp - T(2) * vu[r]) + vm, acc);
        ru[r] = acc;
      }
    }
    // ---- right-hand side, longitudinal ----
    {
      T g[ML];
      if constexpr (BOW)
        tap_gather(g);
      else
        prefix_gather<ML, T>(g, gA, gB, rga, rgb);
#pragma unroll
      for (int r = 0; r < ML; ++r) g[r] *= ratio;
      const T pr = grp_next<G>(p[0]), gr = grp_next<G>(g[0]);
      const T vl = grp_prev<G>(last_of<T, ML>(vz, ml)), vr = grp_next<G>(vz[0]);
#pragma unroll
      for (int r = 0; r < ML; ++r) {
        const bool nx = r + 1 < ML;
        const T pn = nx ? p[r + 1 < ML ? r + 1 : r] : pr;
        const T gn = nx ? g[r + 1 < ML ? r + 1 : r] : gr;
        const T vm = r == 0 ? vl : vz[r > 0 ? r - 1 : 0];
        const T vp = nx ? vz[r + 1 < ML ? r + 1 : r] : vr;
        T acc = aG * ((pn - p[r]) * Nld);
        acc = fma(T(2) * phi2 * Nld, gn - g[r], acc);
        acc = fma(-s0l2, vz[r], acc);
        acc = fma(s1l2, (vp - T(2) * vz[r]) + vm, acc);
        rz[r] = acc;
      }
    }

    // ---- hammer: contact coefficient at time n, right-hand side 2 beta J eta^n ----
    // (without contact anywhere in the wavefront the contact terms vanish:
    // beta = 0, no right-hand side, and the lumped mass moves freely)
    double eta_n = 0.0, cH = 0.0, beta = 0.0;
    if (any_ham) {
      if constexpr (kSide) side_load<G, MM>(cu, side, 0, li);
      const double Iu = (double)slot_dot<G, MT, T>(wH, u, cu);
      eta_n = ham ? uH_n - Iu : 0.0;
      const bool contact = eta_n > 0.0;
      touched = (act && contact) ? 1 : touched;
      if (__ballot(contact) != 0) {
        const double cc = contact_coef(eta_n, omega_pow, alpha_H);
        cH = contact ? cc : 0.0;
        beta = kk * Mr * cH / (1.0 + kk * cH);
        // right-hand side 2 beta J_H eta^n with J_H = I_H^T / h_t
        const T addH = (T)(2.0 * beta * Ntdd * eta_n);
#pragma unroll
        for (int r = 0; r < MT; ++r) ru[r] = fma(wH[r], addH, ru[r]);
      }
    }
    const bool sm_on = beta != 0.0;
    const bool any_sm = __ballot(sm_on) != 0;

    // ---- bow: controls at time n and the part of v_rel that the solve
    // does not change ----
    if (any_bow) {
      double xB, vB, FB;
      bow_controls(bR, (double)n * D.k, xB, vB, FB);
      // I_p(x_B): linear, or the cubic interpolant (four nodes, ghosts
      // mirrored with the end condition's sign)
      int bn0, bn1, bn2 = 0, bn3 = 0;
      double bw0, bw1, bw2 = 0.0, bw3 = 0.0;
      bow_interp(xB, nt + 1, bn0, bn1, bw0, bw1);
      if (__ballot(bowed && D.bow_cubic != 0) != 0) {
        int cn[4];
        double cwt[4];
        cubic_interp(xB, nt + 1, D.clamped ? 1.0 : -1.0, cn, cwt);
        const bool c3 = bowed && D.bow_cubic != 0;
        bn0 = c3 ? cn[0] : bn0;
        bn1 = c3 ? cn[1] : bn1;
        bn2 = c3 ? cn[2] : 0;
        bn3 = c3 ? cn[3] : 0;
        bw0 = c3 ? cwt[0] : bw0;
        bw1 = c3 ? cwt[1] : bw1;
        bw2 = c3 ? cwt[2] : 0.0;
        bw3 = c3 ? cwt[3] : 0.0;
      }
      const double kk = D.k * D.k;
      bR[kBowStepVB] = vB;
      bR[kBowStepK2F] = kk * FB;
      if constexpr (kSide) {
        T cv[MT];
        side_load<G, MM>(cv, side, 1, li);
        bR[kBowStepIv] = point_eval<G, T, MT>(vu, cv, bn0, bw0, bn1, bw1) + point_eval<G, T, MT>(vu, cv, bn2, bw2, bn3, bw3);
      } else {
        bR[kBowStepIv] =
            point_eval<G, T, MT>(vu, cvu, bn0, bw0, bn1, bw1) + point_eval<G, T, MT>(vu, cvu, bn2, bw2, bn3, bw3);
      }
      bR[kBowStepW2] = bw2;
      bR[kBowStepW3] = bw3;
      bR[kBowStepN2] = (double)bn2;
      bR[kBowStepN3] = (double)bn3;
      bR[kBowStepW0] = bw0;
      bR[kBowStepW1] = bw1;
      bR[kBowStepN0] = (double)bn0;
      bR[kBowStepN1] = (double)bn1;
    }

    // ---- coupled solve: block Gauss-Seidel around T_u0 (+ hammer) and T_z ----
    T smr[MT], zero[MT], zero_l[ML];
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      zero[r] = T(0);
      smr[r] = T(0);
    }
#pragma unroll
    for (int r = 0; r < ML; ++r) zero_l[r] = T(0);
    if (!kTL && any_sm) {
#pragma unroll
      for (int r = 0; r < MT; ++r) smr[r] = ld_if<T>(smv, r * G + li, sm_on);
    }
    const T smfac = any_sm ? (T)(beta / (1.0 + beta * IHs)) : T(0);
    // One solve of the step's coupled system A [a_u; a_z] = [f_u; f_z] (the
    // hammer's rank-one term included when `hammer`); returns this group's
    // sweeps and whether it converged.
    auto gs_solve = [&](const T (&fu)[MT], const T (&fz)[ML], bool hammer, T (&au)[MT], T (&az)[ML],
                        bool &conv) -> int {
#pragma unroll
      for (int r = 0; r < MT; ++r) au[r] = T(0);
#pragma unroll
      for (int r = 0; r < ML; ++r) az[r] = T(0);
      conv = false;            // this group's iterates are final
      int sweeps = 0;
      T ascale = T(0);         // tol x the group's largest value after the first sweep
      T iscale = T(0);         // 1 / that largest value (0 for a string at rest)
      T dprev = T(1);          // the group's largest update of the last sweep, times iscale
      for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
        // transverse right-hand side with the current coupling terms:
        // e = q (q D_x- a_u + I_(l)->(t) D_x- a_z), b_u = r_u + phi^2 D_x+ e
        T bu[MT];
        if (sweep == 0) {
  #pragma unroll
          for (int r = 0; r < MT; ++r) bu[r] = fu[r];
        } else {
          const T al = grp_prev<G>(last_of<T, MT>(au, mt));
          const T zl = grp_prev<G>(last_of<T, ML>(az, ml));
  #pragma unroll
          for (int r = 0; r < ML; ++r) {
            const T zm = r == 0 ? zl : az[r > 0 ? r - 1 : 0];
            gP[lb + r] = (az[r] - zm) * Nld;
          }
          __syncthreads();
          T e[MT];
  #pragma unroll
          for (int r = 0; r < MT; ++r) {
            const T am = r == 0 ? al : au[r > 0 ? r - 1 : 0];
            const T d = (au[r] - am) * Ntd;
            const T idz = interp_lt(gP, r);
            e[r] = q[r] * fma(q[r], d, idz);
          }
          __syncthreads();
          const T er = grp_next<G>(e[0]);
  #pragma unroll
          for (int r = 0; r < MT; ++r) {
            const T en = (r + 1 < MT) ? e[r + 1 < MT ? r + 1 : r] : er;
            bu[r] = fma(phi2 * Ntd, en - e[r], fu[r]);
          }
        }
        T nu[MT];
        toeplitz_solve<G, T, MT>(nu, bu, wbu, mask_t, rho_t, itk_t, spt);
        if (hammer && any_sm) {
          // Sherman-Morrison for the rank-one hammer term beta J I
          const T Iy = slot_dot<G, MT, T>(wH, nu, zero);
          const T fac = smfac * Iy;
  #pragma unroll
          for (int r = 0; r < MT; ++r) nu[r] = fma(-fac, kTL ? (sm_on ? smt[r] : T(0)) : smr[r], nu[r]);
        }
        // longitudinal right-hand side: r_z + phi^2 D_x+ I_(t)->(l) (q D_x- a_u)
        T gg[ML];
        {
          const T al = grp_prev<G>(last_of<T, MT>(nu, mt));
          T fq[MT];
  #pragma unroll
          for (int r = 0; r < MT; ++r) {
            const T am = r == 0 ? al : nu[r > 0 ? r - 1 : 0];
            fq[r] = q[r] * ((nu[r] - am) * Ntd);
          }
          if constexpr (BOW) {
            tap_store(fq);
            __syncthreads();
            tap_gather(gg);
          } else {
            prefix_store<G, MT, T>(gA, gB, fq, wi, tb, li, L::kTrash);
            __syncthreads();
            prefix_gather<ML, T>(gg, gA, gB, rga, rgb);
          }
          __syncthreads();
  #pragma unroll
          for (int r = 0; r < ML; ++r) gg[r] *= ratio;
        }
        const T gr = grp_next<G>(gg[0]);
        T bz[ML];
  #pragma unroll
        for (int r = 0; r < ML; ++r) {
          const T gn = (r + 1 < ML) ? gg[r + 1 < ML ? r + 1 : r] : gr;
          bz[r] = fma(phi2 * Nld, gn - gg[r], fz[r]);
        }
        T nz[ML];
        toeplitz_solve<G, T, ML>(nz, bz, wbz, mask_l, rho_l, itk_l, spl);
        // convergence of this group, from the second sweep on (a string without
        // a longitudinal grid is solved exactly by the first).  Block
        // Gauss-Seidel contracts the error by rho per sweep, and rho is
        // estimated by the ratio of the group's largest updates of the last
        // two sweeps, so the accepted iterate's error is about rho times the
        // last update: converged when that estimate (with rho <= 1/2), or the
        // update itself, is below tol times the group's largest first-sweep
        // value.  A converged group keeps its iterates.
        bool now = nl == 0;
        if (any_l) {
          if (sweep == 0) {
            T amax = T(0);
  #pragma unroll
            for (int r = 0; r < MT; ++r) amax = fmax(amax, fabs(nu[r]));
  #pragma unroll
            for (int r = 0; r < ML; ++r) amax = fmax(amax, fabs(nz[r]));
            const T A = grp_reduce<G, true>(amax);
            // a bowed string stops on the update alone, at 100 tol in FP32 (an
            // update of 1e-5 leaves an error of about rho 1e-5, the FP32 target
            // of the estimate)
            ascale = (T)(bow_stop && sizeof(T) == 4 ? 100.0 * a.tol : a.tol) * A;
            iscale = A > T(0) ? T(1) / A : T(0);
          } else {
            T delta = T(0);
  #pragma unroll
            for (int r = 0; r < MT; ++r) delta = fmax(delta, fabs(nu[r] - au[r]));
  #pragma unroll
            for (int r = 0; r < ML; ++r) delta = fmax(delta, fabs(nz[r] - az[r]));
            const T dmax = grp_reduce<G, true>(delta);
            const T dn = dmax * iscale;
            // (a bowed string stops on the update alone: the stick/slip
            // decision of a chaotic bowed string amplifies the solve's error)
            now = now || dmax <= ascale || (!bow_stop && dn <= T(0.5) * dprev && dn * dn <= (T)a.tol * dprev);
            dprev = dn;
          }
        }
        if (__ballot(conv) != 0) {
  #pragma unroll
          for (int r = 0; r < MT; ++r) au[r] = conv ? au[r] : nu[r];
  #pragma unroll
          for (int r = 0; r < ML; ++r) az[r] = conv ? az[r] : nz[r];
        } else {
  #pragma unroll
          for (int r = 0; r < MT; ++r) au[r] = nu[r];
  #pragma unroll
          for (int r = 0; r < ML; ++r) az[r] = nz[r];
        }
        sweeps = conv ? sweeps : sweep + 1;
        conv = conv || now;
        if (__ballot(!conv) == 0) break;
      }
      return sweeps;
    };
    T au[MT], az[ML];
    bool conv;
    int sweeps = gs_solve(ru, rz, true, au, az, conv);
    if constexpr (BOW) {
      if (any_bow) {
        // bow (eq. 5): the system's response to the unit force J_p(x_B),
        // A [d_u; d_z] = [J_p(x_B); 0], then the step's stick/slip problem
        // v_rel = b - c phi with b = I_p(a_u + 2 v^{n-1/2}) / 2k - v_B and
        // c = k F_B I_p d_u / 2, and a -= k^2 F_B phi d
        const int bn0 = (int)bR[kBowStepN0], bn1 = (int)bR[kBowStepN1];
        const int bn2 = (int)bR[kBowStepN2], bn3 = (int)bR[kBowStepN3];
        const double bw0 = bR[kBowStepW0], bw1 = bR[kBowStepW1], bw2 = bR[kBowStepW2], bw3 = bR[kBowStepW3];
        T fb[MT], du[MT], dz[ML];
#pragma unroll
        for (int r = 0; r < MT; ++r) {
          // J_p = I_p^T / h_t (a node listed once, cubic ghosts folded in by the weights)
          const int i = tb + r + 1;
          fb[r] = ((i == bn0 ? (T)(bw0 * (nt + 1)) : T(0)) + (i == bn1 ? (T)(bw1 * (nt + 1)) : T(0))) +
                  ((i == bn2 ? (T)(bw2 * (nt + 1)) : T(0)) + (i == bn3 ? (T)(bw3 * (nt + 1)) : T(0)));
        }
        bool convd;
        sweeps += gs_solve(fb, zero_l, false, du, dz, convd);
        conv = conv && convd;
        const double Ia =
            point_eval<G, T, MT>(au, zero, bn0, bw0, bn1, bw1) + point_eval<G, T, MT>(au, zero, bn2, bw2, bn3, bw3);
        const double Id =
            point_eval<G, T, MT>(du, zero, bn0, bw0, bn1, bw1) + point_eval<G, T, MT>(du, zero, bn2, bw2, bn3, bw3);
        const double bb = (Ia + 2.0 * bR[kBowStepIv]) / (2.0 * D.k) - bR[kBowStepVB];
        const double c = 0.5 * bR[kBowStepK2F] / D.k * Id;
        const double phi = bow_phi(bb, c, bR[kBowA], bR[kBowEps]);
        const T f = (T)(bR[kBowStepK2F] * phi);
#pragma unroll
        for (int r = 0; r < MT; ++r) au[r] = fma(-f, du[r], au[r]);
#pragma unroll
        for (int r = 0; r < ML; ++r) az[r] = fma(-f, dz[r], az[r]);
      }
    }
    flags |= (act && !conv) ? kFlagNoConverge : 0;
    tot_sw += act ? sweeps : 0;
    max_sw = (act && sweeps > max_sw) ? sweeps : max_sw;

    // ---- state update: v^{n+1/2} = v^{n-1/2} + a, w^{n+1} = w^n + v^{n+1/2} ----
    if constexpr (kSide) {
      side_load<G, MM>(cu, side, 0, li);
      side_load<G, MM>(cvu, side, 1, li);
      side_load<G, MM>(cz, side, 2, li);
      side_load<G, MM>(cvz, side, 3, li);
    }
    if (__ballot(!act) == 0) {
#pragma unroll
      for (int r = 0; r < MT; ++r) {
        kahan_add<T, KAHAN>(vu[r], cvu[r], au[r]);
        update_pos<T, KAHAN>(u[r], cu[r], vu[r], cvu[r]);
      }
#pragma unroll
      for (int r = 0; r < ML; ++r) {
        kahan_add<T, KAHAN>(vz[r], cvz[r], az[r]);
        update_pos<T, KAHAN>(z[r], cz[r], vz[r], cvz[r]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < MT; ++r) {
        T nu_ = u[r], nvu = vu[r], ncu = cu[r], ncvu = cvu[r];
        kahan_add<T, KAHAN>(nvu, ncvu, au[r]);
        update_pos<T, KAHAN>(nu_, ncu, nvu, ncvu);
        u[r] = act ? nu_ : u[r];
        vu[r] = act ? nvu : vu[r];
        cu[r] = act ? ncu : cu[r];
        cvu[r] = act ? ncvu : cvu[r];
      }
#pragma unroll
      for (int r = 0; r < ML; ++r) {
        T nz_ = z[r], nvz = vz[r], ncz = cz[r], ncvz = cvz[r];
        kahan_add<T, KAHAN>(nvz, ncvz, az[r]);
        update_pos<T, KAHAN>(nz_, ncz, nvz, ncvz);
        z[r] = act ? nz_ : z[r];
        vz[r] = act ? nvz : vz[r];
        cz[r] = act ? ncz : cz[r];
        cvz[r] = act ? ncvz : cvz[r];
      }
    }

    if constexpr (kSide) {
      side_save<G, MM>(cu, side, 0, li);
      side_save<G, MM>(cvu, side, 1, li);
      side_save<G, MM>(cz, side, 2, li);
      side_save<G, MM>(cvz, side, 3, li);
    }

    // ---- hammer lumped mass (eq. 6) ----
    if (any_ham) {
      double uH_np1 = 2.0 * uH_n - uH_nm1;
      if (any_sm) {
        const double Iu1 = (double)slot_dot<G, MT, T>(wH, u, cu);
        uH_np1 = (2.0 * uH_n - uH_nm1 - kk * cH * (eta_nm1 - Iu1)) / (1.0 + kk * cH);
      }
      const bool upd = act && ham;
      uH_nm1 = upd ? uH_n : uH_nm1;
      uH_n = upd ? uH_np1 : uH_n;
      eta_nm1 = upd ? eta_n : eta_nm1;
    }

    // ---- readout y^{n+1} = I(x_out) u^{n+1} into the group's ring of G samples ----
    const int64_t m = n + 1;
    const T y = slot_dot<G, MT, T>(wO, u, cu);
    const int slot = (int)((m - first_m) & (G - 1));
    ring = (act && li == slot) ? y : ring;
    // second channel: zeta^{n+1} at x_out on the longitudinal grid
    if constexpr (BOW) {
      if (any_zout) {
        const double yz = point_eval<G, T, ML>(z, cz, D.zon0, D.zon0 ? 1.0 - D.zw : 0.0, D.zon1,
                                               D.zon1 ? D.zw : 0.0);
        ring_z = (act && li == slot) ? (T)yz : ring_z;
      }
    }

    // ---- FP64 energy monitor ----
    bool bad = false;
    const bool mon_now = act && a.mon_period > 0 && mon_ctr == 0;
    if (__ballot(mon_now) != 0) {
      if constexpr (kSide) {
        side_load<G, MM>(cu, side, 0, li);
        side_load<G, MM>(cvu, side, 1, li);
        side_load<G, MM>(cz, side, 2, li);
        side_load<G, MM>(cvz, side, 3, li);
      }
      energy_fill<G, MT, ML, T>(gE, u, vu, cu, cvu, z, vz, cz, cvz, li);
      __syncthreads();
      const double H = energy_fp64<G, MM, T, BOW, CUB>(D, g2k2, gE, li);
      __syncthreads();
      H_last = mon_now ? H : H_last;
      H_step = mon_now ? n : H_step;
      bad = mon_now && (!isfinite(H) || (mon_check && !touched && H_ref > 0.0 && H > H_ref * (1.0 + a.mon_tol)));
      H_ref = mon_now ? H : H_ref;
      touched = mon_now ? 0 : touched;
      flags |= bad ? kFlagUnstable : 0;
    }
    // coalesced burst of G samples per group from first_m + G j: every lane
    // stores; lanes past m write slots a later step overwrites (or the padding
    // after n_samples), never a sample before first_m
    const bool flush = act && (slot == G - 1 || it == nsteps - 1 || bad);
    if (__ballot(flush) != 0) {
      const int64_t idx = flush ? first_m + ((m - first_m) & ~(int64_t)(G - 1)) + li : n_samples + li;
      out[idx] = ring;
      if constexpr (BOW) {
        if (zout) ((T *)D.out_z)[idx] = ring_z;   // same samples and padding as out
      }
    }
    steps_done += act ? 1 : 0;
    nsteps = bad ? it + 1 : nsteps;      // a flagged string stops here
    mon_ctr = mon_ctr + 1 == a.mon_period ? 0 : mon_ctr + 1;
    if constexpr (kPoisonLds) {
      __syncthreads();
      poison_lds<G>(gP, L::kStride, li);
      poison_lds<G>(gE, EnergyLds<G, MM>::kStride, li);
      __syncthreads();
    }
  }

  // ---- write back: every lane stores; an empty group writes to the trash ----
  Status *Sw = present ? S : a.trash_status;
  if constexpr (kSide) {
    side_load<G, MM>(cu, side, 0, li);
    side_load<G, MM>(cvu, side, 1, li);
    side_load<G, MM>(cz, side, 2, li);
    side_load<G, MM>(cvz, side, 3, li);
  }
  store_state<G, T, MT, ML>(present ? st : trash, u, vu, cu, cvu, z, vz, cz, cvz, li);
  Sw->samples_done = done + steps_done;
  Sw->flags = flags;
  Sw->max_sweeps = max_sw;
  Sw->total_sweeps = tot_sw;
  Sw->H_latest = H_last;
  Sw->H_step = H_step;
  Sw->H_ref = H_ref;
  Sw->touched = touched;
  Sw->uH_n = uH_n;
  Sw->uH_nm1 = uH_nm1;
  Sw->eta_nm1 = eta_nm1;
}

// Occupancy target per instantiation: the FP32 classes with up to 6 slots per
// lane (the merged launch) run two wavefronts per SIMD (256 registers each;
// the compiler spills a few hundred bytes per lane, which the second
// wavefront more than pays for); the larger and the FP64 classes keep the
// whole register file (one wavefront per SIMD) because forcing them down
// spills their state.
template <int MM, typename T>
constexpr int kWavesPerEU = (sizeof(T) == 4 && MM <= 6) ? 2 : 1;

// FP32 instantiations step the narrower shapes as well (FP64 batches lay
// every string out with shape 0)
template <typename T>
constexpr bool kShapes = sizeof(T) == 4;

// BOW: the instantiation for tasks with bowed or clamped strings or the
// zeta channel (the host keeps them in work lists of their own); the other
// instantiation has no code for any of them.
template <int G, int MM, typename T, bool KAHAN, bool BOW, bool CUB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<MM, T>))) void step_kernel(
    LaunchArgs a) {
  constexpr int kGroups = kWave / G;
  using L = Lds<G, MM, kLdsArrays<CUB>>;
  // the energy monitor's scratch overlays the stepping arrays (never live together)
  constexpr int kStepDoubles = (kGroups * L::kStride * (int)sizeof(T) + 7) / 8;
  constexpr int kEnergyDoubles = kGroups * EnergyLds<G, MM>::kStride;
  __shared__ double lds[kStepDoubles > kEnergyDoubles ? kStepDoubles : kEnergyDoubles];
  // compensation arrays of the largest class (a separate region: they are
  // read while the energy scratch is written)
  constexpr int kSideDoubles = kSideComp<MM, T, KAHAN> ? (kGroups * 4 * MM * G * (int)sizeof(T) + 7) / 8 : 1;
  __shared__ double lds_side[kSideDoubles];
  // per-lane tables (largest class)
  constexpr int kTabDoubles = (kGroups * TabLds<G, MM, T>::kBytes + 7) / 8;
  __shared__ double lds_tab[kTabDoubles > 0 ? kTabDoubles : 1];
  T *sS = (T *)lds;
  double *sE = lds;
  T *sC = (T *)lds_side;
  T *sTf = (T *)lds_tab;
  uint32_t *sTu = (uint32_t *)(sTf + kGroups * TabLds<G, MM, T>::kWordsT);
  __shared__ double lds_bow[BOW ? kGroups * kBowRec : 1];
  __shared__ T lds_w[2 * MM * kWave];   // per-slot weights of the point interpolants
  for (;;) {
    // every lane takes part; only lane 0 adds, so the wave draws one ticket
    int w = atomicAdd(a.counter, lane_id() == 0 ? 1 : 0);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= a.n_work) break;
    {
      // the ticket names the layout (shape) and its task
      const int m = __builtin_amdgcn_readfirstlane(a.tickets[w]), t = m & 0xffffff;
      switch (m >> 24) {
#define SFD_SHAPE(S)                                                                                             \
  case S:                                                                                                       \
    if constexpr (kShapes<T> && shape_ok(class_of(G, MM), S))                                                   \
      run_task<G, level_slots(MM, (S) / 3), level_slots(MM, (S) % 3), T, KAHAN, BOW, CUB>(                       \
          a, a.part_work[S], t, sS, sE, sC, sTu, sTf, lds_bow, lds_w);                                          \
    break;
        SFD_SHAPE(1)
        SFD_SHAPE(2)
        SFD_SHAPE(3)
        SFD_SHAPE(4)
        SFD_SHAPE(5)
        SFD_SHAPE(6)
        SFD_SHAPE(7)
#undef SFD_SHAPE
        default:
          run_task<G, MM, MM, T, KAHAN, BOW, CUB>(a, a.part_work[0], t, sS, sE, sC, sTu, sTf, lds_bow, lds_w);
          break;
      }
    }
  }
}

// The classes up to 384 points in one persistent launch: one ticket counter
// over their tasks in the order the host chose (estimated work, longest
// first), so that the short tasks fill the tail.  They share the occupancy
// target and need neither LDS tables nor LDS compensation.
template <typename T, bool CUB>
constexpr int small_lds_doubles() {
  constexpr int n = kLdsArrays<CUB>;
  // (the class of 64 lanes and 6 slots needs the most)
  constexpr int a = (Lds<64, 6, n>::kStride * (int)sizeof(T) + 7) / 8, ae = EnergyLds<64, 6>::kStride;
  constexpr int b = (2 * Lds<32, 4, n>::kStride * (int)sizeof(T) + 7) / 8, be = 2 * EnergyLds<32, 4>::kStride;
  constexpr int c = (4 * Lds<16, 4, n>::kStride * (int)sizeof(T) + 7) / 8, ce = 4 * EnergyLds<16, 4>::kStride;
  constexpr int d = (4 * Lds<16, 2, n>::kStride * (int)sizeof(T) + 7) / 8, de = 4 * EnergyLds<16, 2>::kStride;
  constexpr int m1 = a > ae ? a : ae, m2 = b > be ? b : be, m3 = c > ce ? c : ce, m4 = d > de ? d : de;
  constexpr int m12 = m1 > m2 ? m1 : m2, m34 = m3 > m4 ? m3 : m4;
  return m12 > m34 ? m12 : m34;
}

template <typename T, bool KAHAN, bool BOW, bool CUB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<4, T>))) void step_kernel_small(
    LaunchArgs a) {
  static_assert(kWavesPerEU<2, T> == kWavesPerEU<4, T> && kWavesPerEU<6, T> == kWavesPerEU<4, T>,
                "one occupancy target for the merged classes");
  static_assert(!kSideComp<6, T, KAHAN> && !kTabLds<6>, "no LDS tables in the merged classes");
  static_assert(kNumSmall == 5 && class_of(64, 6) == 4, "the merged classes");
  __shared__ double lds[small_lds_doubles<T, CUB>()];
  __shared__ double lds_bow[BOW ? 4 * kBowRec : 1];   // up to four groups per wavefront
  __shared__ T lds_w[2 * 6 * kWave];                    // per-slot weights of the point interpolants
  T *sS = (T *)lds;
  double *sE = lds;
  for (;;) {
    int w = atomicAdd(a.counter, lane_id() == 0 ? 1 : 0);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= a.n_work) break;
    const int m = __builtin_amdgcn_readfirstlane(a.tickets[w]), t = m & 0xffffff;
    // part = class * kNumShapes + shape; FP64 batches use shape 0 only
#define SFD_PART(P, G_, MT_, ML_)                                                                              \
  case P:                                                                                                     \
    if constexpr (kShapes<T> || (P) % kNumShapes == 0)                                                        \
      run_task<G_, MT_, ML_, T, KAHAN, BOW, CUB>(a, a.part_work[P], t, sS, sE, sS, nullptr, nullptr, lds_bow, \
                                                 lds_w);                                                      \
    break;
// the shapes of a class of four slots per lane, parts P0 .. P0 + 7
#define SFD_PARTS4(P0, G_)    \
  SFD_PART(P0, G_, 4, 4)      \
  SFD_PART(P0 + 1, G_, 4, 3)  \
  SFD_PART(P0 + 2, G_, 4, 2)  \
  SFD_PART(P0 + 3, G_, 3, 4)  \
  SFD_PART(P0 + 4, G_, 3, 3)  \
  SFD_PART(P0 + 5, G_, 3, 2)  \
  SFD_PART(P0 + 6, G_, 2, 4)  \
  SFD_PART(P0 + 7, G_, 2, 3)
// the shapes of the class of 64 lanes and six slots per lane (its wider grid
// on six)
#define SFD_PARTS6(P0)         \
  SFD_PART(P0, 64, 6, 6)       \
  SFD_PART(P0 + 1, 64, 6, 4)   \
  SFD_PART(P0 + 2, 64, 6, 3)   \
  SFD_PART(P0 + 3, 64, 4, 6)   \
  SFD_PART(P0 + 6, 64, 3, 6)
    switch (m >> 24) {
      SFD_PARTS6(4 * kNumShapes)
      SFD_PARTS4(3 * kNumShapes, 64)
      SFD_PARTS4(2 * kNumShapes, 32)
      SFD_PARTS4(1 * kNumShapes, 16)
      SFD_PART(2, 16, 2, 1)
      SFD_PART(6, 16, 1, 2)
      default:
        run_task<16, 2, 2, T, KAHAN, BOW, CUB>(a, a.part_work[0], t, sS, sE, sS, nullptr, nullptr, lds_bow, lds_w);
        break;
    }
#undef SFD_PARTS6
#undef SFD_PARTS4
#undef SFD_PART
  }
}

template <typename T, bool KAHAN, bool BOW, bool CUB>
static hipError_t launch_kernel_t(int kernel, const LaunchArgs &a, int blocks, hipStream_t st) {
  switch (kernel) {
    case 0: hipLaunchKernelGGL((step_kernel_small<T, KAHAN, BOW, CUB>), dim3(blocks), dim3(64), 0, st, a); break;
    case 1: hipLaunchKernelGGL((step_kernel<64, 8, T, KAHAN, BOW, CUB>), dim3(blocks), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((step_kernel<64, 10, T, KAHAN, BOW, CUB>), dim3(blocks), dim3(64), 0, st, a); break;
    default: hipLaunchKernelGGL((step_kernel<64, 16, T, KAHAN, BOW, CUB>), dim3(blocks), dim3(64), 0, st, a); break;
  }
  return hipGetLastError();
}

template <typename T, bool KAHAN, bool BOW, bool CUB>
static int blocks_per_cu(int kernel) {
  int n = 0;
  hipError_t e;
  switch (kernel) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel_small<T, KAHAN, BOW, CUB>, 64, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<64, 8, T, KAHAN, BOW, CUB>, 64, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<64, 10, T, KAHAN, BOW, CUB>, 64, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<64, 16, T, KAHAN, BOW, CUB>, 64, 0); break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n;
}

// Host entry points of one instantiation family (element type T,
// compensation KAHAN, the bow family's code BOW, the cubic grid interpolant
// CUB), defined by the translation unit that compiles the family.
#define SFD_STEP_FAMILY(NAME, T, KAHAN, BOW, CUB)                                             \
  hipError_t launch_step_##NAME(int kernel, const LaunchArgs &a, int blocks, hipStream_t st) { \
    return launch_kernel_t<T, KAHAN, BOW, CUB>(kernel, a, blocks, st);                        \
  }                                                                                           \
  int blocks_step_##NAME(int kernel) { return blocks_per_cu<T, KAHAN, BOW, CUB>(kernel); }

}  // namespace sfd
