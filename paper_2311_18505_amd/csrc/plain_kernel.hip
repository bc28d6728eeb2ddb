// Plain FP64 per-string method, the comparator of the batched path: eq. (7)
// of the paper in its position form
//     A^n w^{n+1} = -B^n w^n - C^n w^{n-1} - Gamma^n,
// with the blocks of eq. (8)-(9) (loss as in eq. (4), nonlinear couplings
// K^(tl) = -phi^2 D+ Lambda I_(l)->(t) D-^(l), K^(lt) = -phi^2 D+^(l) I_(t)->(l) Lambda D-),
// and the hammer of eq. (6) as one more unknown u_H^{n+1}; a bow (eq. (5))
// by a second right-hand side [J_p(x_B); 0] carried through the same
// elimination and the step's stick/slip problem.  Every step
// assembles the system in an order that merges both grids and the hammer by
// position along the string (a band matrix), eliminates it row by row
// without pivoting (W A is symmetric positive definite for a positive
// diagonal W) and substitutes back.  One string per launch, one wavefront,
// everything in LDS and FP64: no batching, packing or tuning.
#include <hip/hip_runtime.h>

#include "sfd_types.h"
#include "bow.h"

namespace sfd {

namespace {

struct PlainArgs {
  const Desc *desc;
  Status *status;
  int slot;
  int64_t n_steps;
};

__device__ __forceinline__ int lane() { return (int)threadIdx.x; }

// *p = v where ok, else the value goes to the trash: every lane stores.
__device__ __forceinline__ void put_or_trash(double *p, bool ok, double *trash, double v) { *(ok ? p : trash) = v; }

// (gamma^n k)^2 with gamma^n = 2 f0(nk) (vibrato or glide).
__device__ double plain_g2k2(const Desc &D, int64_t n) {
  const double t = (double)n / D.fs;
  double f = D.f0;
  if (D.mod_type == 1)
    f = f * exp2(D.mod_a * sin(2.0 * M_PI * D.mod_b * t));
  else if (D.mod_type == 2)
    f = f * exp2(D.mod_a * (t / D.mod_b));
  return 4.0 * f * f * D.k * D.k;
}

__global__ __launch_bounds__(64) void plain_kernel(PlainArgs a) {
  HIP_DYNAMIC_SHARED(double, lds)
  const Desc &D = a.desc[a.slot];
  Status *S = a.status + a.slot;
  const int Nt = D.Nt, Nl = D.Nl, nt = D.nt, nl = D.nl, n = D.pn, bw = D.pbw, W = 2 * bw + 1;
  const double Ntd = D.Ntd, Nld = D.Nld, th = D.theta, k = D.k;
  const double s0t = D.s0k_t, s1t = D.s1k_t, s0l = D.s0k_l, s1l = D.s1k_l, ratio = D.ratio_lt;
  const bool ham = D.ham_on != 0;
  const int hn0 = D.hn0, hn1 = D.hn1, ph = D.ph;
  const double hw0 = D.hw0, hw1 = D.hw1;

  double *band = lds;                 // n rows of W: entry (r, c) at r W + c - r + bw
  double *rhs = band + n * W;         // n (+1: trash entry), becomes the solution
  double *trash = rhs + n + 1;        // W: write target of idle lanes
  double *U = trash + W;              // u^n at nodes 0..Nt (ends 0)
  double *Um = U + (Nt + 1);          // u^{n-1}
  double *Z = Um + (Nt + 1);          // zeta^n at nodes 0..Nl
  double *Zm = Z + (Nl + 1);          // zeta^{n-1}
  double *q = Zm + (Nl + 1);          // D- u^n at halves 1..Nt
  double *pt = q + (Nt + 2);          // I_(l)->(t) D- zeta^n
  double *ptm = pt + (Nt + 2);        // I_(l)->(t) D- zeta^{n-1}
  double *cxx = ptm + (Nt + 2);       // D_xx u^n at nodes 0..Nt (ends: from the boundary condition)
  double *gz = cxx + (Nt + 2);        // I_(t)->(l) (q D- u^{n-1}) at l-halves 1..Nl
  double *rhs2 = gz + (Nl + 2);       // bow: n (+1 trash), becomes A^{-1} [J_p(x_B); 0]
  const bool bow = D.bow_on != 0;
  const double bR[kBowRec] = {D.bx0, bow_x_rate(D.bx0, D.bx1, D.bT), D.bT, D.bvB, D.bFB, bow_ramp_rate(D.bta),
                             D.ba, D.beps, 0, 0, 0, 0, 0, 0, 0, D.bt0};

  const int32_t *pos_t = D.ptab, *pos_l = pos_t + nt, *jab = pos_l + nl;
  const int32_t *rga = jab + Nt, *rgb = rga + Nl;
  const double *pw = D.pw;
  double *st = (double *)D.st;        // u^n | u^{n-1} | zeta^n | zeta^{n-1}
  double *out = (double *)D.out;

  // ---- state into LDS ----
  for (int b = 0; b <= Nt; b += 64) {
    const int i = b + lane();
    const bool in = i >= 1 && i <= nt;
    const double u = st[in ? i - 1 : 0], um = st[in ? nt + i - 1 : 0];
    put_or_trash(U + i, i <= Nt, trash, in ? u : 0.0);
    put_or_trash(Um + i, i <= Nt, trash, in ? um : 0.0);
  }
  for (int b = 0; b <= Nl; b += 64) {
    const int j = b + lane();
    const bool in = j >= 1 && j <= nl;
    const double z = st[in ? 2 * nt + j - 1 : 0], zm = st[in ? 2 * nt + nl + j - 1 : 0];
    put_or_trash(Z + j, j <= Nl, trash, in ? z : 0.0);
    put_or_trash(Zm + j, j <= Nl, trash, in ? zm : 0.0);
  }
  int64_t done = S->samples_done;
  int64_t steps = a.n_steps < D.n_samples - done ? a.n_steps : D.n_samples - done;
  if (S->flags != 0 || done < 2 || steps < 0) steps = 0;
  double uH_n = S->uH_n, uH_nm1 = S->uH_nm1;
  int flags = 0;
  int64_t it = 0;
  __syncthreads();

  for (; it < steps; ++it) {
    const int64_t tn = done - 1 + it;   // the step produces w^{tn+1}
    const double G = D.mod_type ? plain_g2k2(D, tn) : D.g2k2_0;
    const double phi2 = G * D.a2m1_4;

    // ---- half-point and node quantities of this step; clear the system ----
    for (int b = 0; b < Nt + 2; b += 64) {
      const int h = b + lane();
      const bool hv = h >= 1 && h <= Nt;
      const int hc = hv ? h : 1;
      const uint32_t ab = nl > 0 ? (uint32_t)jab[hc - 1] : 0x00010001u;
      const int ja = (int)(ab & 0xffffu), jb = (int)(ab >> 16);
      const double w = nl > 0 ? pw[hc - 1] : 0.0;
      const double qq = Ntd * (U[hc] - U[hc - 1]);
      const double p1 = (1.0 - w) * Nld * (Z[ja] - Z[ja - 1]) + w * Nld * (Z[jb] - Z[jb - 1]);
      const double p0 = (1.0 - w) * Nld * (Zm[ja] - Zm[ja - 1]) + w * Nld * (Zm[jb] - Zm[jb - 1]);
      const bool nv = h >= 1 && h <= nt;
      const int ic = nv ? h : 1;
      const double cx = Ntd * Ntd * (U[ic + 1] - 2.0 * U[ic] + U[ic - 1]);
      const bool in = h < Nt + 2;
      // clamped ends: mirrored ghost nodes give D_xx u = 2 u_1 / h^2 at node 0
      // (2 u_{Nt-1} / h^2 at node Nt); simply supported ends give 0
      const bool end = D.clamped != 0 && (h == 0 || h == Nt);
      const double cend = end ? 2.0 * Ntd * Ntd * U[h == 0 ? 1 : Nt - 1] : 0.0;
      put_or_trash(q + h, in, trash, hv ? qq : 0.0);
      put_or_trash(pt + h, in, trash, hv && nl > 0 ? p1 : 0.0);
      put_or_trash(ptm + h, in, trash, hv && nl > 0 ? p0 : 0.0);
      put_or_trash(cxx + h, in, trash, nv ? cx : cend);
    }
    for (int b = 0; b < n * W; b += 64) put_or_trash(band + b + lane(), b + lane() < n * W, trash, 0.0);
    for (int b = 0; b <= n; b += 64) put_or_trash(rhs + b + lane(), b + lane() <= n, trash, 0.0);
    for (int b = 0; b <= n; b += 64) put_or_trash(rhs2 + b + lane(), bow && b + lane() <= n, trash, 0.0);
    // bow: controls at time tn and the interpolant at x_B
    double xB = 0.0, vB = 0.0, FB = 0.0, bw0 = 0.0, bw1 = 0.0;
    int bn0 = 0, bn1 = 0;
    if (bow) {
      bow_controls(bR, (double)tn * k, xB, vB, FB);
      bow_interp(xB, Nt, bn0, bn1, bw0, bw1);
    }
    __syncthreads();
    if (bow && lane() == 0) {
      if (bn0) rhs2[pos_t[bn0 - 1]] += bw0 * Ntd;
      if (bn1) rhs2[pos_t[bn1 - 1]] += bw1 * Ntd;
    }

    // I_(t)->(l)(q D- u^{n-1}) at the l-halves (ranges of t-halves per tap)
    for (int b = 0; b < Nl + 2; b += 64) {
      const int m = b + lane();
      const bool mv = m >= 1 && m <= Nl;
      const uint32_t ra = mv ? (uint32_t)rga[m - 1] : 0u, rb = mv ? (uint32_t)rgb[m - 1] : 0u;
      const int sa = (int)(ra & 0xffffu), na = (int)(ra >> 16), sb = (int)(rb & 0xffffu), nb = (int)(rb >> 16);
      double acc = 0.0;
      for (int c = 0; c < D.gmax; ++c) {
        const int ha = c < na ? sa + c : 1, hb = c < nb ? sb + c : 1;
        const double ta = (1.0 - pw[ha - 1]) * q[ha] * Ntd * (Um[ha] - Um[ha - 1]);
        const double tb = pw[hb - 1] * q[hb] * Ntd * (Um[hb] - Um[hb - 1]);
        acc += (c < na ? ta : 0.0) + (c < nb ? tb : 0.0);
      }
      put_or_trash(gz + m, m < Nl + 2, trash, mv ? ratio * acc : 0.0);
    }

    // hammer: eta^n = u_H^n - I u^n decides the contact coefficient of eq. (6)
    const double eta_n = uH_n - (hw0 * U[hn0] + hw1 * U[hn1]);
    const double eta_nm1 = uH_nm1 - (hw0 * Um[hn0] + hw1 * Um[hn1]);
    const double c_n = (ham && eta_n > 0.0) ? 0.5 * D.omega_pow * pow(eta_n, D.alpha_H - 1.0) : 0.0;
    const double kc = k * k * c_n;
    __syncthreads();

    // ---- transverse rows ----
    for (int b = 0; b < nt; b += 64) {
      const int i = b + lane();
      const bool ok = i < nt;
      const int ii = ok ? i + 1 : 1;    // node 1..nt
      const int r = pos_t[ii - 1];
      double *row = ok ? band + r * W + bw - r : trash + bw;   // row[c] for column position c
      auto put = [&](bool v, int c, double x) {
        double *d = (ok && v) ? row + c : trash;
        *d += x;
      };
      const double qi = q[ii], qn = q[ii + 1];
      put(true, r, th + s0t + 2.0 * s1t + phi2 * Ntd * Ntd * (qi * qi + qn * qn));
      put(ii > 1, pos_t[ii > 1 ? ii - 2 : 0], 0.5 * (1.0 - th) - s1t - phi2 * Ntd * Ntd * qi * qi);
      put(ii < nt, pos_t[ii < nt ? ii : 0], 0.5 * (1.0 - th) - s1t - phi2 * Ntd * Ntd * qn * qn);
      // K^(tl): half h = ii (sign -) and ii + 1 (sign +), two taps each, D-^(l) on the l-nodes
      if (nl > 0) {
        for (int s = 0; s < 2; ++s) {
          const int h = ii + s;
          const double coef = -phi2 * Ntd * (s ? 1.0 : -1.0) * q[h];
          const uint32_t ab = (uint32_t)jab[h - 1];
          const int ja = (int)(ab & 0xffffu), jb = (int)(ab >> 16);
          const double w = pw[h - 1];
          const int js[4] = {ja, ja - 1, jb, jb - 1};
          const double vs[4] = {coef * (1.0 - w) * Nld, -coef * (1.0 - w) * Nld, coef * w * Nld, -coef * w * Nld};
          for (int t = 0; t < 4; ++t) {
            const bool v = js[t] >= 1 && js[t] <= nl;
            put(v, pos_l[v ? js[t] - 1 : 0], vs[t]);
          }
        }
      }
      // hammer block: -k^2 M J c (u_H - I u) on the rows of I_H's nodes
      double rh = 0.0;
      if (ham) {
        for (int t = 0; t < 2; ++t) {
          const int na = t ? hn1 : hn0;
          const double J = (t ? hw1 : hw0) * Ntd;
          const bool on = na != 0 && ii == na;
          const double f = k * k * D.Mr * J * c_n;
          put(on, ph, -f);
          put(on && hn0 != 0, pos_t[hn0 ? hn0 - 1 : 0], f * hw0);
          put(on && hn1 != 0, pos_t[hn1 ? hn1 - 1 : 0], f * hw1);
          rh += on ? f * eta_nm1 : 0.0;
        }
      }
      // right-hand side -B w^n - C w^{n-1}
      const double u = U[ii], ul = U[ii - 1], ur = U[ii + 1];
      const double um = Um[ii], uml = Um[ii - 1], umr = Um[ii + 1];
      const double Bu = -2.0 * (th * u + 0.5 * (1.0 - th) * (ur + ul)) - G * cxx[ii] +
                        D.cS * (cxx[ii + 1] - 2.0 * cxx[ii] + cxx[ii - 1]);
      const double Ktl_n = -phi2 * Ntd * (qn * pt[ii + 1] - qi * pt[ii]);
      const double Ktl_m = -phi2 * Ntd * (qn * ptm[ii + 1] - qi * ptm[ii]);
      const double dmi = Ntd * (um - uml), dmn = Ntd * (umr - um);
      const double Cu = th * um + 0.5 * (1.0 - th) * (umr + uml) - s0t * um + s1t * (umr - 2.0 * um + uml) -
                        phi2 * Ntd * (qn * qn * dmn - qi * qi * dmi);
      rhs[ok ? r : n] = -Bu - 2.0 * Ktl_n - Cu - Ktl_m + rh;
    }
    // ---- longitudinal rows ----
    for (int b = 0; b < nl; b += 64) {
      const int j0 = b + lane();
      const bool ok = j0 < nl;
      const int j = ok ? j0 + 1 : 1;
      const int r = pos_l[j - 1];
      double *row = ok ? band + r * W + bw - r : trash + bw;
      auto put = [&](bool v, int c, double x) {
        double *d = (ok && v) ? row + c : trash;
        *d += x;
      };
      put(true, r, 1.0 + s0l + 2.0 * s1l);
      put(j > 1, pos_l[j > 1 ? j - 2 : 0], -s1l);
      put(j < nl, pos_l[j < nl ? j : 0], -s1l);
      // K^(lt): l-halves m = j + 1 (sign +) and j (sign -), taps over ranges of t-halves
      for (int s = 0; s < 2; ++s) {
        const int m = j + 1 - s;
        const double sg = s ? -1.0 : 1.0;
        const uint32_t ra = (uint32_t)rga[m - 1], rb = (uint32_t)rgb[m - 1];
        for (int tap = 0; tap < 2; ++tap) {
          const uint32_t rr = tap ? rb : ra;
          const int s0 = (int)(rr & 0xffffu), cnt = (int)(rr >> 16);
          for (int c = 0; c < D.gmax; ++c) {
            const bool v = c < cnt;
            const int h = v ? s0 + c : 1;
            const double wt = tap ? pw[h - 1] : 1.0 - pw[h - 1];
            const double coef = -phi2 * Nld * sg * ratio * wt * q[h] * Ntd;
            put(v && h <= nt, pos_t[h <= nt ? h - 1 : 0], coef);
            put(v && h >= 2, pos_t[h >= 2 ? h - 2 : 0], -coef);
          }
        }
      }
      const double z = Z[j], zl = Z[j - 1], zr = Z[j + 1];
      const double zm = Zm[j], zml = Zm[j - 1], zmr = Zm[j + 1];
      const double Bz = -2.0 * z - D.a2 * G * Nld * Nld * (zr - 2.0 * z + zl);
      const double Klt_m = -phi2 * Nld * (gz[j + 1] - gz[j]);
      const double Cz = (1.0 - s0l) * zm + s1l * (zmr - 2.0 * zm + zml);
      rhs[ok ? r : n] = -Bz - Klt_m - Cz;
    }
    // ---- hammer row: (1 + k^2 c) u_H^{n+1} - k^2 c I u^{n+1} = 2 u_H^n - u_H^{n-1} - k^2 c eta^{n-1} ----
    if (ham) {
      band[ph * W + bw] = 1.0 + kc;
      if (hn0) band[ph * W + pos_t[hn0 - 1] - ph + bw] = -kc * hw0;
      if (hn1) band[ph * W + pos_t[hn1 - 1] - ph + bw] = -kc * hw1;
      rhs[ph] = 2.0 * uH_n - uH_nm1 - kc * eta_nm1;
    }
    __syncthreads();

    // ---- elimination without pivoting, right-hand side(s) carried along ----
    const int cols = bw + (bow ? 2 : 1);     // band columns right of the pivot, then rhs (, rhs2)
    const int tasks = bw * cols;
    for (int kk = 0; kk < n - 1; ++kk) {
      const double piv = band[kk * W + bw];
      for (int t0 = 0; t0 < tasks; t0 += 64) {
        const int t = t0 + lane();
        const int ao = t / cols + 1, bo = t % cols + 1;
        const int i = kk + ao;
        const bool ok = t < tasks && i < n;
        const double L = ok ? band[i * W + bw - ao] / piv : 0.0;
        const bool col = bo <= bw, second = bo == bw + 2;
        const bool okc = ok && (col ? kk + bo < n : true);
        const double src = col ? band[kk * W + bw + (col ? bo : 0)] : second ? rhs2[kk] : rhs[kk];
        double *dst = !okc ? trash : col ? band + i * W + bw + bo - ao : second ? rhs2 + i : rhs + i;
        *dst -= L * src;
      }
      __syncthreads();
    }
    // ---- back substitution (every lane computes the same values) ----
    for (int kk = n - 1; kk >= 0; --kk) {
      double s = rhs[kk], s2 = bow ? rhs2[kk] : 0.0;
      for (int bo = 1; bo <= bw; ++bo) {
        const bool in = kk + bo < n;
        const double a_ = in ? band[kk * W + bw + bo] : 0.0;
        s -= a_ * rhs[in ? kk + bo : kk];
        s2 -= bow ? a_ * rhs2[in ? kk + bo : kk] : 0.0;
      }
      const double x = s / band[kk * W + bw], x2 = s2 / band[kk * W + bw];
      __syncthreads();
      rhs[kk] = x;
      put_or_trash(rhs2 + kk, bow, trash, x2);
      __syncthreads();
    }
    // ---- bow: the step's stick/slip problem, then w -= k^2 F_B phi A^{-1} [J; 0] ----
    if (bow) {
      const double Iw = (bn0 ? bw0 * rhs[pos_t[bn0 - 1]] : 0.0) + (bn1 ? bw1 * rhs[pos_t[bn1 - 1]] : 0.0);
      const double Ig = (bn0 ? bw0 * rhs2[pos_t[bn0 - 1]] : 0.0) + (bn1 ? bw1 * rhs2[pos_t[bn1 - 1]] : 0.0);
      const double Ium = bw0 * Um[bn0] + bw1 * Um[bn1];
      const double bb = (Iw - Ium) / (2.0 * k) - vB;
      const double c = 0.5 * k * FB * Ig;
      const double f = k * k * FB * bow_phi(bb, c, D.ba, D.beps);
      __syncthreads();
      for (int b = 0; b < n; b += 64) {
        const int i = b + lane();
        const bool ok = i < n;
        const double v = rhs[ok ? i : 0] - f * rhs2[ok ? i : 0];
        put_or_trash(rhs + i, ok, trash, v);
      }
      __syncthreads();
    }

    // ---- new time level, hammer, readout ----
    for (int b = 0; b < nt; b += 64) {
      const int i = b + lane();
      const bool ok = i < nt;
      const double u = U[ok ? i + 1 : 0], x = rhs[pos_t[ok ? i : 0]];
      put_or_trash(Um + i + 1, ok, trash, u);
      put_or_trash(U + i + 1, ok, trash, x);
    }
    for (int b = 0; b < nl; b += 64) {
      const int j = b + lane();
      const bool ok = j < nl;
      const double z = Z[ok ? j + 1 : 0], x = rhs[pos_l[ok ? j : 0]];
      put_or_trash(Zm + j + 1, ok, trash, z);
      put_or_trash(Z + j + 1, ok, trash, x);
    }
    const double uH_new = ham ? rhs[ph] : 0.0;
    uH_nm1 = uH_n;
    uH_n = uH_new;
    __syncthreads();
    const double y = D.ow0 * U[D.on0] + D.ow1 * U[D.on1];
    out[tn + 1] = y;
    if (!isfinite(y)) {
      flags |= kFlagUnstable;
      ++it;
      break;
    }
  }

  // ---- state back to global memory ----
  __syncthreads();
  for (int b = 0; b < nt; b += 64) {
    const int i = b + lane();
    const bool ok = i < nt;
    // idle lanes rewrite the first element with its own value
    const double u = U[ok ? i + 1 : 1], um = Um[ok ? i + 1 : 1];
    st[ok ? i : 0] = u;
    st[ok ? nt + i : nt] = um;
  }
  for (int b = 0; b < nl; b += 64) {
    const int j = b + lane();
    const bool ok = j < nl;
    const double z = Z[ok ? j + 1 : 1], zm = Zm[ok ? j + 1 : 1];
    st[ok ? 2 * nt + j : 2 * nt] = z;
    st[ok ? 2 * nt + nl + j : 2 * nt + nl] = zm;
  }
  S->samples_done = done + it;
  S->flags = flags;
  S->uH_n = uH_n;
  S->uH_nm1 = uH_nm1;
}

}  // namespace

hipError_t launch_plain(const Desc *d_desc, Status *d_status, int slot, int64_t n_steps, size_t lds_bytes,
                        hipStream_t st) {
  PlainArgs a{d_desc, d_status, slot, n_steps};
  hipLaunchKernelGGL(plain_kernel, dim3(1), dim3(64), lds_bytes, st, a);
  return hipGetLastError();
}

}  // namespace sfd
