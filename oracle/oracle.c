/*
 * FP64 CPU oracle: plain, slow, literal implementation of the finite
 * difference scheme of arXiv 2311.18505 ("String Sound Synthesizer on
 * GPU-Accelerated Finite Difference Scheme").
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  Shares nothing with the GPU library.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared oracle.c -lm
 * (FMA contraction off so that results do not depend on the compiler.)
 *
 * Structure, following the paper:
 *   grid          Sec. 3 (t = nk, x = lh) and the spacings of Sec. 3.2
 *   operators     delta/mu operators of eq. (3)-(4) as sparse matrices,
 *                 sized as in the remark after eq. (9)
 *   interpolants  I_(l)->(t), I_(t)->(l) of Sec. 3.1
 *   blocks        Q+-, K^(tl), K^(lt), V, Lambda, G, S, Theta of eq. (9)
 *   recursion     eq. (7)-(8), excitation Gamma of eq. (6) solved jointly
 *                 with the string (Sec. 3.3 / 3.4); the bow of eq. (5) by
 *                 one extra solve A g = [J; 0] and the step's scalar
 *                 stick/slip problem
 * Readings of passages that are silent or inconsistent are marked READING.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Compressed sparse row matrices                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nr, nc, nnz;
    int *rp;      /* nr+1 */
    int *ci;      /* nnz  */
    double *v;    /* nnz  */
} csr;

static csr csr_alloc(int nr, int nc, int nnz) {
    csr a;
    a.nr = nr; a.nc = nc; a.nnz = nnz;
    a.rp = (int *)calloc((size_t)nr + 1, sizeof(int));
    a.ci = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    a.v = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    return a;
}

static void csr_free(csr *a) {
    free(a->rp); free(a->ci); free(a->v);
    a->rp = NULL; a->ci = NULL; a->v = NULL;
}

/* Build from coordinate triplets; duplicates are summed, columns sorted. */
static csr csr_from_coo(int nr, int nc, int n, const int *r, const int *c, const double *v) {
    int *cnt = (int *)calloc((size_t)nr + 1, sizeof(int));
    for (int t = 0; t < n; ++t) cnt[r[t] + 1]++;
    for (int i = 0; i < nr; ++i) cnt[i + 1] += cnt[i];
    int *pos = (int *)malloc(sizeof(int) * (size_t)(nr + 1));
    memcpy(pos, cnt, sizeof(int) * (size_t)(nr + 1));
    int *tc = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *tv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int t = 0; t < n; ++t) {
        int p = pos[r[t]]++;
        tc[p] = c[t]; tv[p] = v[t];
    }
    /* sort each row by column (insertion sort: rows are short) */
    for (int i = 0; i < nr; ++i) {
        for (int p = cnt[i] + 1; p < cnt[i + 1]; ++p) {
            int kc = tc[p]; double kv = tv[p]; int q = p - 1;
            while (q >= cnt[i] && tc[q] > kc) { tc[q + 1] = tc[q]; tv[q + 1] = tv[q]; --q; }
            tc[q + 1] = kc; tv[q + 1] = kv;
        }
    }
    /* merge duplicates */
    int m = 0;
    for (int i = 0; i < nr; ++i)
        for (int p = cnt[i]; p < cnt[i + 1]; ++p)
            if (!(p > cnt[i] && tc[p] == tc[p - 1])) ++m;
    csr a = csr_alloc(nr, nc, m);
    int o = 0;
    for (int i = 0; i < nr; ++i) {
        a.rp[i] = o;
        for (int p = cnt[i]; p < cnt[i + 1]; ++p) {
            if (p > cnt[i] && tc[p] == tc[p - 1]) { a.v[o - 1] += tv[p]; }
            else { a.ci[o] = tc[p]; a.v[o] = tv[p]; ++o; }
        }
    }
    a.rp[nr] = o;
    free(cnt); free(pos); free(tc); free(tv);
    return a;
}

static csr csr_eye(int n, double s) {
    csr a = csr_alloc(n, n, n);
    for (int i = 0; i < n; ++i) { a.rp[i] = i; a.ci[i] = i; a.v[i] = s; }
    a.rp[n] = n;
    return a;
}

static csr csr_diag(int n, const double *d) {
    csr a = csr_alloc(n, n, n);
    for (int i = 0; i < n; ++i) { a.rp[i] = i; a.ci[i] = i; a.v[i] = d[i]; }
    a.rp[n] = n;
    return a;
}

/* C = A * B (structural entries kept even when they cancel to zero) */
static csr csr_mul(const csr *A, const csr *B) {
    int *mark = (int *)malloc(sizeof(int) * (size_t)(B->nc > 0 ? B->nc : 1));
    double *acc = (double *)calloc((size_t)(B->nc > 0 ? B->nc : 1), sizeof(double));
    int *list = (int *)malloc(sizeof(int) * (size_t)(B->nc > 0 ? B->nc : 1));
    for (int j = 0; j < B->nc; ++j) mark[j] = -1;
    /* first pass: count */
    int total = 0;
    for (int i = 0; i < A->nr; ++i) {
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int kk = A->ci[p];
            for (int q = B->rp[kk]; q < B->rp[kk + 1]; ++q) {
                int j = B->ci[q];
                if (mark[j] != i) { mark[j] = i; ++total; }
            }
        }
    }
    for (int j = 0; j < B->nc; ++j) mark[j] = -1;
    csr C = csr_alloc(A->nr, B->nc, total);
    int o = 0;
    for (int i = 0; i < A->nr; ++i) {
        int nl = 0;
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int kk = A->ci[p]; double a = A->v[p];
            for (int q = B->rp[kk]; q < B->rp[kk + 1]; ++q) {
                int j = B->ci[q];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; list[nl++] = j; }
                acc[j] += a * B->v[q];
            }
        }
        /* sort the columns of this row */
        for (int p = 1; p < nl; ++p) {
            int key = list[p]; int q = p - 1;
            while (q >= 0 && list[q] > key) { list[q + 1] = list[q]; --q; }
            list[q + 1] = key;
        }
        C.rp[i] = o;
        for (int p = 0; p < nl; ++p) { C.ci[o] = list[p]; C.v[o] = acc[list[p]]; ++o; }
    }
    C.rp[A->nr] = o;
    free(mark); free(acc); free(list);
    return C;
}

/* C = a*A + b*B (same shape) */
static csr csr_add(double a, const csr *A, double b, const csr *B) {
    int n = A->nnz + B->nnz;
    int *r = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *c = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int t = 0;
    for (int i = 0; i < A->nr; ++i)
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) { r[t] = i; c[t] = A->ci[p]; v[t] = a * A->v[p]; ++t; }
    for (int i = 0; i < B->nr; ++i)
        for (int p = B->rp[i]; p < B->rp[i + 1]; ++p) { r[t] = i; c[t] = B->ci[p]; v[t] = b * B->v[p]; ++t; }
    csr C = csr_from_coo(A->nr, A->nc, t, r, c, v);
    free(r); free(c); free(v);
    return C;
}

static csr csr_scale(double s, const csr *A) {
    csr C = csr_alloc(A->nr, A->nc, A->nnz);
    memcpy(C.rp, A->rp, sizeof(int) * (size_t)(A->nr + 1));
    memcpy(C.ci, A->ci, sizeof(int) * (size_t)(A->nnz > 0 ? A->nnz : 1));
    for (int p = 0; p < A->nnz; ++p) C.v[p] = s * A->v[p];
    return C;
}

static csr csr_transpose(const csr *A) {
    int *r = (int *)malloc(sizeof(int) * (size_t)(A->nnz > 0 ? A->nnz : 1));
    int *c = (int *)malloc(sizeof(int) * (size_t)(A->nnz > 0 ? A->nnz : 1));
    int t = 0;
    for (int i = 0; i < A->nr; ++i)
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) { r[t] = A->ci[p]; c[t] = i; ++t; }
    csr C = csr_from_coo(A->nc, A->nr, t, r, c, A->v);
    free(r); free(c);
    return C;
}

/* y = A x ; adds 2 flops per stored entry to *fl */
static void csr_matvec(const csr *A, const double *x, double *y, double *fl) {
    for (int i = 0; i < A->nr; ++i) {
        double s = 0.0;
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) s += A->v[p] * x[A->ci[p]];
        y[i] = s;
    }
    if (fl) *fl += 2.0 * A->nnz;
}

/* 2x2 block matrix [[A11, A12], [A21, A22]]; NULL blocks are zero.  The
 * row/column sizes are n1 and n2. */
static csr csr_block2(int n1, int n2, const csr *A11, const csr *A12, const csr *A21, const csr *A22) {
    const csr *blk[4] = {A11, A12, A21, A22};
    int n = 0;
    for (int b = 0; b < 4; ++b) if (blk[b]) n += blk[b]->nnz;
    int *r = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *c = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int t = 0;
    for (int b = 0; b < 4; ++b) {
        const csr *M = blk[b];
        if (!M) continue;
        int ro = (b >= 2) ? n1 : 0, co = (b & 1) ? n1 : 0;
        for (int i = 0; i < M->nr; ++i)
            for (int p = M->rp[i]; p < M->rp[i + 1]; ++p) { r[t] = ro + i; c[t] = co + M->ci[p]; v[t] = M->v[p]; ++t; }
    }
    csr C = csr_from_coo(n1 + n2, n1 + n2, t, r, c, v);
    free(r); free(c); free(v);
    return C;
}

/* ------------------------------------------------------------------------ */
/* Banded LU with partial pivoting                                           */
/* ------------------------------------------------------------------------ */

/* Solve M x = rhs.  perm[new] = old gives an ordering of the unknowns in which
 * M is banded; the band is formed from the stored entries and factored by
 * Gaussian elimination with partial pivoting (row interchanges inside the
 * band, fill up to kl above the upper bandwidth).  Adds its arithmetic to *fl,
 * and to *fl_nf what the same elimination costs without the interchanges'
 * fill (row updates and back substitution over the upper bandwidth ku only):
 * W A is symmetric positive definite, so no pivoting is needed in exact
 * arithmetic and that is the method's own count. */
static int band_solve(const csr *M, const int *perm, const double *rhs, double *x, double *fl, double *fl_nf) {
    int n = M->nr;
    int *inv = (int *)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) inv[perm[i]] = i;
    int kl = 0, ku = 0;
    for (int i = 0; i < n; ++i)
        for (int p = M->rp[i]; p < M->rp[i + 1]; ++p) {
            int d = inv[M->ci[p]] - inv[i];
            if (d > ku) ku = d;
            if (-d > kl) kl = -d;
        }
    int W = 2 * kl + ku + 1;           /* row i holds columns i-kl .. i+ku+kl */
    double *a = (double *)calloc((size_t)n * (size_t)W, sizeof(double));
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
#define AB(i, c) a[(size_t)(i) * (size_t)W + (size_t)((c) - (i) + kl)]
    for (int i = 0; i < n; ++i) {
        int ni = inv[i];
        b[ni] = rhs[i];
        for (int p = M->rp[i]; p < M->rp[i + 1]; ++p) AB(ni, inv[M->ci[p]]) += M->v[p];
    }
    int status = ORC_OK;
    double flops = 0.0, flops_nf = 0.0;
    for (int kk = 0; kk < n; ++kk) {
        int last = kk + kl < n - 1 ? kk + kl : n - 1;
        int cmax = kk + ku + kl < n - 1 ? kk + ku + kl : n - 1;
        int umax = kk + ku < n - 1 ? kk + ku : n - 1;
        int piv = kk; double best = fabs(AB(kk, kk));
        for (int r = kk + 1; r <= last; ++r)
            if (fabs(AB(r, kk)) > best) { best = fabs(AB(r, kk)); piv = r; }
        if (best == 0.0) { status = ORC_ESINGULAR; break; }
        if (piv != kk) {
            for (int c = kk; c <= cmax; ++c) { double t = AB(kk, c); AB(kk, c) = AB(piv, c); AB(piv, c) = t; }
            double t = b[kk]; b[kk] = b[piv]; b[piv] = t;
        }
        double pv = AB(kk, kk);
        for (int r = kk + 1; r <= last; ++r) {
            double m = AB(r, kk) / pv;
            flops += 1.0;
            flops_nf += 1.0;
            if (m == 0.0) continue;
            AB(r, kk) = 0.0;
            for (int c = kk + 1; c <= cmax; ++c) AB(r, c) -= m * AB(kk, c);
            b[r] -= m * b[kk];
            flops += 2.0 * (cmax - kk) + 2.0;
            flops_nf += 2.0 * (umax - kk) + 2.0;
        }
    }
    if (status == ORC_OK) {
        double *y = (double *)malloc(sizeof(double) * (size_t)n);
        for (int i = n - 1; i >= 0; --i) {
            int cmax = i + ku + kl < n - 1 ? i + ku + kl : n - 1;
            double s = b[i];
            for (int c = i + 1; c <= cmax; ++c) s -= AB(i, c) * y[c];
            y[i] = s / AB(i, i);
            flops += 2.0 * (cmax - i) + 1.0;
            flops_nf += 2.0 * ((i + ku < n - 1 ? i + ku : n - 1) - i) + 1.0;
        }
        for (int i = 0; i < n; ++i) x[i] = y[inv[i]];
        free(y);
    }
#undef AB
    if (fl) *fl += flops;
    if (fl_nf) *fl_nf += flops_nf;
    free(inv); free(a); free(b);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Grid (Sec. 3 and Sec. 3.2)                                                */
/* ------------------------------------------------------------------------ */

static double theta_of(const orc_string *s) {
    /* Sec. 3.2: theta = (1 + 4/pi^2)/2 */
    return s->theta > 0.0 ? s->theta : 0.5 * (1.0 + 4.0 / (M_PI * M_PI));
}

/* gamma^n = 2 f0(nk) (Sec. 4.1: f0 = gamma/2).  READING (f0 modulation is named
 * in the abstract but not specified): vibrato f0 2^{(d/1200) sin(2 pi f_v t)},
 * or a glide f0 2^{(s/12)(t/T)} linear in semitones over the duration T. */
double orc_gamma_at(const orc_string *s, int64_t n) {
    double t = (double)n / s->fs;
    double f = s->f0;
    if (s->mod_type == 1) {
        f = f * exp2((s->mod_depth_cents / 1200.0) * sin(2.0 * M_PI * s->mod_rate_hz * t));
    } else if (s->mod_type == 2) {
        double T = (double)s->n_samples / s->fs;
        f = f * exp2((s->glide_semitones / 12.0) * (t / T));
    }
    return 2.0 * f;
}

static int clamped_stable(int Nt, double th, double gamma, double kappa, double k);

int orc_grid_plan(const orc_string *s, orc_grid *g) {
    if (!s || !g) return ORC_EINVAL;
    if (!(s->fs > 0.0) || !(s->f0 > 0.0) || !(s->B >= 0.0) || !(s->alpha >= 1.0)) return ORC_EINVAL;
    if (!isfinite(s->fs) || !isfinite(s->f0) || !isfinite(s->B) || !isfinite(s->alpha)) return ORC_EINVAL;
    double th = theta_of(s);
    if (!(th > 0.5) || !(th <= 1.0)) return ORC_EINVAL;
    if (s->boundary != 0 && s->boundary != 1) return ORC_EINVAL;
    if (s->grid_interp != 0 && s->grid_interp != 1 && s->grid_interp != 3) return ORC_EINVAL;
    double k = 1.0 / s->fs;
    double gamma0 = 2.0 * s->f0;
    /* Sec. 4.1: K = (pi kappa / gamma)^2, with K read as the inharmonicity B */
    double kappa = gamma0 * sqrt(s->B) / M_PI;
    double gmax = gamma0;
    if (s->mod_type == 1) gmax = gamma0 * exp2(fabs(s->mod_depth_cents) / 1200.0);
    else if (s->mod_type == 2) gmax = gamma0 * exp2((s->glide_semitones > 0.0 ? s->glide_semitones : 0.0) / 12.0);
    /* READING of the transverse spacing of Sec. 3.2: the printed h^(t) is the
     * bound of the explicit (theta = 1) scheme.  Von Neumann analysis of
     * eq. (4a) with the theta-average gives lambda^2 + 4 nu^2 <= 2 theta - 1,
     * i.e. h^2 >= (g^2k^2 + sqrt(g^4k^4 + 16(2theta-1)kappa^2k^2)) / (2(2theta-1)),
     * which reduces to the printed formula at theta = 1. */
    double gk2 = gmax * gmax * k * k;
    double h2 = (gk2 + sqrt(gk2 * gk2 + 16.0 * (2.0 * th - 1.0) * kappa * kappa * k * k)) / (2.0 * (2.0 * th - 1.0));
    int Nt = s->grid_t > 0 ? s->grid_t : (int)floor(1.0 / sqrt(h2));
    if (s->boundary == 1 && s->grid_t <= 0)
        while (Nt >= 2 && !clamped_stable(Nt, th, gmax, kappa, k)) --Nt;
    int Nl = 0;
    if (s->alpha != 1.0) {
        /* Sec. 3.2: h^(l) = gamma alpha k (bound), N_l = floor(1/h^(l)) */
        Nl = s->grid_l > 0 ? s->grid_l : (int)floor(1.0 / (gmax * s->alpha * k));
        if (Nl < 2) return ORC_EINVAL;
    }
    if (Nt < 2) return ORC_EINVAL;
    g->N_t = Nt; g->N_l = Nl;
    g->h_t = 1.0 / Nt; g->h_l = Nl > 0 ? 1.0 / Nl : 0.0; g->k = k;
    g->gamma0 = gamma0; g->gamma_max = gmax; g->kappa = kappa; g->theta = th;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Operators of eq. (3)-(4), sized as stated after eq. (9)                   */
/* ------------------------------------------------------------------------ */

/* D_{x-}: (N) x (N-1).  (D_{x-} u)_i = (u_i - u_{i-1})/h at the half point
 * x_{i-1/2}, i = 1..N, with the fixed ends u_0 = u_N = 0 (READING: simply
 * supported ends, the (N-1)-sized matrices of eq. (9)). */
static csr op_Dminus(int N, double h) {
    int n = 2 * N, t = 0;
    int *r = (int *)malloc(sizeof(int) * (size_t)n);
    int *c = (int *)malloc(sizeof(int) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    for (int i = 1; i <= N; ++i) {
        if (i <= N - 1) { r[t] = i - 1; c[t] = i - 1; v[t] = 1.0 / h; ++t; }
        if (i - 1 >= 1) { r[t] = i - 1; c[t] = i - 2; v[t] = -1.0 / h; ++t; }
    }
    csr A = csr_from_coo(N, N - 1, t, r, c, v);
    free(r); free(c); free(v);
    return A;
}

/* delta_xxxx of a clamped string: (N-1) x (N-1), the five-point difference
 * (u_{l+2} - 4u_{l+1} + 6u_l - 4u_{l-1} + u_{l-2})/h^4 on the interior nodes,
 * with the ends fixed (u_0 = u_N = 0) and of zero slope, (u_1 - u_{-1})/(2h)
 * = (u_{N+1} - u_{N-1})/(2h) = 0, so the ghost nodes mirror: u_{-1} = u_1 and
 * u_{N+1} = u_{N-1}.  (Sec. 4.1 names the clamped string whose partials eq.
 * (10) gives.) */
static csr op_D4_clamped(int N, double h) {
    static const double stencil[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    int n = 5 * (N - 1), t = 0;
    int *r = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *c = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double h4 = h * h * h * h;
    for (int l = 1; l <= N - 1; ++l) {
        for (int d = -2; d <= 2; ++d) {
            int m = l + d;
            if (m == -1) m = 1;              /* ghost u_{-1} = u_1 */
            if (m == N + 1) m = N - 1;       /* ghost u_{N+1} = u_{N-1} */
            if (m == 0 || m == N) continue;  /* fixed ends */
            r[t] = l - 1; c[t] = m - 1; v[t] = stencil[d + 2] / h4; ++t;   /* duplicates add up */
        }
    }
    csr A = csr_from_coo(N - 1, N - 1, t, r, c, v);
    free(r); free(c); free(v);
    return A;
}

/* mu_{x.}: (N-1) x (N-1), (u_{l+1} + u_{l-1})/2 with u_0 = u_N = 0. */
static csr op_Mx(int N) {
    int n = 2 * (N - 1), t = 0;
    int *r = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *c = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int l = 1; l <= N - 1; ++l) {
        if (l - 1 >= 1) { r[t] = l - 1; c[t] = l - 2; v[t] = 0.5; ++t; }
        if (l + 1 <= N - 1) { r[t] = l - 1; c[t] = l; v[t] = 0.5; ++t; }
    }
    csr A = csr_from_coo(N - 1, N - 1, t, r, c, v);
    free(r); free(c); free(v);
    return A;
}

/* READING of the transverse spacing with clamped ends: the bound in
 * orc_grid_plan comes from the sine modes of simply supported ends.  For any
 * ends, eq. (4a) without loss and nonlinearity keeps a non-negative energy
 * exactly when 4 Theta - k^2 (gamma^2 (-D_xx) + kappa^2 D_xxxx) is positive
 * semi-definite (energy method), so a clamped grid takes the largest N_t, not
 * above the simply supported one, for which that matrix is positive
 * definite: all pivots of its LDL^T factorisation positive (Sylvester). */
static double csr_at(const csr *A, int i, int j) {
    for (int p = A->rp[i]; p < A->rp[i + 1]; ++p)
        if (A->ci[p] == j) return A->v[p];
    return 0.0;
}

static int clamped_stable(int Nt, double th, double gamma, double kappa, double k) {
    int n = Nt - 1;
    double h = 1.0 / Nt;
    csr Dm = op_Dminus(Nt, h);
    csr DmT = csr_transpose(&Dm);
    csr L = csr_mul(&DmT, &Dm);                       /* -D_xx */
    csr D4 = op_D4_clamped(Nt, h);
    csr Kop = csr_add(gamma * gamma, &L, kappa * kappa, &D4);
    csr I = csr_eye(n, 1.0), Mx = op_Mx(Nt);
    csr Th = csr_add(th, &I, 1.0 - th, &Mx);
    csr M = csr_add(4.0, &Th, -k * k, &Kop);
    /* band LDL^T, half-bandwidth 2: l1[i] = L(i, i-1), l2[i] = L(i, i-2) */
    double *d = (double *)calloc((size_t)n + 2, sizeof(double));
    double *l1 = (double *)calloc((size_t)n + 2, sizeof(double));
    int ok = 1;
    for (int i = 0; i < n && ok; ++i) {
        double a2 = i >= 2 ? csr_at(&M, i, i - 2) / d[i - 2] : 0.0;
        double a1 = i >= 1 ? (csr_at(&M, i, i - 1) - (i >= 2 ? a2 * l1[i - 1] * d[i - 2] : 0.0)) / d[i - 1] : 0.0;
        d[i] = csr_at(&M, i, i) - (i >= 1 ? a1 * a1 * d[i - 1] : 0.0) - (i >= 2 ? a2 * a2 * d[i - 2] : 0.0);
        l1[i] = a1;
        ok = d[i] > 0.0;
    }
    free(d); free(l1);
    csr_free(&Dm); csr_free(&DmT); csr_free(&L); csr_free(&D4); csr_free(&Kop);
    csr_free(&I); csr_free(&Mx); csr_free(&Th); csr_free(&M);
    return ok;
}

/* I_(l)->(t): N_t x N_l.  READING of Sec. 3.1 ("p-th order upsampling
 * interpolant", order unstated): Lagrange interpolation of order p = 1
 * (default) or p = 3 from the longitudinal half points (j-1/2)h_l to the
 * transverse half points (i-1/2)h_t.  In units of h_l the t-half point sits
 * at xi = x/h_l + 1/2 (l-half j at xi = j), formed as the exact ratio
 * ((2i-1) N_l + N_t) / (2 N_t); with j0 = floor(xi) and a = xi - j0, p = 1
 * takes j0, j0+1 with weights 1-a, a and p = 3 takes j0-1 .. j0+2 with the
 * cubic Lagrange weights.  Half points past an end stand for their mirror
 * images (p_0 = p_1, p_{-1} = p_2, p_{N_l+1} = p_{N_l}, ...): p = D_x- zeta
 * is even about a fixed end of zeta.  For p = 1 this holds the end values
 * constant outside the outermost half points. */
static csr op_I_lt(int Nt, int Nl, int order) {
    int n = 4 * Nt, t = 0;
    int *r = (int *)malloc(sizeof(int) * (size_t)n);
    int *c = (int *)malloc(sizeof(int) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    for (int i = 1; i <= Nt; ++i) {
        long long num = (long long)(2 * i - 1) * Nl + Nt;
        long long den = 2LL * Nt;
        int j0 = (int)(num / den);
        double a = (double)(num % den) / (double)den;
        int nk = order == 3 ? 4 : 2;
        int first = order == 3 ? j0 - 1 : j0;
        double w[4];
        if (order == 3) {
            w[0] = -a * (a - 1.0) * (a - 2.0) / 6.0;
            w[1] = (a + 1.0) * (a - 1.0) * (a - 2.0) / 2.0;
            w[2] = -(a + 1.0) * a * (a - 2.0) / 2.0;
            w[3] = (a + 1.0) * a * (a - 1.0) / 6.0;
        } else {
            w[0] = 1.0 - a;
            w[1] = a;
        }
        for (int k = 0; k < nk; ++k) {
            int j = first + k;
            if (j < 1) j = 1 - j;                 /* mirror about x = 0 */
            if (j > Nl) j = 2 * Nl + 1 - j;       /* mirror about x = 1 */
            r[t] = i - 1; c[t] = j - 1; v[t] = w[k]; ++t;   /* repeated entries add up */
        }
    }
    csr A = csr_from_coo(Nt, Nl, t, r, c, v);
    free(r); free(c); free(v);
    return A;
}

/* For tests: pt = I_(l)->(t) p (order 1 or 3) on grids of N_t and N_l intervals. */
int orc_apply_I_lt(int Nt, int Nl, int order, const double *p, double *pt) {
    if (Nt < 2 || Nl < 2 || (order != 1 && order != 3) || !p || !pt) return ORC_EINVAL;
    csr A = op_I_lt(Nt, Nl, order);
    csr_matvec(&A, p, pt, NULL);
    csr_free(&A);
    return ORC_OK;
}

/* Interpolation row I_p(x) of Sec. 3.3 on the N-1 interior nodes: READING:
 * linear interpolation between nodes floor(xN) and floor(xN)+1; the fixed
 * end nodes contribute zero. */
static void interp_row(double x, int N, int *idx, double *wt) {
    int l = (int)floor(x * N);
    double w = x * N - l;
    idx[0] = (l >= 1 && l <= N - 1) ? l - 1 : -1;           wt[0] = 1.0 - w;
    idx[1] = (l + 1 >= 1 && l + 1 <= N - 1) ? l : -1;        wt[1] = w;
}

/* Cubic I_3(x) of Sec. 3.3 (the p-th order interpolant with p = 3): Lagrange
 * interpolation through the nodes l-1, l, l+1, l+2 around x = (l + a) h,
 * written on the N-1 interior nodes.  The fixed end nodes contribute zero;
 * a node outside the string stands for its mirror image, u_{-1} = s u_1 and
 * u_{N+1} = s u_{N-1} (s = -1 for simply supported ends, +1 for clamped
 * ones: the same ghosts the boundary conditions give).  Entries of idx are
 * -1 where absent; a node reached twice gets the sum of its weights. */
static void interp_row_cubic(double x, int N, double s, int *idx, double *wt) {
    int l = (int)floor(x * N);
    double a = x * N - l;
    double w[4] = {-a * (a - 1.0) * (a - 2.0) / 6.0, (a + 1.0) * (a - 1.0) * (a - 2.0) / 2.0,
                   -(a + 1.0) * a * (a - 2.0) / 2.0, (a + 1.0) * a * (a - 1.0) / 6.0};
    for (int k = 0; k < 4; ++k) { idx[k] = -1; wt[k] = 0.0; }
    int used = 0;
    for (int k = 0; k < 4; ++k) {
        int m = l - 1 + k;
        double c = w[k];
        if (m == -1) { m = 1; c *= s; }
        if (m == N + 1) { m = N - 1; c *= s; }
        if (m < 1 || m > N - 1) continue;
        int j = 0;
        while (j < used && idx[j] != m - 1) ++j;
        if (j == used) { idx[used] = m - 1; wt[used] = 0.0; ++used; }
        wt[j] += c;
    }
}

static double interp_apply4(const int *idx, const double *wt, const double *u) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k)
        if (idx[k] >= 0) s += wt[k] * u[idx[k]];
    return s;
}

static double interp_apply(const int *idx, const double *wt, const double *u) {
    double s = 0.0;
    if (idx[0] >= 0) s += wt[0] * u[idx[0]];
    if (idx[1] >= 0) s += wt[1] * u[idx[1]];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Precomputed, step-independent operators                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    orc_grid g;
    int nt, nl, n;        /* nt = N_t-1, nl = N_l-1 (0 if none), n = nt+nl */
    csr Dm_t, Dp_t, Dxx_t, Dxxxx_t, Theta, I_t;
    csr Dm_l, Dp_l, Dxx_l, I_l;
    csr I_lt, I_tl;
    csr Qp_t, Qm_t, Qp_l, Qm_l;
    int has_l;
} ops_t;

static void ops_build(const orc_string *s, const orc_grid *g, ops_t *o) {
    memset(o, 0, sizeof(*o));
    o->g = *g;
    int Nt = g->N_t, Nl = g->N_l;
    double k = g->k, th = g->theta;
    o->nt = Nt - 1; o->nl = Nl > 0 ? Nl - 1 : 0; o->n = o->nt + o->nl;
    o->has_l = Nl > 0;
    o->Dm_t = op_Dminus(Nt, g->h_t);
    o->Dp_t = csr_transpose(&o->Dm_t);                   /* D_{x+} = -D_{x-}^T */
    { csr t = csr_scale(-1.0, &o->Dp_t); csr_free(&o->Dp_t); o->Dp_t = t; }
    o->Dxx_t = csr_mul(&o->Dp_t, &o->Dm_t);              /* delta_xx = delta_x+ delta_x- */
    if (s->boundary == 1)
        o->Dxxxx_t = op_D4_clamped(Nt, g->h_t);
    else
        o->Dxxxx_t = csr_mul(&o->Dxx_t, &o->Dxx_t);      /* READING: simply supported, D_xxxx = D_xx^2 */
    o->I_t = csr_eye(o->nt, 1.0);
    {   /* Theta = theta I + (1-theta) M_x (eq. 9) */
        csr M = op_Mx(Nt);
        o->Theta = csr_add(th, &o->I_t, 1.0 - th, &M);
        csr_free(&M);
    }
    /* READING of the loss factor: eq. (4) gives -2 sigma0 delta_t. u +
     * 2 sigma1 delta_t. delta_xx u, i.e. k^2-scaled terms -+ sigma k; the "2"
     * printed inside Q+- of eq. (9) is not used (it would double the loss). */
    {
        csr a = csr_add(1.0, &o->Theta, s->sigma0_t * k, &o->I_t);
        o->Qp_t = csr_add(1.0, &a, -s->sigma1_t * k, &o->Dxx_t);
        csr_free(&a);
        a = csr_add(1.0, &o->Theta, -s->sigma0_t * k, &o->I_t);
        o->Qm_t = csr_add(1.0, &a, s->sigma1_t * k, &o->Dxx_t);
        csr_free(&a);
    }
    if (o->has_l) {
        o->Dm_l = op_Dminus(Nl, g->h_l);
        o->Dp_l = csr_transpose(&o->Dm_l);
        { csr t = csr_scale(-1.0, &o->Dp_l); csr_free(&o->Dp_l); o->Dp_l = t; }
        o->Dxx_l = csr_mul(&o->Dp_l, &o->Dm_l);
        o->I_l = csr_eye(o->nl, 1.0);
        o->I_lt = op_I_lt(Nt, Nl, s->grid_interp == 3 ? 3 : 1);
        /* READING: I_(t)->(l) = (h_t/h_l) I_(l)->(t)^T, the weighted adjoint */
        csr tr = csr_transpose(&o->I_lt);
        o->I_tl = csr_scale(g->h_t / g->h_l, &tr);
        csr_free(&tr);
        csr a = csr_eye(o->nl, 1.0 + s->sigma0_l * k);
        o->Qp_l = csr_add(1.0, &a, -s->sigma1_l * k, &o->Dxx_l);
        csr_free(&a);
        a = csr_eye(o->nl, 1.0 - s->sigma0_l * k);
        o->Qm_l = csr_add(1.0, &a, s->sigma1_l * k, &o->Dxx_l);
        csr_free(&a);
    }
}

static void ops_free(ops_t *o) {
    csr *all[] = {&o->Dm_t, &o->Dp_t, &o->Dxx_t, &o->Dxxxx_t, &o->Theta, &o->I_t,
                  &o->Dm_l, &o->Dp_l, &o->Dxx_l, &o->I_l, &o->I_lt, &o->I_tl,
                  &o->Qp_t, &o->Qm_t, &o->Qp_l, &o->Qm_l};
    for (size_t i = 0; i < sizeof(all) / sizeof(all[0]); ++i)
        if (all[i]->rp) csr_free(all[i]);
}

/* ------------------------------------------------------------------------ */
/* Blocks of eq. (8)-(9) for the state at time n                             */
/* ------------------------------------------------------------------------ */

typedef struct { csr A, B, C; } system_t;

static void system_build(const orc_string *s, const ops_t *o, double gamma, const double *u_n, system_t *sy) {
    const orc_grid *g = &o->g;
    double k = g->k;
    double a2 = s->alpha * s->alpha;
    double G = gamma * gamma * k * k;                    /* G = gamma^2 k^2 D_xx */
    double S = g->kappa * g->kappa * k * k;              /* S = kappa^2 k^2 D_xxxx */
    double phi2 = gamma * gamma * k * k * (a2 - 1.0) / 4.0;   /* phi^2 after eq. (9) */
    int Nt = g->N_t;

    /* Lambda^n = diag(D_{x-} u^n) */
    double *q = (double *)malloc(sizeof(double) * (size_t)Nt);
    csr_matvec(&o->Dm_t, u_n, q, NULL);
    csr Lam = csr_diag(Nt, q);
    csr Lam2 = csr_mul(&Lam, &Lam);

    /* V = -phi^2 D_{x+} Lambda^2 D_{x-} */
    csr t1 = csr_mul(&o->Dp_t, &Lam2);
    csr t2 = csr_mul(&t1, &o->Dm_t);
    csr V = csr_scale(-phi2, &t2);
    csr_free(&t1); csr_free(&t2);

    /* uu blocks */
    csr Auu = csr_add(1.0, &o->Qp_t, 1.0, &V);
    csr Cuu = csr_add(1.0, &o->Qm_t, 1.0, &V);
    csr Buu;
    {
        csr a = csr_add(-2.0, &o->Theta, -G, &o->Dxx_t);
        Buu = csr_add(1.0, &a, S, &o->Dxxxx_t);
        csr_free(&a);
    }
    if (o->has_l) {
        /* READING (Sec. 3.1 / eq. 9 as printed apply the interpolant at the
         * nodes and use I_(l)->(t) in both couplings): the couplings are the
         * discrete forms of the nonlinear terms of eq. (4),
         *   K^(tl) = -phi^2 D_{x+} Lambda I_(l)->(t) D^(l)_{x-}
         *   K^(lt) = -phi^2 D^(l)_{x+} I_(t)->(l) Lambda D_{x-}            */
        csr a = csr_mul(&o->Dp_t, &Lam);
        csr b = csr_mul(&a, &o->I_lt);
        csr c = csr_mul(&b, &o->Dm_l);
        csr Ktl = csr_scale(-phi2, &c);
        csr_free(&a); csr_free(&b); csr_free(&c);
        a = csr_mul(&o->Dp_l, &o->I_tl);
        b = csr_mul(&a, &Lam);
        c = csr_mul(&b, &o->Dm_t);
        csr Klt = csr_scale(-phi2, &c);
        csr_free(&a); csr_free(&b); csr_free(&c);
        csr Ktl2 = csr_scale(2.0, &Ktl);
        csr Bll;
        {
            csr e = csr_eye(o->nl, -2.0);
            Bll = csr_add(1.0, &e, -a2 * G, &o->Dxx_l);
            csr_free(&e);
        }
        /* eq. (8) */
        sy->A = csr_block2(o->nt, o->nl, &Auu, &Ktl, &Klt, &o->Qp_l);
        sy->B = csr_block2(o->nt, o->nl, &Buu, &Ktl2, NULL, &Bll);
        sy->C = csr_block2(o->nt, o->nl, &Cuu, &Ktl, &Klt, &o->Qm_l);
        csr_free(&Ktl); csr_free(&Klt); csr_free(&Ktl2); csr_free(&Bll);
    } else {
        sy->A = csr_scale(1.0, &Auu);
        sy->B = csr_scale(1.0, &Buu);
        sy->C = csr_scale(1.0, &Cuu);
    }
    csr_free(&Auu); csr_free(&Buu); csr_free(&Cuu); csr_free(&V);
    csr_free(&Lam); csr_free(&Lam2);
    free(q);
}

static void system_free(system_t *sy) { csr_free(&sy->A); csr_free(&sy->B); csr_free(&sy->C); }

/* ------------------------------------------------------------------------ */
/* Excitations (Sec. 3.3)                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int on;
    int iH[4]; double wH[4];       /* I_p(x_H) on the transverse nodes (-1: absent) */
    double omega_pow;              /* omega_H^{1+alpha_H} = K_H / M_H   */
    double Mr;                     /* mass ratio M = M_H / (rho A L), L = 1 */
    double aH;
} hammer_t;

static int exc_validate(const orc_excitation *e) {
    if (!e) return ORC_OK;
    if (e->type < 0 || e->type > 3) return ORC_EINVAL;
    if (e->interp_order != 0 && e->interp_order != 1 && e->interp_order != 3) return ORC_EINVAL;
    if (e->type == 0) return ORC_OK;
    if (!(e->x > 0.0 && e->x < 1.0)) return ORC_EINVAL;
    if (e->type == 1 && !isfinite(e->c0)) return ORC_EINVAL;
    if (e->type == 2) {
        if (!(e->M_H > 0.0) || !(e->K_H > 0.0) || !(e->alpha_H >= 1.0) || !(e->rhoA > 0.0)) return ORC_EINVAL;
        if (!isfinite(e->v_H) || !isfinite(e->M_H) || !isfinite(e->K_H) || !isfinite(e->alpha_H)) return ORC_EINVAL;
    }
    if (e->type == 3) {
        if (!(e->x_end > 0.0 && e->x_end < 1.0) || !isfinite(e->v_B) || !(e->F_B >= 0.0) || !isfinite(e->F_B))
            return ORC_EINVAL;
        if (!(e->attack >= 0.0) || !(e->fric_a >= 0.0) || !isfinite(e->fric_a)) return ORC_EINVAL;
        if (!(e->fric_eps >= 0.0 && e->fric_eps <= 1.0)) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Bow (eq. 5)                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int on;
    double t0;                     /* time the bow was set on the string */
    double x0, x1, T;              /* position x0 -> x1 over T seconds from t0 */
    double vB, FB, ta;             /* bow velocity and force, attack time */
    double a, eps;                 /* friction curve */
    int order;                     /* I_p: 1 linear, 3 cubic (Sec. 3.3's p-th order interpolant) */
    double ghost;                  /* sign of the mirrored ghost nodes of the cubic I_p */
} bow_t;

/* Control values at time t.  READING: the paper gives the controls as
 * time-varying without their form; here force and velocity rise linearly
 * over the attack and then hold, and the position moves linearly. */
static void bow_controls(const bow_t *bw, double t, double *x, double *vB, double *FB) {
    t -= bw->t0;
    double r = bw->ta > 0.0 ? (t < bw->ta ? t / bw->ta : 1.0) : 1.0;
    double q = bw->T > 0.0 ? (t < bw->T ? t / bw->T : 1.0) : 0.0;
    *x = bw->x0 + (bw->x1 - bw->x0) * q;
    *vB = bw->vB * r;
    *FB = bw->FB * r;
}

/* The step's scalar problem.  With w* the solution of eq. (7) without the
 * bow and g = A^{-1} [J_p(x_B); 0], the bow adds -k^2 F_B phi g, so
 *     v_rel = I_p(x_B)(u^{n+1} - u^{n-1}) / 2k - v_B = b - c phi,
 *     b = I_p(x_B)(u* - u^{n-1}) / 2k - v_B,   c = k F_B I_p(x_B) g / 2 >= 0.
 * READING (the paper names Newton-Raphson without the treatment of the
 * curve's jump at v_rel = 0, and writes eta for v_rel in phi): phi(0) is any
 * value in [-1, 1] (static friction).  If |b| <= c the string sticks to the
 * bow: v_rel = 0, phi = b/c.  Otherwise it slips with v_rel = sign(b) x, where
 * x in (0, |b|) is the root of h(x) = x + c (eps + (1-eps) e^{-a x}) - |b|.
 * h(0) = c - |b| < 0 and h(|b|) = c (eps + (1-eps) e^{-a|b|}) > 0, and h is
 * convex, so the root is unique; it is found by plain bisection of that
 * bracket until the midpoint no longer moves (full FP64 precision). */
double orc_bow_solve(double b, double c, double a, double eps, double *v) {
    if (!(c > 0.0)) {            /* no bow force */
        *v = b;
        return 0.0;
    }
    if (fabs(b) <= c) {
        *v = 0.0;
        return b / c;
    }
    double sg = b > 0.0 ? 1.0 : -1.0, ab = fabs(b);
    double lo = 0.0, hi = ab;    /* h(lo) < 0 < h(hi) */
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;     /* adjacent doubles */
        double h = mid + c * (eps + (1.0 - eps) * exp(-a * mid)) - ab;
        if (h > 0.0) hi = mid;
        else if (h < 0.0) lo = mid;
        else { lo = hi = mid; break; }
    }
    double x = 0.5 * (lo + hi);
    *v = sg * x;
    return sg * (eps + (1.0 - eps) * exp(-a * x));
}

/* A bow set on the string at level n0 (0 for the initial excitation): its
 * controls run from t0 = n0 k and its position sweep over the rest of the
 * note, (n_samples - n0) / fs. */
static void bow_setup(const orc_excitation *e, const orc_string *s, int64_t n0, bow_t *bw) {
    memset(bw, 0, sizeof(*bw));
    if (!e || e->type != 3) return;
    bw->on = 1;
    bw->t0 = (double)n0 / s->fs;
    bw->x0 = e->x;
    bw->x1 = e->x_end;
    bw->T = (double)(s->n_samples - n0) / s->fs;
    bw->vB = e->v_B;
    bw->FB = e->F_B;
    bw->ta = e->attack;
    bw->a = e->fric_a;
    bw->eps = e->fric_eps;
    bw->order = e->interp_order == 3 ? 3 : 1;
    bw->ghost = s->boundary == 1 ? 1.0 : -1.0;
}

/* Contact coefficient at time n of eq. (6): F_H = c_n (eta^{n+1} + eta^{n-1})
 * with c_n = omega_H^{1+alpha_H} ([eta^n]^+)^{alpha_H - 1} / 2; READING: the
 * power factor is taken at time n, which makes F_H linear in the unknowns,
 * and the contact is open (c_n = 0) for eta^n <= 0. */
static double hammer_c(const hammer_t *hm, double eta_n) {
    if (!(eta_n > 0.0)) return 0.0;
    return 0.5 * hm->omega_pow * pow(eta_n, hm->aH - 1.0);
}

/* ------------------------------------------------------------------------ */
/* Energy                                                                    */
/* ------------------------------------------------------------------------ */

/* H^{n+1/2} of the lossless, unforced scheme from w^{n+1} = (u1, z1) and
 * w^n = (u0, z0): kinetic and linear potential terms of each grid plus the
 * discrete form of the nonlinear potential (gamma^2 (alpha^2-1)/2)
 * (p q^2/2 + q^4/8) built from the pairing q^{n+1} q^n of eq. (4). */
static double energy_half(const orc_string *s, const ops_t *o, double gamma,
                          const double *u1, const double *u0, const double *z1, const double *z0) {
    const orc_grid *g = &o->g;
    double k = g->k, ht = g->h_t, hl = g->h_l;
    int Nt = g->N_t, Nl = g->N_l, nt = o->nt, nl = o->nl;
    double *du = (double *)malloc(sizeof(double) * (size_t)nt);
    double *tdu = (double *)malloc(sizeof(double) * (size_t)nt);
    double *q1 = (double *)malloc(sizeof(double) * (size_t)Nt);
    double *q0 = (double *)malloc(sizeof(double) * (size_t)Nt);
    double *c1 = (double *)malloc(sizeof(double) * (size_t)nt);
    double *c0 = (double *)malloc(sizeof(double) * (size_t)nt);
    for (int i = 0; i < nt; ++i) du[i] = u1[i] - u0[i];
    csr_matvec(&o->Theta, du, tdu, NULL);
    csr_matvec(&o->Dm_t, u1, q1, NULL);
    csr_matvec(&o->Dm_t, u0, q0, NULL);
    csr_matvec(&o->Dxx_t, u1, c1, NULL);
    csr_matvec(&o->Dxx_t, u0, c0, NULL);
    double kin = 0.0, pot = 0.0, stiff = 0.0;
    if (s->boundary == 1) {
        /* clamped: the stiffness energy is u^{n+1} . D_xxxx u^n (D_xxxx is
         * symmetric; with simply supported ends it equals D_xx u^{n+1} . D_xx u^n) */
        csr_matvec(&o->Dxxxx_t, u0, c0, NULL);
        for (int i = 0; i < nt; ++i) { kin += du[i] * tdu[i]; stiff += u1[i] * c0[i]; }
    } else {
        for (int i = 0; i < nt; ++i) { kin += du[i] * tdu[i]; stiff += c1[i] * c0[i]; }
    }
    for (int i = 0; i < Nt; ++i) pot += q1[i] * q0[i];
    double H = ht / (2.0 * k * k) * kin + gamma * gamma * ht / 2.0 * pot + g->kappa * g->kappa * ht / 2.0 * stiff;
    if (o->has_l) {
        double *p1 = (double *)malloc(sizeof(double) * (size_t)Nl);
        double *p0 = (double *)malloc(sizeof(double) * (size_t)Nl);
        double *pt1 = (double *)malloc(sizeof(double) * (size_t)Nt);
        double *pt0 = (double *)malloc(sizeof(double) * (size_t)Nt);
        csr_matvec(&o->Dm_l, z1, p1, NULL);
        csr_matvec(&o->Dm_l, z0, p0, NULL);
        csr_matvec(&o->I_lt, p1, pt1, NULL);
        csr_matvec(&o->I_lt, p0, pt0, NULL);
        double kz = 0.0, pz = 0.0, nlt = 0.0;
        for (int j = 0; j < nl; ++j) { double d = z1[j] - z0[j]; kz += d * d; }
        for (int j = 0; j < Nl; ++j) pz += p1[j] * p0[j];
        for (int i = 0; i < Nt; ++i) {
            double qq = q1[i] * q0[i];
            nlt += qq * qq / 4.0 + qq * (pt1[i] + pt0[i]) / 2.0;
        }
        double a2 = s->alpha * s->alpha;
        H += hl / (2.0 * k * k) * kz + gamma * gamma * a2 * hl / 2.0 * pz + gamma * gamma * (a2 - 1.0) / 2.0 * ht * nlt;
        free(p1); free(p0); free(pt1); free(pt0);
    }
    free(du); free(tdu); free(q1); free(q0); free(c1); free(c0);
    return H;
}

/* ------------------------------------------------------------------------ */
/* Ordering of the unknowns by position (for the banded solve)               */
/* ------------------------------------------------------------------------ */

typedef struct { double x; int kind; int idx; } item_t;

static int item_cmp(const void *a, const void *b) {
    const item_t *p = (const item_t *)a, *q = (const item_t *)b;
    if (p->x < q->x) return -1;
    if (p->x > q->x) return 1;
    if (p->kind != q->kind) return p->kind - q->kind;
    return p->idx - q->idx;
}

static int *position_order(const ops_t *o, int with_hammer, double xH) {
    int n = o->n + (with_hammer ? 1 : 0);
    item_t *it = (item_t *)malloc(sizeof(item_t) * (size_t)n);
    int t = 0;
    for (int i = 0; i < o->nt; ++i) { it[t].x = (double)(i + 1) / o->g.N_t; it[t].kind = 0; it[t].idx = i; ++t; }
    for (int j = 0; j < o->nl; ++j) { it[t].x = (double)(j + 1) / o->g.N_l; it[t].kind = 1; it[t].idx = o->nt + j; ++t; }
    if (with_hammer) { it[t].x = xH; it[t].kind = 2; it[t].idx = o->n; ++t; }
    qsort(it, (size_t)n, sizeof(item_t), item_cmp);
    int *perm = (int *)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) perm[i] = it[i].idx;
    free(it);
    return perm;
}

/* ------------------------------------------------------------------------ */
/* Joint system for (w^{n+1}, u_H^{n+1})                                     */
/* ------------------------------------------------------------------------ */

/* Builds the (n[+1]) x (n[+1]) matrix and right-hand side of eq. (7) at step
 * n, with the hammer of eq. (6) as an extra unknown u_H^{n+1}:
 *   A w^{n+1} - k^2 M J F^n = -B w^n - C w^{n-1}           (Gamma^n = -k^2 [J M F; 0])
 *   u_H^{n+1} - 2u_H^n + u_H^{n-1} = -k^2 F^n              (lumped mass)
 *   F^n = c_n (eta^{n+1} + eta^{n-1}),  eta = u_H - I_p(x_H) u,  J = I_p^T / h.
 * READING: the sign of Gamma follows the statement that the excitation is
 * added to the right-hand side of eq. (4a). */
static csr joint_build(const ops_t *o, const system_t *sy, const hammer_t *hm, double c_n,
                       const double *w_n, const double *w_nm1, double uH_n, double uH_nm1,
                       double *rhs, double *fl) {
    int n = o->n;
    double k = o->g.k;
    double *t1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)n);
    csr_matvec(&sy->B, w_n, t1, fl);
    csr_matvec(&sy->C, w_nm1, t2, fl);
    for (int i = 0; i < n; ++i) rhs[i] = -t1[i] - t2[i];
    free(t1); free(t2);
    if (!hm->on) return csr_scale(1.0, &sy->A);

    double ht = o->g.h_t;
    double eta_nm1 = uH_nm1 - interp_apply4(hm->iH, hm->wH, w_nm1);
    double kc = k * k * c_n;
    /* extra entries: column n (u_H) in the string rows, row n (hammer) */
    int cap = sy->A.nnz + 32;          /* 4 x (1 + 4) string-row entries + 5 hammer-row entries */
    int *r = (int *)malloc(sizeof(int) * (size_t)cap);
    int *c = (int *)malloc(sizeof(int) * (size_t)cap);
    double *v = (double *)malloc(sizeof(double) * (size_t)cap);
    int t = 0;
    for (int i = 0; i < sy->A.nr; ++i)
        for (int p = sy->A.rp[i]; p < sy->A.rp[i + 1]; ++p) { r[t] = i; c[t] = sy->A.ci[p]; v[t] = sy->A.v[p]; ++t; }
    for (int a = 0; a < 4; ++a) {
        if (hm->iH[a] < 0) continue;
        double J = hm->wH[a] / ht;
        /* -k^2 M J c (u_H^{n+1} - I u^{n+1}) moved to the left-hand side */
        r[t] = hm->iH[a]; c[t] = n; v[t] = -k * k * hm->Mr * J * c_n; ++t;
        for (int b = 0; b < 4; ++b) {
            if (hm->iH[b] < 0) continue;
            r[t] = hm->iH[a]; c[t] = hm->iH[b]; v[t] = k * k * hm->Mr * J * c_n * hm->wH[b]; ++t;
        }
        rhs[hm->iH[a]] += k * k * hm->Mr * J * c_n * eta_nm1;
    }
    /* hammer row: (1 + k^2 c) u_H^{n+1} - k^2 c I u^{n+1} = 2u_H^n - u_H^{n-1} - k^2 c eta^{n-1} */
    r[t] = n; c[t] = n; v[t] = 1.0 + kc; ++t;
    for (int b = 0; b < 4; ++b) {
        if (hm->iH[b] < 0) continue;
        r[t] = n; c[t] = hm->iH[b]; v[t] = -kc * hm->wH[b]; ++t;
    }
    rhs[n] = 2.0 * uH_n - uH_nm1 - kc * eta_nm1;
    csr M = csr_from_coo(n + 1, n + 1, t, r, c, v);
    free(r); free(c); free(v);
    return M;
}

/* ------------------------------------------------------------------------ */
/* Driver                                                                    */
/* ------------------------------------------------------------------------ */

static int hammer_setup(const orc_excitation *e, const orc_string *s, const orc_grid *g, hammer_t *hm) {
    memset(hm, 0, sizeof(*hm));
    for (int a = 0; a < 4; ++a) hm->iH[a] = -1;
    if (!e || e->type != 2) return ORC_OK;
    hm->on = 1;
    if (e->interp_order == 3)
        interp_row_cubic(e->x, g->N_t, s->boundary == 1 ? 1.0 : -1.0, hm->iH, hm->wH);
    else
        interp_row(e->x, g->N_t, hm->iH, hm->wH);
    hm->omega_pow = e->K_H / e->M_H;         /* omega_H^{1+alpha_H} */
    hm->Mr = e->M_H / e->rhoA;               /* READING: M = M_H / (rho A L), L = 1 */
    hm->aH = e->alpha_H;
    return ORC_OK;
}

int orc_run(const orc_string *s, const orc_excitation *e, orc_outputs *out) {
    return orc_run_schedule(s, e, 0, NULL, NULL, out);
}

int orc_run_schedule(const orc_string *s, const orc_excitation *e, int n_re, const int64_t *re_step,
                     const orc_excitation *re_exc, orc_outputs *out) {
    if (!s || !out) return ORC_EINVAL;
    orc_grid g;
    int st = orc_grid_plan(s, &g);
    if (st) return st;
    if (!(s->x_out > 0.0 && s->x_out < 1.0) || s->n_samples < 2) return ORC_EINVAL;
    if (s->mod_type < 0 || s->mod_type > 2) return ORC_EINVAL;
    if (!(s->sigma0_t >= 0.0) || !(s->sigma1_t >= 0.0) || !(s->sigma0_l >= 0.0) || !(s->sigma1_l >= 0.0)) return ORC_EINVAL;
    if ((st = exc_validate(e))) return st;
    for (int r = 0; r < n_re; ++r) {
        if (!re_exc || !re_step || re_step[r] < 1 || (r > 0 && re_step[r] <= re_step[r - 1])) return ORC_EINVAL;
        if (re_exc[r].type != 2 && re_exc[r].type != 3) return ORC_EINVAL;
        if ((st = exc_validate(&re_exc[r]))) return st;
    }

    ops_t o;
    ops_build(s, &g, &o);
    hammer_t hm;
    hammer_setup(e, s, &g, &hm);
    bow_t bw;
    bow_setup(e, s, 0, &bw);
    int n = o.n, nt = o.nt, nl = o.nl, Ns = (int)s->n_samples;
    int next_re = 0;
    /* three rotating time levels; each has room for the hammer unknown */
    double *w0 = (double *)calloc((size_t)n + 1, sizeof(double));   /* w^{n-1} */
    double *w1 = (double *)calloc((size_t)n + 1, sizeof(double));   /* w^n     */
    double *w2 = (double *)calloc((size_t)n + 1, sizeof(double));   /* w^{n+1} (+ u_H^{n+1}) */
    double *rhs = (double *)calloc((size_t)n + 1, sizeof(double));
    double *gb = (double *)calloc((size_t)n + 1, sizeof(double));   /* bow: A^{-1} [J_B; 0] */
    double *rb = (double *)calloc((size_t)n + 1, sizeof(double));
    double uH0 = 0.0, uH1 = 0.0;
    int io[2]; double wo[2];
    interp_row(s->x_out, g.N_t, io, wo);
    int iz[2] = {-1, -1}; double wz[2] = {0.0, 0.0};
    if (o.has_l) interp_row(s->x_out, g.N_l, iz, wz);

    /* initial conditions w^0, w^1 */
    if (e && e->type == 1) {
        /* READING of the pluck (Sec. 3.3: "setting an initial condition"):
         * a triangle of peak c0 at x_P, released from rest (u^1 = u^0), zeta = 0 */
        for (int i = 0; i < nt; ++i) {
            double x = (double)(i + 1) / g.N_t;
            double u = x <= e->x ? e->c0 * x / e->x : e->c0 * (1.0 - x) / (1.0 - e->x);
            w0[i] = u; w1[i] = u;
        }
    } else if (e && e->type == 2) {
        /* READING: the hammer starts touching the string at rest with
         * velocity v_H: u_H^0 = 0, u_H^1 = k v_H */
        uH0 = 0.0; uH1 = g.k * e->v_H;
    }
    /* the bow starts on the string at rest (w^0 = w^1 = 0) */
    int *perm = position_order(&o, hm.on, e && e->type == 2 ? e->x : 0.0);

    double flops = 0.0, flops_nf = 0.0;
    /* samples 0 and 1 */
    for (int m = 0; m < 2 && m < Ns; ++m) {
        const double *w = m == 0 ? w0 : w1;
        if (out->y_u) out->y_u[m] = interp_apply(io, wo, w);
        if (out->y_z) out->y_z[m] = o.has_l ? interp_apply(iz, wz, w + nt) : 0.0;
        if (out->traj_u) memcpy(out->traj_u + (size_t)m * nt, w, sizeof(double) * (size_t)nt);
        if (out->traj_z && nl) memcpy(out->traj_z + (size_t)m * nl, w + nt, sizeof(double) * (size_t)nl);
        if (out->u_H) out->u_H[m] = m == 0 ? uH0 : uH1;
    }
    if (out->energy) {
        out->energy[0] = energy_half(s, &o, orc_gamma_at(s, 0), w1, w0, w1 + nt, w0 + nt);
        out->energy[Ns - 1] = 0.0;
    }
    if (out->bow_phi) memset(out->bow_phi, 0, sizeof(double) * (size_t)Ns);
    if (out->bow_vrel) memset(out->bow_vrel, 0, sizeof(double) * (size_t)Ns);
    int status = ORC_OK;
    int64_t steps = 0;
    for (int step = 1; step <= Ns - 2; ++step) {
        if (next_re < n_re && re_step[next_re] == step) {
            /* a new excitation on the sounding string (Sec. 3.3, several
             * excitations per note).  READING: a hammer arrives touching the
             * string at level n-1 and moves with v_H: u_H^{n-1} = I_H u^{n-1},
             * u_H^n = u_H^{n-1} + k v_H (the initial hammer when the string
             * rests); a bow's controls restart from level n-1, so that its
             * first step is n, as step 1 is for the initial bow. */
            const orc_excitation *x = &re_exc[next_re++];
            hammer_setup(x, s, &g, &hm);
            bow_setup(x, s, step - 1, &bw);
            if (hm.on) {
                uH0 = interp_apply4(hm.iH, hm.wH, w0);
                uH1 = uH0 + g.k * x->v_H;
            }
            free(perm);
            perm = position_order(&o, hm.on, x->type == 2 ? x->x : 0.0);
        }
        double gamma = orc_gamma_at(s, step);
        system_t sy;
        system_build(s, &o, gamma, w1, &sy);
        double c_n = 0.0;
        if (hm.on) c_n = hammer_c(&hm, uH1 - interp_apply4(hm.iH, hm.wH, w1));
        double mv = 0.0;
        csr M = joint_build(&o, &sy, &hm, c_n, w1, w0, uH1, uH0, rhs, &mv);
        flops += mv;
        flops_nf += mv;
        status = band_solve(&M, perm, rhs, w2, &flops, &flops_nf);
        if (!status && bw.on) {
            /* eq. (5): Gamma^n = k^2 [J_B F_B phi; 0] (friction against v_rel) */
            double xB, vB, FB;
            bow_controls(&bw, step * g.k, &xB, &vB, &FB);
            /* I_p(x_B) and J_p(x_B) = I_p^T / h_t: linear, or the cubic of the
             * hammer's R21 reading (four nodes, ghosts mirrored with the end
             * condition's sign) */
            int iB[4] = {-1, -1, -1, -1}; double wB[4] = {0.0, 0.0, 0.0, 0.0};
            if (bw.order == 3)
                interp_row_cubic(xB, g.N_t, bw.ghost, iB, wB);
            else
                interp_row(xB, g.N_t, iB, wB);
            memset(rb, 0, sizeof(double) * (size_t)(n + 1));
            for (int a = 0; a < 4; ++a)
                if (iB[a] >= 0) rb[iB[a]] += wB[a] / g.h_t;
            status = band_solve(&M, perm, rb, gb, &flops, &flops_nf);
            if (!status) {
                double c = g.k * FB * interp_apply4(iB, wB, gb) / 2.0;
                double b = (interp_apply4(iB, wB, w2) - interp_apply4(iB, wB, w0)) / (2.0 * g.k) - vB;
                double vrel;
                double phi = orc_bow_solve(b, c, bw.a, bw.eps, &vrel);
                for (int i = 0; i < n; ++i) w2[i] -= g.k * g.k * FB * phi * gb[i];
                if (out->bow_phi) out->bow_phi[step] = phi;
                if (out->bow_vrel) out->bow_vrel[step] = vrel;
            }
        }
        csr_free(&M);
        system_free(&sy);
        if (status) break;
        double uH2 = hm.on ? w2[n] : 0.0;
        int m = step + 1;
        if (out->y_u) out->y_u[m] = interp_apply(io, wo, w2);
        if (out->y_z) out->y_z[m] = o.has_l ? interp_apply(iz, wz, w2 + nt) : 0.0;
        if (out->traj_u) memcpy(out->traj_u + (size_t)m * nt, w2, sizeof(double) * (size_t)nt);
        if (out->traj_z && nl) memcpy(out->traj_z + (size_t)m * nl, w2 + nt, sizeof(double) * (size_t)nl);
        if (out->u_H) out->u_H[m] = uH2;
        if (out->energy) out->energy[step] = energy_half(s, &o, gamma, w2, w1, w2 + nt, w1 + nt);
        /* rotate time levels */
        double *tmp = w0; w0 = w1; w1 = w2; w2 = tmp;
        uH0 = uH1; uH1 = uH2;
        ++steps;
    }
    out->flops = flops;
    out->flops_nofill = flops_nf;
    out->steps_done = steps;
    free(perm); free(w0); free(w1); free(w2); free(rhs); free(gb); free(rb);
    ops_free(&o);
    return status;
}

int orc_dump_system(const orc_string *s, const orc_excitation *e, int64_t step,
                    const double *w_n, const double *w_nm1, double uH_n, double uH_nm1,
                    double *A, double *Bm, double *C, double *rhs) {
    orc_grid g;
    int st = orc_grid_plan(s, &g);
    if (st) return st;
    if ((st = exc_validate(e))) return st;
    ops_t o;
    ops_build(s, &g, &o);
    hammer_t hm;
    hammer_setup(e, s, &g, &hm);
    system_t sy;
    double gamma = orc_gamma_at(s, step);
    system_build(s, &o, gamma, w_n, &sy);
    double c_n = hm.on ? hammer_c(&hm, uH_n - interp_apply4(hm.iH, hm.wH, w_n)) : 0.0;
    int n = o.n, na = n + (hm.on ? 1 : 0);
    double *r = (double *)calloc((size_t)na, sizeof(double));
    csr M = joint_build(&o, &sy, &hm, c_n, w_n, w_nm1, uH_n, uH_nm1, r, NULL);
    if (A) {
        memset(A, 0, sizeof(double) * (size_t)na * (size_t)na);
        for (int i = 0; i < M.nr; ++i)
            for (int p = M.rp[i]; p < M.rp[i + 1]; ++p) A[(size_t)i * na + M.ci[p]] = M.v[p];
    }
    const csr *src[2] = {&sy.B, &sy.C};
    double *dst[2] = {Bm, C};
    for (int m = 0; m < 2; ++m) {
        if (!dst[m]) continue;
        memset(dst[m], 0, sizeof(double) * (size_t)n * (size_t)n);
        for (int i = 0; i < src[m]->nr; ++i)
            for (int p = src[m]->rp[i]; p < src[m]->rp[i + 1]; ++p) dst[m][(size_t)i * n + src[m]->ci[p]] = src[m]->v[p];
    }
    if (rhs) memcpy(rhs, r, sizeof(double) * (size_t)na);
    free(r);
    csr_free(&M);
    system_free(&sy);
    ops_free(&o);
    return ORC_OK;
}
