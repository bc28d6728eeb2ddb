/*
 * FP64 CPU oracle for the planar nonlinear stiff lossy string scheme of
 * "String Sound Synthesizer on GPU-Accelerated Finite Difference Scheme"
 * (Lee, Choi, Lee; arXiv 2311.18505).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the tests, the smoke check and the CPU baseline of the benchmark compare
 * the GPU library against.  It shares no code, header, table or constant
 * with the GPU path, and no product code may call it.
 *
 * It steps the matrix-vector recursion of eq. (7),
 *     A^n w^{n+1} + B^n w^n + C^n w^{n-1} + Gamma^n = 0,
 * with the blocks of eq. (8)-(9) assembled literally from sparse operator
 * matrices each step, and solves for w^{n+1} with a banded LU (partial
 * pivoting) after ordering the unknowns of both grids by position.  The
 * bow's scalar stick/slip problem is solved by bisection.
 *
 * Units: the string is normalised to length L = 1 (positions are fractions
 * of L), displacements are in metres, time in seconds.
 */
#ifndef STRING_ORACLE_H
#define STRING_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double fs;            /* sample rate; k = 1/fs (Sec. 3) */
    double f0;            /* fundamental of the ideal string, gamma = 2 f0 (Sec. 4.1) */
    double B;             /* inharmonicity K = (pi kappa/gamma)^2 (Sec. 4.1) */
    double alpha;         /* stiffness-to-tension ratio (Table 1), >= 1 */
    double theta;         /* theta-scheme parameter (Sec. 3.2); <= 0 selects (1+4/pi^2)/2 */
    double sigma0_t, sigma1_t, sigma0_l, sigma1_l;   /* losses of eq. (4) */
    double x_out;         /* readout position in (0,1) */
    int64_t n_samples;    /* number of output samples y^0 .. y^{n_samples-1} */
    int32_t mod_type;     /* 0 none, 1 vibrato, 2 linear glide (in semitones) */
    int32_t grid_t;       /* 0: N_t from the stability bound; else forced N_t */
    double mod_depth_cents, mod_rate_hz, glide_semitones;
    int32_t grid_l;       /* 0: N_l from h_l >= gamma alpha k; else forced N_l */
    int32_t boundary;     /* transverse ends: 0 simply supported, 1 clamped (Sec. 4.1, eq. 10) */
    int32_t grid_interp;  /* order p of I_(l)->(t) (Sec. 3.1's p-th order interpolant): 0 or 1 linear, 3 cubic */
} orc_string;

typedef struct {
    int32_t type;         /* 0 none, 1 pluck (initial condition), 2 hammer (eq. 6), 3 bow (eq. 5) */
    int32_t interp_order; /* I_p of the hammer or the bow: 0 or 1 linear, 3 cubic (Sec. 3.3's p-th order interpolant) */
    double x;             /* excitation position in (0,1); the bow's position at t = 0 */
    double c0;            /* pluck peak displacement [m] */
    double v_H;           /* hammer initial velocity [m/s] */
    double M_H;           /* hammer mass [kg] */
    double K_H;           /* hammer felt stiffness [N/m^alpha_H] */
    double alpha_H;       /* hammer nonlinear exponent */
    double rhoA;          /* string linear mass density [kg/m] */
    /* bow (eq. 5): position x -> x_end linearly over the note (T = n_samples/fs),
     * bow velocity v_B [m/s] and force F_B (per unit linear density, m/s^2 on
     * the normalised string) rising linearly over `attack` seconds; friction
     * curve phi(v) = sign(v) (eps + (1 - eps) exp(-a |v|)) */
    double x_end, v_B, F_B, attack, fric_a, fric_eps;
} orc_excitation;

typedef struct {
    int32_t N_t, N_l;     /* intervals of the transverse / longitudinal grids (N_l = 0: no zeta) */
    double h_t, h_l, k;
    double gamma0, gamma_max, kappa, theta;
} orc_grid;

typedef struct {
    /* every pointer may be NULL; sizes in doubles */
    double *y_u;          /* [n_samples]  readout I(x_out) u^n                         */
    double *y_z;          /* [n_samples]  readout I(x_out) zeta^n on the l-grid        */
    double *energy;       /* [n_samples]  energy[n] = H^{n+1/2}, n = 0..n_samples-2    */
    double *traj_u;       /* [n_samples*(N_t-1)] full transverse trajectory           */
    double *traj_z;       /* [n_samples*(N_l-1)] full longitudinal trajectory          */
    double *u_H;          /* [n_samples]  hammer displacement                          */
    double flops;         /* out: floating point operations of the RHS matvecs and the
                             banded factor/solve (the direct method's arithmetic)     */
    int64_t steps_done;   /* out: number of recursion steps taken                      */
    double *bow_phi;      /* [n_samples]  bow: friction value phi used at step n        */
    double *bow_vrel;     /* [n_samples]  bow: relative velocity v_rel at step n        */
    double flops_nofill;  /* out: the same arithmetic with the banded elimination kept
                             inside the band (no row interchanges, which W A being
                             symmetric positive definite makes unnecessary)          */
} orc_outputs;

/* status codes */
#define ORC_OK        0
#define ORC_EINVAL   -1
#define ORC_ENOMEM   -2
#define ORC_ESINGULAR -3

int orc_grid_plan(const orc_string *s, orc_grid *g);
int orc_run(const orc_string *s, const orc_excitation *e, orc_outputs *out);

/* The same with n_re more excitations (hammer or bow) applied to the sounding
 * string: re_exc[r] before the step that computes w^{re_step[r]+1}
 * (re_step increasing, >= 1).  A hammer arrives touching the string at level
 * n-1 with velocity v_H; a bow's controls restart from level n-1 (its first
 * step is n, as step 1 is for the initial bow). */
int orc_run_schedule(const orc_string *s, const orc_excitation *e, int n_re, const int64_t *re_step,
                     const orc_excitation *re_exc, orc_outputs *out);

/* Assemble A^n, B^n, C^n (eq. 8-9, hammer block included) for a given state and
 * return them densely (row-major, size n x n with n = N_t-1 + N_l-1) together
 * with the right-hand side -B w^n - C w^{n-1} - Gamma^n.  For tests only. */
int orc_dump_system(const orc_string *s, const orc_excitation *e, int64_t n,
                    const double *w_n, const double *w_nm1, double uH_n, double uH_nm1,
                    double *A, double *Bm, double *C, double *rhs);

/* For tests: pt[0..N_t) = I_(l)->(t) p[0..N_l) (Sec. 3.1's p-th order
 * interpolant, order 1 or 3, the same operator the scheme assembles). */
int orc_apply_I_lt(int Nt, int Nl, int order, const double *p, double *pt);

/* gamma^n = 2 f0(n k) under the modulation of the string (Sec. 1 abstract). */
double orc_gamma_at(const orc_string *s, int64_t n);

/* The bow's scalar problem of one step (eq. 5): v = b - c phi with phi the
 * friction curve at v (slip, v != 0) or any value in [-1, 1] at v = 0
 * (stick).  Returns phi and stores v. */
double orc_bow_solve(double b, double c, double a, double eps, double *v);

#ifdef __cplusplus
}
#endif
#endif
