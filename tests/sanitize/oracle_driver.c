/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * every entry point of oracle.h on short strings that reach its branches
 * (pluck, linear and cubic hammer, bow with the cubic I_p, clamped ends,
 * the cubic grid interpolant, f0 modulation, restrikes, the dumped system,
 * invalid parameters).  Prints one line per case, "name status steps
 * sum(y_u) sum(energy)", compared by tests/test_sanitizers.py with the same
 * cases run through the uninstrumented oracle. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static orc_string base_string(double f0, double B, double alpha, int64_t n) {
    orc_string s;
    memset(&s, 0, sizeof(s));
    s.fs = 48000.0;
    s.f0 = f0;
    s.B = B;
    s.alpha = alpha;
    s.sigma0_t = 1.0;
    s.sigma1_t = 3e-4;
    s.sigma0_l = 1.0;
    s.sigma1_l = 3e-4;
    s.x_out = 0.3;
    s.n_samples = n;
    return s;
}

static orc_excitation pluck(double x, double c0) {
    orc_excitation e;
    memset(&e, 0, sizeof(e));
    e.type = 1;
    e.x = x;
    e.c0 = c0;
    return e;
}

static orc_excitation hammer(double x, double v, int order) {
    orc_excitation e;
    memset(&e, 0, sizeof(e));
    e.type = 2;
    e.interp_order = order;
    e.x = x;
    e.v_H = v;
    e.M_H = 4.9e-3;
    e.K_H = 4.5e9;
    e.alpha_H = 2.5;
    e.rhoA = 6.3e-3;
    return e;
}

static orc_excitation bow(double x, double x_end, int order) {
    orc_excitation e;
    memset(&e, 0, sizeof(e));
    e.type = 3;
    e.interp_order = order;
    e.x = x;
    e.x_end = x_end;
    e.v_B = 0.1;
    e.F_B = 100.0;
    e.attack = 0.002;
    e.fric_a = 100.0;
    e.fric_eps = 0.2;
    return e;
}

static void report(const char *name, const orc_string *s, int st, const orc_outputs *o) {
    double sy = 0.0, se = 0.0;
    if (st == ORC_OK) {
        for (int64_t i = 0; i < s->n_samples; ++i) sy += o->y_u[i];
        for (int64_t i = 0; i + 1 < s->n_samples; ++i) se += o->energy[i];
    }
    printf("%s %d %lld %.17g %.17g\n", name, st, (long long)o->steps_done, sy, se);
}

static void run_case(const char *name, const orc_string *s, const orc_excitation *e) {
    orc_outputs o;
    memset(&o, 0, sizeof(o));
    o.y_u = calloc((size_t)s->n_samples, sizeof(double));
    o.y_z = calloc((size_t)s->n_samples, sizeof(double));
    o.energy = calloc((size_t)s->n_samples, sizeof(double));
    o.u_H = calloc((size_t)s->n_samples, sizeof(double));
    o.bow_phi = calloc((size_t)s->n_samples, sizeof(double));
    o.bow_vrel = calloc((size_t)s->n_samples, sizeof(double));
    const int st = orc_run(s, e, &o);
    report(name, s, st, &o);
    free(o.y_u);
    free(o.y_z);
    free(o.energy);
    free(o.u_H);
    free(o.bow_phi);
    free(o.bow_vrel);
}

int main(void) {
    const int64_t n = 400;
    orc_string s = base_string(110.0, 1e-4, 1.5, n);
    orc_excitation e = pluck(0.27, 1e-3);
    run_case("pluck", &s, &e);

    s = base_string(220.0, 3e-4, 2.5, n);
    e = hammer(0.12, 2.0, 1);
    run_case("hammer_linear", &s, &e);
    e = hammer(0.02, 2.0, 3);
    run_case("hammer_cubic_end", &s, &e);

    s = base_string(196.0, 1e-4, 1.0, n);
    e = bow(0.12, 0.2, 3);
    run_case("bow_cubic", &s, &e);
    s.alpha = 2.0;
    e = bow(0.015, 0.05, 1);
    run_case("bow_linear_nonlinear", &s, &e);

    s = base_string(80.0, 2e-4, 2.0, n);
    s.boundary = 1;
    e = hammer(0.11, 3.0, 3);
    run_case("clamped_hammer", &s, &e);

    s = base_string(300.0, 1e-3, 3.0, n);
    s.grid_interp = 3;
    e = pluck(0.14, 0.02);
    run_case("cubic_grid", &s, &e);

    s = base_string(150.0, 1e-4, 1.7, n);
    s.mod_type = 1;
    s.mod_depth_cents = 25.0;
    s.mod_rate_hz = 6.0;
    e = pluck(0.3, 1e-3);
    run_case("vibrato", &s, &e);
    s.mod_type = 2;
    s.glide_semitones = -2.0;
    run_case("glide", &s, &e);

    /* restrikes: a hammer, then a second hammer and a bow while sounding */
    s = base_string(130.0, 1e-4, 1.6, n);
    e = hammer(0.13, 1.5, 1);
    {
        const int64_t at[2] = {120, 260};
        orc_excitation re[2];
        re[0] = hammer(0.2, 1.0, 3);
        re[1] = bow(0.1, 0.15, 1);
        orc_outputs o;
        memset(&o, 0, sizeof(o));
        o.y_u = calloc((size_t)n, sizeof(double));
        o.energy = calloc((size_t)n, sizeof(double));
        const int st = orc_run_schedule(&s, &e, 2, at, re, &o);
        report("restrike", &s, st, &o);
        free(o.y_u);
        free(o.energy);
    }

    /* the assembled system of one step */
    {
        orc_grid g;
        s = base_string(200.0, 1e-4, 2.0, n);
        int st = orc_grid_plan(&s, &g);
        const int m = (g.N_t - 1) + (g.N_l - 1);
        double *w = calloc((size_t)m, sizeof(double)), *w1 = calloc((size_t)m, sizeof(double));
        double *A = calloc((size_t)m * m, sizeof(double)), *Bm = calloc((size_t)m * m, sizeof(double));
        double *C = calloc((size_t)m * m, sizeof(double)), *r = calloc((size_t)m, sizeof(double));
        for (int i = 0; i < m; ++i) {
            w[i] = 1e-4 * sin(0.37 * i);
            w1[i] = 0.9 * w[i];
        }
        e = pluck(0.3, 1e-3);
        if (st == ORC_OK) st = orc_dump_system(&s, &e, 5, w, w1, 0.0, 0.0, A, Bm, C, r);
        double sa = 0.0;
        for (int i = 0; i < m * m; ++i) sa += A[i] + Bm[i] + C[i];
        printf("dump_system %d %d %.17g 0\n", st, m, sa);
        free(w);
        free(w1);
        free(A);
        free(Bm);
        free(C);
        free(r);
    }

    /* the grid interpolant and the scalar bow solve */
    {
        /* p on the 40 l-half points, pt on the 60 t-half points */
        double p[40], pt[60];
        for (int i = 0; i < 40; ++i) p[i] = cos(0.2 * i);
        const int st = orc_apply_I_lt(60, 40, 3, p, pt);
        double sp = 0.0;
        for (int i = 0; i < 60; ++i) sp += pt[i];
        printf("apply_I_lt %d 0 %.17g 0\n", st, sp);
        double v = 0.0;
        const double phi = orc_bow_solve(-0.3, 0.05, 100.0, 0.2, &v);
        printf("bow_solve 0 0 %.17g %.17g\n", phi, v);
    }

    /* invalid parameters are refused */
    s = base_string(110.0, 1e-4, 0.5, n);
    e = pluck(0.27, 1e-3);
    run_case("invalid_alpha", &s, &e);
    s = base_string(NAN, 1e-4, 1.5, n);
    run_case("invalid_f0", &s, &e);
    s = base_string(110.0, 1e-4, 1.5, n);
    e = pluck(1.0, 1e-3);
    run_case("invalid_position", &s, &e);
    return 0;
}
