/*
 * sanitize_main.c -- TEST INFRASTRUCTURE ONLY.  A host program that steps
 * the FP64 oracle (lb_oracle.c) through every mode it implements, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitizers.py compiles and runs it with gcc).  It
 * checks nothing numerically beyond finiteness and mass bookkeeping; the
 * sanitizers do the checking: any out-of-bounds access, leak, use after
 * free or undefined operation aborts the run.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_channel orc_channel;
typedef struct orc_qgrid orc_qgrid;

orc_channel *orc_create(int lx, int ly, double tau_lb, double g_inf, double tau_m,
                        double gamma_c, int n_hist, double gx, double gy, const double *u0);
void orc_destroy(orc_channel *c);
void orc_set_force(orc_channel *c, double gx, double gy);
int orc_set_history_grid(orc_channel *c, int B, int C);
int orc_set_finger(orc_channel *c);
int orc_set_paper_coupling(orc_channel *c);
int orc_trace_prev(const orc_channel *c, double *out);
int orc_set_law(orc_channel *c, int law);
void orc_step(orc_channel *c, long n_steps);
int orc_fields(const orc_channel *c, double *rho, double *ux, double *uy);
int orc_stress(const orc_channel *c, double *sxy, double *n1);
int orc_grad(const orc_channel *c, double *kappa);
double orc_mass(const orc_channel *c);
void orc_get_state(const orc_channel *c, double *n, double *sig_xy, double *sig_xx,
                   double *ring_s, double *ring_r, double *ring_g, double *gam, long *t);
void orc_set_state(orc_channel *c, const double *n, const double *sig_xy,
                   const double *sig_xx, const double *ring_s, const double *ring_r,
                   const double *ring_g, const double *gam, long t);
orc_qgrid *orc_qgrid_create(int B, int C);
void orc_qgrid_destroy(orc_qgrid *g);
void orc_qgrid_push(orc_qgrid *g, long t, double kxx, double kxy, double kyx, double kyy);
int orc_qgrid_capacity(const orc_qgrid *g);
int orc_qgrid_entries(const orc_qgrid *g, double *t0, double *dt, double *k4, double *strain);
void orc_qgrid_sum(const orc_qgrid *g, long t, double g_inf, double tau_m, double gamma_c,
                   double *sxy, double *n1);
void orc_expm2(const double *A, double *out);

static int failures = 0;

static void check_outputs(const char *mode, orc_channel *c, int lx, int ly)
{
    const int N = lx * ly;
    double *buf = (double *)malloc(sizeof(double) * 9 * (size_t)N);
    if (orc_fields(c, buf, buf + N, buf + 2 * N) != 0 || orc_stress(c, buf + 3 * N, buf + 4 * N) != 0 ||
        orc_grad(c, buf + 5 * N) != 0) {
        printf("%s: readout refused\n", mode);
        failures++;
    }
    for (int k = 0; k < 9 * N; ++k)
        if (!isfinite(buf[k])) {
            printf("%s: non-finite output at %d\n", mode, k);
            failures++;
            break;
        }
    free(buf);
}

/* mode: 0 nlM, 1 UCM, 2 grid, 3 full tensor, 4 paper coupling,
 * 5 accumulated-strain damping, 6 instantaneous law */
static void run_mode(int mode, const char *name)
{
    const int lx = 4, ly = 9, H = 24, steps = 60;
    double *u0 = (double *)calloc(2 * (size_t)lx * ly, sizeof(double));
    for (int k = 0; k < 2 * lx * ly; ++k)
        u0[k] = 1e-3 * sin(0.7 * k + 0.3);
    const double gamma_c = mode == 1 ? INFINITY : 0.1;
    orc_channel *c = orc_create(lx, ly, 0.9, 2e-3, 30.0, gamma_c, H, 2e-5, 1e-6, u0);
    if (!c) {
        printf("%s: create failed\n", name);
        failures++;
        free(u0);
        return;
    }
    int rc = 0;
    if (mode == 2)
        rc = orc_set_history_grid(c, 3, 8);
    else if (mode == 3)
        rc = orc_set_finger(c);
    else if (mode == 4)
        rc = orc_set_paper_coupling(c);
    else if (mode == 5)
        rc = orc_set_law(c, 1);
    else if (mode == 6)
        rc = orc_set_law(c, 2);
    if (rc != 0) {
        printf("%s: mode switch refused\n", name);
        failures++;
    }
    const double m0 = orc_mass(c);
    orc_step(c, steps / 2);
    orc_set_force(c, 0.0, 0.0);
    orc_step(c, steps / 2);
    check_outputs(name, c, lx, ly);
    if (mode == 4) {
        double *tr = (double *)malloc(sizeof(double) * lx * ly);
        if (orc_trace_prev(c, tr) != 0)
            failures++;
        free(tr);
    } else if (fabs(orc_mass(c) - m0) > 1e-12 * m0) {
        printf("%s: mass not conserved\n", name);
        failures++;
    }
    if (mode == 0 || mode == 1) {
        /* state round trip, then more steps */
        const size_t N = (size_t)lx * ly, R = (size_t)H * N;
        double *n = malloc(sizeof(double) * 9 * N), *sxy = malloc(sizeof(double) * N),
               *sxx = malloc(sizeof(double) * N), *rs = malloc(sizeof(double) * R),
               *rr = malloc(sizeof(double) * R), *rg = malloc(sizeof(double) * R),
               *gam = malloc(sizeof(double) * N);
        long t = 0;
        orc_get_state(c, n, sxy, sxx, rs, rr, rg, gam, &t);
        orc_set_state(c, n, sxy, sxx, rs, rr, rg, gam, t);
        if (orc_fields(c, n, NULL, NULL) != -1) {
            printf("%s: readout allowed after a state load\n", name);
            failures++;
        }
        orc_step(c, 5);
        check_outputs(name, c, lx, ly);
        free(n), free(sxy), free(sxx), free(rs), free(rr), free(rg), free(gam);
    }
    orc_destroy(c);
    free(u0);
    printf("%s: ok\n", name);
}

int main(void)
{
    const char *names[] = {"nlm", "ucm", "grid", "full_tensor", "paper_coupling",
                           "strain_damping", "instantaneous"};
    for (int m = 0; m < 7; ++m)
        run_mode(m, names[m]);

    /* the grid on its own: pushes past several combinations, entry walk, sum */
    orc_qgrid *g = orc_qgrid_create(4, 6);
    const int cap = orc_qgrid_capacity(g);
    double *t0 = malloc(sizeof(double) * cap), *dt = malloc(sizeof(double) * cap),
           *k4 = malloc(sizeof(double) * 4 * cap), *strain = malloc(sizeof(double) * cap);
    for (long t = 0; t < 200; ++t)
        orc_qgrid_push(g, t, 1e-4, 2e-3 * cos(0.01 * t), -1e-4, 5e-5);
    const int n = orc_qgrid_entries(g, t0, dt, k4, strain);
    double sxy = 0.0, n1 = 0.0;
    orc_qgrid_sum(g, 199, 1e-3, 40.0, 0.1, &sxy, &n1);
    if (n <= 0 || n > cap || !isfinite(sxy) || !isfinite(n1)) {
        printf("grid walk: bad entry count %d or sum\n", n);
        failures++;
    }
    free(t0), free(dt), free(k4), free(strain);
    orc_qgrid_destroy(g);

    /* matrix exponential of a small and a large velocity gradient */
    const double A[4] = {1e-3, 2e-3, -5e-4, -1e-3}, B[4] = {3.0, -2.0, 1.5, -1.0};
    double E[4];
    orc_expm2(A, E);
    orc_expm2(B, E);
    printf("%s\n", failures ? "FAILED" : "all modes ok");
    return failures ? 1 : 0;
}
