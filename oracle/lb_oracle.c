/*
 * lb_oracle.c -- FP64 CPU oracle of the hybrid lattice-Boltzmann scheme with
 * the integral nonlinear Maxwell (nlM) constitutive equation of
 * Papenkort & Voigtmann, "Lattice Boltzmann simulations of a viscoelastic
 * shear-thinning fluid" (arXiv:1504.06123).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it; the product path never does.  It shares no source, header, table
 * or helper with the GPU path.
 *
 * Style: plain loops, doubles everywhere, one function per step of the
 * scheme, in the order the paper describes them.  Nothing is fused, blocked
 * or reordered.  The readings taken where the paper is silent or ambiguous
 * are stated next to the code they affect.
 *
 * Per time step t (state: populations n(t) after streaming, the stress of
 * the previous step sigma^{t-1}, the history ring, the strain prefix
 * Gamma_t):
 *   1. density and momentum  rho = sum n_i,  j = sum c_i n_i
 *   2. force density  f = rho*g + div sigma^{t-1}
 *   3. velocity  u = (j + f/2)/rho                        (Eq. hydrofields)
 *   4. velocity gradient kappa_ab = d_b u_a by 2nd-order differences, shear
 *      rate s = kappa_xy and r = sqrt(II_D)              (Sec. II, Sec. III)
 *   5. push (s_t, r_t, Gamma_t) into the ring, Gamma_{t+1} = Gamma_t + s_t
 *   6. history integral (Eq. gitt with Eq. nlmax) -> sigma^t
 *   7. BGK collision with the forcing term (Eq. bodyforce, f^ex part)
 *   8. streaming with halfway bounce-back walls at y = -1/2 and y = ly-1/2.
 *
 * Steps 5-6 use either the uniform window of the last n_hist steps or, when
 * orc_set_history_grid() was called, the quasi-logarithmic grid of Sec. III
 * (blocks whose step doubles going back; the two oldest entries of a full
 * block are combined into the next block).  The grid keeps kappa and the
 * deformation factors exactly as the paper describes and multiplies the
 * factors to obtain the strain.  With orc_set_finger() the stress is taken
 * from the full Finger tensor instead of its simple-shear reduction: the
 * window keeps kappa(t') and exp(kappa(t') dt), E(t, t') is their ordered
 * product (Eq. eeval) and -d_t' B = E kappa E^T + (E kappa E^T)^T; then
 * sigma_yy enters the force and N1 = sigma_xx - sigma_yy.  State exchange
 * (orc_get/set_state) covers the uniform window of the reduced path only.
 * With orc_set_paper_coupling() the stress reaches the fluid through the
 * paper's own forcing term (Eq. bodyforce in full): the traceless part in the
 * second moment of F_i, the trace through d_t delta rho = -(tr sigma^{t-1} -
 * tr sigma^{t-2}) / (2 cs2), rho = sum n + d_t rho / 2 and f = rho g only
 * (Eq. hydrofields) -- instead of the body force div sigma.  orc_set_law()
 * selects the accumulated-strain variant of the damping (Sec. II) or the
 * instantaneous law of Eq. inlM instead of the integral nlM model.
 *
 * Parity status: every function below is pinned by the CPU test suite
 * (closed forms, moment identities, polynomial exactness, recursion
 * equivalence, conservation, symmetry, the Newtonian Poiseuille solution).
 * The coupled nonlinear transient as a whole has no closed form; it is
 * pinned only through its components and invariants.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* D2Q9 lattice (Sec. III): c_0 = 0, c_1..4 = (+-1,0),(0,+-1), c_5..8 the     */
/* diagonals; weights 4/9, 1/9, 1/36; c_s^2 = 1/3 in lattice units.          */
/* The numbering of the directions is not given in the paper; this one is    */
/* the oracle's own.                                                          */
/* ------------------------------------------------------------------------ */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

void orc_lattice(int *cx, int *cy, double *w, int *opp)
{
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        w[i] = WT[i];
        opp[i] = OPP[i];
    }
}

/* Node index: x fastest. */
static int idx(int lx, int x, int y) { return y * lx + x; }
static int wrap(int x, int lx) { return ((x % lx) + lx) % lx; }

/* ------------------------------------------------------------------------ */
/* Step 7a: equilibrium (Sec. III, second-order D2Q9 form).  The printed      */
/* formula is garbled (a stray parenthesis, u_{i alpha}); the reading is the  */
/* standard                                                                   */
/*   n_i^eq = a_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)].        */
/* ------------------------------------------------------------------------ */
void orc_equilibrium(double rho, double ux, double uy, double *neq)
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        neq[i] = WT[i] * rho *
                 (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* ------------------------------------------------------------------------ */
/* Step 7b: forcing term, the f^ex part of Eq. (bodyforce) with             */
/* d_t(delta rho) = 0:                                                        */
/*   F_i = a_i (1 - 1/(2 tau_LB)) [ c_a f_a / cs2                             */
/*          + (c_a c_b - cs2 delta_ab)(u_b f_a + u_a f_b) / (2 cs2^2) ].      */
/* Written with the tensor contraction exactly as printed.                   */
/* ------------------------------------------------------------------------ */
void orc_force_term(double tau_lb, double ux, double uy, double fx, double fy,
                    double *F)
{
    double u[2] = {ux, uy};
    double f[2] = {fx, fy};
    double pre = 1.0 - 1.0 / (2.0 * tau_lb);
    for (int i = 0; i < 9; ++i) {
        double c[2] = {(double)CX[i], (double)CY[i]};
        double lin = (c[0] * f[0] + c[1] * f[1]) / CS2;
        double quad = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double q = c[a] * c[b] - (a == b ? CS2 : 0.0);
                quad += q * (u[b] * f[a] + u[a] * f[b]);
            }
        F[i] = WT[i] * pre * (lin + quad / (2.0 * CS2 * CS2));
    }
}

/* ------------------------------------------------------------------------ */
/* Step 7: BGK collision plus forcing (Sec. III):                             */
/*   n*_i = n_i - (n_i - n_i^eq(rho,u)) / tau_LB + F_i.                      */
/* ------------------------------------------------------------------------ */
/* The paper's own forcing term, Eq. bodyforce in full: the traceless       */
/* non-Newtonian stress sbar (xx, xy, yy) enters the second moment, the      */
/* density rate dr = d_t delta rho (with dt = 1) carries its trace:          */
/*   F_i = a_i { -sbar:(c c - cs2 I) / (2 cs2^2 tau)                          */
/*         + (1 - 1/(2 tau)) [ dr + c.f / cs2                                 */
/*           + (c c - cs2 I):(-dr u u + u f + f u) / (2 cs2^2) ] }.           */
void orc_force_term_paper(double tau_lb, double ux, double uy, double fx,
                          double fy, const double *sbar, double dr, double *F)
{
    double u[2] = {ux, uy};
    double f[2] = {fx, fy};
    double S[2][2] = {{sbar[0], sbar[1]}, {sbar[1], sbar[2]}};
    double pre = 1.0 - 1.0 / (2.0 * tau_lb);
    for (int i = 0; i < 9; ++i) {
        double c[2] = {(double)CX[i], (double)CY[i]};
        double stress = 0.0, quad = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double q = c[a] * c[b] - (a == b ? CS2 : 0.0);
                stress += S[a][b] * q;
                quad += q * (-dr * u[a] * u[b] + u[b] * f[a] + u[a] * f[b]);
            }
        double lin = (c[0] * f[0] + c[1] * f[1]) / CS2;
        F[i] = WT[i] * (-stress / (2.0 * CS2 * CS2 * tau_lb) +
                        pre * (dr + lin + quad / (2.0 * CS2 * CS2)));
    }
}

void orc_collide(double tau_lb, const double *n, double rho, double ux,
                 double uy, double fx, double fy, double *nstar)
{
    double neq[9], F[9];
    orc_equilibrium(rho, ux, uy, neq);
    orc_force_term(tau_lb, ux, uy, fx, fy, F);
    for (int i = 0; i < 9; ++i)
        nstar[i] = n[i] - (n[i] - neq[i]) / tau_lb + F[i];
}

/* Step 1: zeroth and first moments of the populations at one node. */
void orc_density_momentum(const double *n, double *rho, double *jx, double *jy)
{
    double r = 0.0, a = 0.0, b = 0.0;
    for (int i = 0; i < 9; ++i) {
        r += n[i];
        a += CX[i] * n[i];
        b += CY[i] * n[i];
    }
    *rho = r;
    *jx = a;
    *jy = b;
}

/* ------------------------------------------------------------------------ */
/* Step 4: velocity gradient kappa_ab = d_b u_a (kappa = (grad v)^T, Sec. I)  */
/* with second-order finite differences (Sec. III).  d/dx: periodic central.  */
/* d/dy: central in the interior; at the wall-adjacent rows the 3-point       */
/* second-order stencil through the no-slip wall value u = 0 at y = -1/2      */
/* (resp. y = ly - 1/2):                                                      */
/*   d_y u(0) = u(0) + u(1)/3,   d_y u(ly-1) = -u(ly-1) - u(ly-2)/3.         */
/* The paper says only "second-order finite difference"; the wall stencil is  */
/* the oracle's reading.  Arrays are [ly][lx].                               */
/* ------------------------------------------------------------------------ */
static double ddy(const double *u, int lx, int ly, int x, int y)
{
    if (y == 0)
        return u[idx(lx, x, 0)] + u[idx(lx, x, 1)] / 3.0;
    if (y == ly - 1)
        return -u[idx(lx, x, ly - 1)] - u[idx(lx, x, ly - 2)] / 3.0;
    return 0.5 * (u[idx(lx, x, y + 1)] - u[idx(lx, x, y - 1)]);
}

static double ddx(const double *u, int lx, int x, int y)
{
    return 0.5 * (u[idx(lx, wrap(x + 1, lx), y)] - u[idx(lx, wrap(x - 1, lx), y)]);
}

void orc_velocity_gradient(int lx, int ly, const double *ux, const double *uy,
                           double *kxx, double *kxy, double *kyx, double *kyy)
{
    for (int y = 0; y < ly; ++y)
        for (int x = 0; x < lx; ++x) {
            int k = idx(lx, x, y);
            kxx[k] = ddx(ux, lx, x, y);
            kxy[k] = ddy(ux, lx, ly, x, y);
            kyx[k] = ddx(uy, lx, x, y);
            kyy[k] = ddy(uy, lx, ly, x, y);
        }
}

/* ------------------------------------------------------------------------ */
/* Local shear rate (Sec. II): gamma_dot^2 = II_D = (1/2) tr D^2 with         */
/* D = kappa + kappa^T (no factor 1/2 in D, as printed).                     */
/* ------------------------------------------------------------------------ */
double orc_shear_rate(double kxx, double kxy, double kyx, double kyy)
{
    double D[2][2] = {{kxx + kxx, kxy + kyx}, {kyx + kxy, kyy + kyy}};
    double tr = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            tr += D[a][b] * D[b][a];
    return sqrt(0.5 * tr);
}

/* ------------------------------------------------------------------------ */
/* Step 2: divergence of the stress, f_a = d_b sigma_ab, entering the force   */
/* density of Eq. (ns).  d/dx periodic central; d/dy central in the interior  */
/* and the one-sided 3-point second-order stencil at the first and last rows  */
/*   d_y s(0) = (-3 s0 + 4 s1 - s2)/2,  d_y s(L-1) = (3 s_{L-1} - 4 s_{L-2}   */
/*   + s_{L-3})/2.                                                            */
/* syy may be NULL (zero).                                                    */
/* ------------------------------------------------------------------------ */
static double ddy_onesided(const double *s, int lx, int ly, int x, int y)
{
    if (y == 0)
        return 0.5 * (-3.0 * s[idx(lx, x, 0)] + 4.0 * s[idx(lx, x, 1)] -
                      s[idx(lx, x, 2)]);
    if (y == ly - 1)
        return 0.5 * (3.0 * s[idx(lx, x, ly - 1)] - 4.0 * s[idx(lx, x, ly - 2)] +
                      s[idx(lx, x, ly - 3)]);
    return 0.5 * (s[idx(lx, x, y + 1)] - s[idx(lx, x, y - 1)]);
}

void orc_stress_divergence(int lx, int ly, const double *sxx, const double *sxy,
                           const double *syy, double *fx, double *fy)
{
    for (int y = 0; y < ly; ++y)
        for (int x = 0; x < lx; ++x) {
            int k = idx(lx, x, y);
            fx[k] = ddx(sxx, lx, x, y) + ddy_onesided(sxy, lx, ly, x, y);
            fy[k] = ddx(sxy, lx, x, y) +
                    (syy ? ddy_onesided(syy, lx, ly, x, y) : 0.0);
        }
}

/* ------------------------------------------------------------------------ */
/* Step 8: streaming n_i(r + c_i, t+1) = n*_i(r, t) (Sec. III collision-and-  */
/* streaming rule), x periodic.  A population that would leave through a     */
/* wall (y < 0 or y >= ly) is reflected into the opposite direction at the   */
/* node it left (halfway bounce-back).  Arrays are [9][ly][lx].              */
/* ------------------------------------------------------------------------ */
void orc_stream(int lx, int ly, const double *nstar, double *nout)
{
    int N = lx * ly;
    for (int y = 0; y < ly; ++y)
        for (int x = 0; x < lx; ++x)
            for (int i = 0; i < 9; ++i) {
                double v = nstar[i * N + idx(lx, x, y)];
                int yy = y + CY[i];
                if (yy < 0 || yy >= ly)
                    nout[OPP[i] * N + idx(lx, x, y)] = v;
                else
                    nout[i * N + idx(lx, wrap(x + CX[i], lx), yy)] = v;
            }
}

/* ------------------------------------------------------------------------ */
/* Step 6: the history integral of Eq. (gitt) with the modulus of           */
/* Eq. (nlmax), reduced to simple shear.                                      */
/*                                                                            */
/* For unidirectional flow kappa = [[0,s],[0,0]] is nilpotent, so the         */
/* time-ordered product of Eq. (eeval) collapses to E = [[1,g],[0,1]] with    */
/* the accumulated strain g = Gamma_t - Gamma_t', and the Finger-tensor rate  */
/* of Sec. III, -d_t' B = E kappa(t') E^T + (E kappa(t') E^T)^T, becomes      */
/* s(t') [[2 g, 1], [1, 0]].  Hence                                           */
/*   sigma_xy = sum_k w_k s G_k,  sigma_xx = sum_k w_k 2 s g G_k,            */
/*   sigma_yy = 0,  with  G_k = G_inf exp(-k/tau) exp(-k r(t')/gamma_c).      */
/* The damping rate uses the shear rate at the past time t' (Eq. nlmax; the  */
/* stray "dt'" inside the printed modulus is read as a typo).  The          */
/* trapezoidal rule (Sec. III) is applied with fixed weights over the full    */
/* window of n_hist entries: w = 1/2 at the newest (k = 0) and oldest        */
/* (k = n_hist - 1) entry, 1 elsewhere; entries older than the start of the  */
/* run are zero (stress-free rest state before t = 0, Eq. maxwell).          */
/*                                                                            */
/* Inputs are by age k = t - t' for k < n_live (n_live <= n_hist): s, r and   */
/* the accumulated strain dgam_k = Gamma_t - Gamma_{t-k}.                    */
/* ------------------------------------------------------------------------ */
void orc_history_sum(int n_hist, int n_live, const double *s_age,
                     const double *r_age, const double *dgam_age, double g_inf,
                     double tau_m, double gamma_c, double *sxy, double *sxx)
{
    double a = 0.0, b = 0.0;
    for (int k = 0; k < n_live && k < n_hist; ++k) {
        double w = (k == 0 || k == n_hist - 1) ? 0.5 : 1.0;
        double G = g_inf * exp(-(double)k / tau_m) *
                   exp(-(double)k * r_age[k] / gamma_c);
        a += w * s_age[k] * G;
        b += w * 2.0 * s_age[k] * dgam_age[k] * G;
    }
    *sxy = a;
    *sxx = b;
}

/* The White-Metzner-type variant of Sec. II: the rate-dependent second      */
/* exponential of Eq. nlmax becomes the accumulated strain, here the total    */
/* shear accumulated from t' to t, R = sum of r(j) over the steps             */
/* j = t', ..., t - 1 (the same steps as the strain gamma):                    */
/*   G(t, t') = G exp(-(t - t')/tau) exp(-R(t, t')/gamma_c).                   */
/* Inputs by age as in orc_history_sum.                                        */
void orc_history_sum_wm(int n_hist, int n_live, const double *s_age,
                        const double *r_age, const double *dgam_age, double g_inf,
                        double tau_m, double gamma_c, double *sxy, double *sxx)
{
    double a = 0.0, b = 0.0, R = 0.0;
    for (int k = 0; k < n_live && k < n_hist; ++k) {
        if (k > 0)
            R += r_age[k];
        double w = (k == 0 || k == n_hist - 1) ? 0.5 : 1.0;
        double G = g_inf * exp(-(double)k / tau_m) * exp(-R / gamma_c);
        a += w * s_age[k] * G;
        b += w * 2.0 * s_age[k] * dgam_age[k] * G;
    }
    *sxy = a;
    *sxx = b;
}

/* Eq. inlM read at time t (the instantaneous nonlinear Maxwell model of Sec. */
/* IV): sigma_struc = sum_{n>=1} G tau_M^n d^(n), which for the simple-shear   */
/* reduction (kappa nilpotent: d^(1) = kappa + kappa^T, d^(2) = 2 kappa        */
/* kappa^T, d^(n>2) = 0) is sigma_xy = G tau_M s, sigma_xx = 2 G tau_M^2 s^2,   */
/* with tau_M = 1/(1/tau + r/gamma_c).                                         */
void orc_instantaneous(double s, double r, double g_inf, double tau_m,
                       double gamma_c, double *sxy, double *sxx)
{
    double taum = 1.0 / (1.0 / tau_m + r / gamma_c);
    *sxy = g_inf * taum * s;
    *sxx = 2.0 * g_inf * taum * taum * s * s;
}

/* Same sum from the shear history alone (all n_hist ages given, zeros for   */
/* times before the run).  The strain prefix is built the way the scheme      */
/* keeps it: Gamma grows from the oldest entry forward, Gamma_{t'+1} =        */
/* Gamma_{t'} + s(t') (exclusive prefix, Eq. eeval: the newest factor of E    */
/* is exp(kappa(t - dt) dt), the oldest exp(kappa(t') dt)).                  */
void orc_history_sum_ages(int n_hist, const double *s_age, const double *r_age,
                          double g_inf, double tau_m, double gamma_c,
                          double *sxy, double *sxx)
{
    double *gam = (double *)malloc(sizeof(double) * (size_t)n_hist);
    double *dg = (double *)malloc(sizeof(double) * (size_t)n_hist);
    /* gam[k] = Gamma at time t - k, taking Gamma = 0 at the oldest entry. */
    gam[n_hist - 1] = 0.0;
    for (int k = n_hist - 1; k > 0; --k)
        gam[k - 1] = gam[k] + s_age[k];
    for (int k = 0; k < n_hist; ++k)
        dg[k] = gam[0] - gam[k];
    orc_history_sum(n_hist, n_hist, s_age, r_age, dg, g_inf, tau_m, gamma_c,
                    sxy, sxx);
    free(gam);
    free(dg);
}

/* ------------------------------------------------------------------------ */
/* Quasi-logarithmic history grid (Sec. III).                                 */
/*                                                                            */
/* B blocks of equidistant entries; block b = 1..B has the step               */
/* dt_b = 2^(B-b) (block B, the newest, has the LB step 1).  Each entry keeps */
/* its start time t0, its duration dt, the velocity gradient kappa averaged   */
/* over [t0, t0 + dt) and its factor of the deformation tensor, which in the  */
/* simple-shear reduction is F = [[1, kappa_xy dt], [0, 1]].  A new entry     */
/* enters block B every step.  When a block then holds more than C entries,   */
/* its two oldest are combined -- factors multiplied, kappa averaged,         */
/* durations added -- into the newest entry of block b - 1; what block 1      */
/* combines falls off the grid.  Readings where the paper is silent: a block  */
/* holds at most C entries and combines when a push makes it C + 1; before    */
/* t = 0 every block is full of zero entries of its own step, contiguous in   */
/* time (the rest state); the time integral uses the trapezoid rule on the    */
/* entries' start times, and the damping uses sqrt(II_D) of the averaged      */
/* kappa.                                                                     */
/* ------------------------------------------------------------------------ */
static double *zalloc_q(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

typedef struct {
    double t0, dt;
    double k[4];   /* kxx, kxy, kyx, kyy averaged over the entry */
    double F[4];   /* deformation factor, row-major 2x2 */
} orc_qentry;

typedef struct orc_qgrid {
    int B, C;
    int *count;          /* [B] entries in each block */
    orc_qentry *e;       /* [B][C + 1], oldest first within a block */
} orc_qgrid;

static void qgrid_init(orc_qgrid *g, int B, int C)
{
    g->B = B;
    g->C = C;
    g->count = (int *)calloc((size_t)B, sizeof(int));
    g->e = (orc_qentry *)calloc((size_t)B * (size_t)(C + 1), sizeof(orc_qentry));
    /* zero prefill, newest block first, walking back in time from t' = 0 */
    double t_end = 0.0;
    for (int b = B; b >= 1; --b) {
        double dt = ldexp(1.0, B - b);
        orc_qentry *blk = g->e + (size_t)(b - 1) * (C + 1);
        for (int i = C - 1; i >= 0; --i) {
            orc_qentry *q = &blk[i];
            t_end -= dt;
            q->t0 = t_end;
            q->dt = dt;
            q->F[0] = 1.0;
            q->F[3] = 1.0;
        }
        g->count[b - 1] = C;
    }
}

static void qgrid_free(orc_qgrid *g)
{
    free(g->count);
    free(g->e);
}

/* Push the entry of step t with velocity gradient k[4], then let every full  */
/* block pass its two oldest entries on, newest block first.                  */
static void qgrid_push(orc_qgrid *g, long t, const double *k)
{
    const int B = g->B, C = g->C;
    orc_qentry in;
    memset(&in, 0, sizeof in);
    in.t0 = (double)t;
    in.dt = 1.0;
    for (int a = 0; a < 4; ++a)
        in.k[a] = k[a];
    in.F[0] = 1.0;
    in.F[1] = k[1] * 1.0;  /* exp(kappa dt) of simple shear */
    in.F[3] = 1.0;
    for (int b = B; b >= 1; --b) {
        orc_qentry *blk = g->e + (size_t)(b - 1) * (C + 1);
        blk[g->count[b - 1]] = in;
        g->count[b - 1] += 1;
        if (g->count[b - 1] <= C)
            return;
        /* the two oldest: blk[0] (older) and blk[1] */
        orc_qentry m;
        memset(&m, 0, sizeof m);
        m.t0 = blk[0].t0;
        m.dt = blk[0].dt + blk[1].dt;
        for (int a = 0; a < 4; ++a)
            m.k[a] = 0.5 * (blk[0].k[a] + blk[1].k[a]);
        /* E accumulates newer factors on the left: F(newer) F(older) */
        m.F[0] = blk[1].F[0] * blk[0].F[0] + blk[1].F[1] * blk[0].F[2];
        m.F[1] = blk[1].F[0] * blk[0].F[1] + blk[1].F[1] * blk[0].F[3];
        m.F[2] = blk[1].F[2] * blk[0].F[0] + blk[1].F[3] * blk[0].F[2];
        m.F[3] = blk[1].F[2] * blk[0].F[1] + blk[1].F[3] * blk[0].F[3];
        memmove(blk, blk + 2, sizeof(orc_qentry) * (size_t)(g->count[b - 1] - 2));
        g->count[b - 1] -= 2;
        in = m;  /* moves to block b - 1 (dropped after block 1) */
    }
}

/* Number of live entries, newest first: fills t0[], dt[], kxy[] and the      */
/* strain gamma(t, t0) = E_xy of the ordered product of the factors from the  */
/* newest-but-one entry down to the entry itself (Eq. eeval).                  */
static int qgrid_walk(const orc_qgrid *g, double *t0, double *dt, double *k4,
                      double *strain)
{
    int n = 0;
    double E[4] = {1.0, 0.0, 0.0, 1.0};
    for (int b = g->B; b >= 1; --b) {
        const orc_qentry *blk = g->e + (size_t)(b - 1) * (g->C + 1);
        for (int i = g->count[b - 1] - 1; i >= 0; --i) {
            const orc_qentry *q = &blk[i];
            if (n > 0) {
                /* E(t, t0) = E(t, t0 + dt) F(entry) */
                double e0 = E[0] * q->F[0] + E[1] * q->F[2];
                double e1 = E[0] * q->F[1] + E[1] * q->F[3];
                double e2 = E[2] * q->F[0] + E[3] * q->F[2];
                double e3 = E[2] * q->F[1] + E[3] * q->F[3];
                E[0] = e0; E[1] = e1; E[2] = e2; E[3] = e3;
            }
            t0[n] = q->t0;
            dt[n] = q->dt;
            for (int a = 0; a < 4; ++a)
                k4[4 * n + a] = q->k[a];
            strain[n] = E[1];
            ++n;
        }
    }
    return n;
}

/* Eq. gitt with Eq. nlmax on the grid's entries: trapezoid weights from the  */
/* start times, w_e = (t0_{e-1} - t0_{e+1})/2 with the end intervals halved.   */
static void qgrid_sum(int n, long t, const double *t0, const double *k4,
                      const double *strain, double g_inf, double tau_m,
                      double gamma_c, double *sxy, double *sxx)
{
    double a = 0.0, b = 0.0;
    for (int e = 0; e < n; ++e) {
        double newer = e > 0 ? t0[e - 1] : t0[e];
        double older = e + 1 < n ? t0[e + 1] : t0[e];
        double w = 0.5 * (newer - older);
        double age = (double)t - t0[e];
        double s = k4[4 * e + 1];
        double r = orc_shear_rate(k4[4 * e], k4[4 * e + 1], k4[4 * e + 2], k4[4 * e + 3]);
        double G = g_inf * exp(-age / tau_m) * exp(-age * r / gamma_c);
        a += w * s * G;
        b += w * 2.0 * s * strain[e] * G;
    }
    *sxy = a;
    *sxx = b;
}

/* Standalone grid for the pins: create, push a step, read the entries, sum. */
orc_qgrid *orc_qgrid_create(int B, int C)
{
    if (B < 1 || C < 2)
        return NULL;
    orc_qgrid *g = (orc_qgrid *)calloc(1, sizeof(orc_qgrid));
    qgrid_init(g, B, C);
    return g;
}

void orc_qgrid_destroy(orc_qgrid *g)
{
    if (!g)
        return;
    qgrid_free(g);
    free(g);
}

void orc_qgrid_push(orc_qgrid *g, long t, double kxx, double kxy, double kyx, double kyy)
{
    double k[4] = {kxx, kxy, kyx, kyy};
    qgrid_push(g, t, k);
}

int orc_qgrid_capacity(const orc_qgrid *g) { return g->B * (g->C + 1); }

int orc_qgrid_entries(const orc_qgrid *g, double *t0, double *dt, double *k4,
                      double *strain)
{
    return qgrid_walk(g, t0, dt, k4, strain);
}

void orc_qgrid_sum(const orc_qgrid *g, long t, double g_inf, double tau_m,
                   double gamma_c, double *sxy, double *sxx)
{
    int cap = orc_qgrid_capacity(g);
    double *t0 = zalloc_q(cap), *dt = zalloc_q(cap), *k4 = zalloc_q(4 * (size_t)cap),
           *st = zalloc_q(cap);
    int n = qgrid_walk(g, t0, dt, k4, st);
    qgrid_sum(n, t, t0, k4, st, g_inf, tau_m, gamma_c, sxy, sxx);
    free(t0);
    free(dt);
    free(k4);
    free(st);
}

/* ------------------------------------------------------------------------ */
/* Full-tensor Finger path (Sec. I Eq. gitt, Sec. III Eq. eeval and the       */
/* relation for -d_t' B).                                                     */
/*                                                                            */
/* exp of a 2x2 matrix: scaling and squaring of the Taylor series (the norm  */
/* is halved until it is at most 1/4, 24 Taylor terms, then squared back).   */
/* ------------------------------------------------------------------------ */
static void mat2_mul(const double *a, const double *b, double *out)
{
    double r0 = a[0] * b[0] + a[1] * b[2];
    double r1 = a[0] * b[1] + a[1] * b[3];
    double r2 = a[2] * b[0] + a[3] * b[2];
    double r3 = a[2] * b[1] + a[3] * b[3];
    out[0] = r0;
    out[1] = r1;
    out[2] = r2;
    out[3] = r3;
}

void orc_expm2(const double *A, double *out)
{
    double nrm = fabs(A[0]) + fabs(A[1]) + fabs(A[2]) + fabs(A[3]);
    int sq = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++sq;
    }
    double sc = ldexp(1.0, -sq);
    double B[4] = {A[0] * sc, A[1] * sc, A[2] * sc, A[3] * sc};
    double T[4] = {1.0, 0.0, 0.0, 1.0}, term[4] = {1.0, 0.0, 0.0, 1.0};
    for (int n = 1; n <= 24; ++n) {
        mat2_mul(term, B, term);
        for (int i = 0; i < 4; ++i) {
            term[i] /= (double)n;
            T[i] += term[i];
        }
    }
    for (int i = 0; i < sq; ++i)
        mat2_mul(T, T, T);
    for (int i = 0; i < 4; ++i)
        out[i] = T[i];
}

/* Eq. gitt over a window given by age k = 0..n_live-1 (n_live <= n_hist):  */
/* kappa_k[4] and the factors F_k = exp(kappa_k dt).  The deformation tensor */
/* E(t, t - k) = F_1 F_2 ... F_k (Eq. eeval: newest factor on the left; the */
/* entry at age 0 contributes no factor), -d_t' B = E kappa E^T + (E kappa  */
/* E^T)^T, weights and modulus as in the simple-shear sum.  Output: sigma   */
/* xx, xy, yy.                                                                */
void orc_finger_sum(int n_hist, int n_live, const double *k_age, const double *f_age,
                    double g_inf, double tau_m, double gamma_c, double *sig3)
{
    double E[4] = {1.0, 0.0, 0.0, 1.0};
    double sxx = 0.0, sxy = 0.0, syy = 0.0;
    for (int k = 0; k < n_live && k < n_hist; ++k) {
        const double *kap = k_age + 4 * (size_t)k;
        if (k > 0)
            mat2_mul(E, f_age + 4 * (size_t)k, E);
        double Et[4] = {E[0], E[2], E[1], E[3]};
        double M[4];
        mat2_mul(E, kap, M);
        mat2_mul(M, Et, M);
        double w = (k == 0 || k == n_hist - 1) ? 0.5 : 1.0;
        double r = orc_shear_rate(kap[0], kap[1], kap[2], kap[3]);
        double G = g_inf * exp(-(double)k / tau_m) * exp(-(double)k * r / gamma_c);
        sxx += w * 2.0 * M[0] * G;
        sxy += w * (M[1] + M[2]) * G;
        syy += w * 2.0 * M[3] * G;
    }
    sig3[0] = sxx;
    sig3[1] = sxy;
    sig3[2] = syy;
}

/* ------------------------------------------------------------------------ */
/* One channel: state and time loop.                                          */
/* ------------------------------------------------------------------------ */
typedef struct orc_channel {
    int lx, ly, N, n_hist;
    double tau_lb, g_inf, tau_m, gamma_c, gx, gy;
    long t;          /* completed steps */
    int has_out;     /* outputs below belong to step t-1 */
    double *n;       /* [9][N] populations n(t), after streaming */
    double *sig_xy;  /* [N] sigma_xy of the last completed step (sigma^{t-1}) */
    double *sig_xx;  /* [N] sigma_xx of the last completed step */
    double *ring_s;  /* [n_hist][N] shear rate s(t'), slot t' mod n_hist */
    double *ring_r;  /* [n_hist][N] r(t') = sqrt(II_D(t')) */
    double *ring_g;  /* [n_hist][N] Gamma_{t'} */
    double *gam;     /* [N] Gamma_t */
    struct orc_qgrid *qg; /* [N] quasi-logarithmic history grids, or NULL */
    /* full-tensor Finger path (NULL unless enabled): per entry the velocity   */
    /* gradient and its factor exp(kappa dt) of the deformation tensor         */
    double *ring_k;  /* [n_hist][4][N] kxx, kxy, kyx, kyy of t' */
    double *ring_f;  /* [n_hist][4][N] exp(kappa(t') dt), row-major 2x2 */
    double *sig_yy;  /* [N] sigma_yy of the last completed step (full tensor) */
    int paper_coupling; /* 1: stress through Eq. bodyforce instead of div sigma */
    int law;         /* 0: Eq. nlmax; 1: accumulated-strain damping; 2: Eq. inlM */
    double *tr_prev; /* [N] trace of sigma two steps back (paper coupling) */
    double *new_yy;
    /* outputs of the last completed step */
    double *rho_o, *ux_o, *uy_o, *kap_o; /* kap_o: [4][N] kxx,kxy,kyx,kyy */
    /* scratch */
    double *nstar, *fx, *fy, *jx, *jy, *sxx_div, *new_xy, *new_xx;
    double *s_age, *r_age, *dg_age;
} orc_channel;

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

orc_channel *orc_create(int lx, int ly, double tau_lb, double g_inf,
                        double tau_m, double gamma_c, int n_hist, double gx,
                        double gy, const double *u0)
{
    if (lx < 1 || ly < 3 || n_hist < 2 || !(tau_lb > 0.5))
        return NULL;
    orc_channel *c = (orc_channel *)calloc(1, sizeof(orc_channel));
    size_t N = (size_t)lx * (size_t)ly;
    c->lx = lx;
    c->ly = ly;
    c->N = (int)N;
    c->n_hist = n_hist;
    c->tau_lb = tau_lb;
    c->g_inf = g_inf;
    c->tau_m = tau_m;
    c->gamma_c = gamma_c;
    c->gx = gx;
    c->gy = gy;
    c->t = 0;
    c->n = zalloc(9 * N);
    c->sig_xy = zalloc(N);
    c->sig_xx = zalloc(N);
    c->ring_s = zalloc((size_t)n_hist * N);
    c->ring_r = zalloc((size_t)n_hist * N);
    c->ring_g = zalloc((size_t)n_hist * N);
    c->gam = zalloc(N);
    c->rho_o = zalloc(N);
    c->ux_o = zalloc(N);
    c->uy_o = zalloc(N);
    c->kap_o = zalloc(4 * N);
    c->nstar = zalloc(9 * N);
    c->fx = zalloc(N);
    c->fy = zalloc(N);
    c->jx = zalloc(N);
    c->jy = zalloc(N);
    c->sxx_div = zalloc(N);
    c->new_xy = zalloc(N);
    c->new_xx = zalloc(N);
    c->s_age = zalloc((size_t)n_hist);
    c->r_age = zalloc((size_t)n_hist);
    c->dg_age = zalloc((size_t)n_hist);
    /* Initial state: n_i = n_i^eq(rho = 1, u0), i.e. a_i at rest. */
    for (size_t k = 0; k < N; ++k) {
        double neq[9];
        double ux = u0 ? u0[k] : 0.0;
        double uy = u0 ? u0[N + k] : 0.0;
        orc_equilibrium(1.0, ux, uy, neq);
        for (int i = 0; i < 9; ++i)
            c->n[i * N + k] = neq[i];
    }
    return c;
}

void orc_destroy(orc_channel *c)
{
    if (!c)
        return;
    double *bufs[] = {c->n,      c->sig_xy, c->sig_xx, c->ring_s, c->ring_r,
                      c->ring_g, c->gam,    c->rho_o,  c->ux_o,   c->uy_o,
                      c->kap_o,  c->nstar,  c->fx,     c->fy,     c->jx,
                      c->jy,     c->sxx_div, c->new_xy, c->new_xx, c->s_age,
                      c->r_age,  c->dg_age};
    for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i)
        free(bufs[i]);
    if (c->qg) {
        for (int k = 0; k < c->N; ++k)
            qgrid_free(&c->qg[k]);
        free(c->qg);
    }
    free(c->ring_k);
    free(c->ring_f);
    free(c->tr_prev);
    free(c->sig_yy);
    free(c->new_yy);
    free(c);
}

void orc_set_force(orc_channel *c, double gx, double gy)
{
    c->gx = gx;
    c->gy = gy;
}

/* Switch the channel to the quasi-logarithmic history grid of B blocks of   */
/* C entries (before its first step); the uniform window is then unused.      */
int orc_set_history_grid(orc_channel *c, int B, int C)
{
    if (c->t != 0 || c->qg || c->ring_k || c->law || B < 1 || C < 2)
        return -1;
    c->qg = (orc_qgrid *)calloc((size_t)c->N, sizeof(orc_qgrid));
    for (int k = 0; k < c->N; ++k)
        qgrid_init(&c->qg[k], B, C);
    return 0;
}

/* Switch the channel to the full Finger tensor on its uniform window (before */
/* its first step): sigma_yy no longer vanishes and enters the force.         */
int orc_set_finger(orc_channel *c)
{
    if (c->t != 0 || c->qg || c->ring_k || c->law)
        return -1;
    size_t N = (size_t)c->N, H = (size_t)c->n_hist;
    c->ring_k = zalloc(4 * H * N);
    c->ring_f = zalloc(4 * H * N);
    for (size_t sl = 0; sl < H; ++sl)
        for (size_t k = 0; k < N; ++k) {
            c->ring_f[(sl * 4 + 0) * N + k] = 1.0;  /* zero gradient: identity */
            c->ring_f[(sl * 4 + 3) * N + k] = 1.0;
        }
    c->sig_yy = zalloc(N);
    c->new_yy = zalloc(N);
    return 0;
}

/* Enter the stress through the paper's forcing term (Eq. bodyforce:       */
/* traceless part in the second moment, trace through d_t delta rho)        */
/* instead of the body force div sigma (before the first step).              */
int orc_set_paper_coupling(orc_channel *c)
{
    if (c->t != 0 || c->paper_coupling)
        return -1;
    c->paper_coupling = 1;
    c->tr_prev = zalloc((size_t)c->N);
    return 0;
}

/* Trace of sigma two steps back (the paper coupling's state); n = N.       */
int orc_trace_prev(const orc_channel *c, double *out)
{
    if (!c->paper_coupling)
        return -1;
    memcpy(out, c->tr_prev, sizeof(double) * (size_t)c->N);
    return 0;
}

/* Constitutive law (before the first step): 0 the integral nlM model of    */
/* Eqs. gitt and nlmax, 1 its accumulated-strain (White-Metzner-type)        */
/* variant on the uniform window, 2 the instantaneous law of Eq. inlM.        */
int orc_set_law(orc_channel *c, int law)
{
    if (c->t != 0 || law < 0 || law > 2)
        return -1;
    if (law != 0 && (c->qg || c->ring_k))
        return -1;
    c->law = law;
    return 0;
}

long orc_time(const orc_channel *c) { return c->t; }

static void one_step(orc_channel *c)
{
    const int lx = c->lx, ly = c->ly, N = c->N, H = c->n_hist;
    const long t = c->t;
    double *kxx = c->kap_o, *kxy = c->kap_o + N, *kyx = c->kap_o + 2 * N,
           *kyy = c->kap_o + 3 * N;

    /* 1. density and momentum */
    for (int k = 0; k < N; ++k) {
        double nk[9];
        for (int i = 0; i < 9; ++i)
            nk[i] = c->n[i * N + k];
        orc_density_momentum(nk, &c->rho_o[k], &c->jx[k], &c->jy[k]);
    }
    if (c->paper_coupling) {
        /* The paper's coupling (Sec. III, Eqs. bodyforce and hydrofields):    */
        /* no stress divergence; d_t delta rho = -(tr sigma^{t-1} - tr         */
        /* sigma^{t-2}) / (2 cs2) carries the trace, rho = sum n + d_t rho / 2, */
        /* f = rho g (the external force only).                                */
        for (int k = 0; k < N; ++k) {
            double tr1 = c->sig_xx[k] + (c->sig_yy ? c->sig_yy[k] : 0.0);
            double dr = -(tr1 - c->tr_prev[k]) / (2.0 * CS2);
            c->tr_prev[k] = tr1;
            c->rho_o[k] += 0.5 * dr;
            c->fx[k] = c->rho_o[k] * c->gx;
            c->fy[k] = c->rho_o[k] * c->gy;
            c->ux_o[k] = (c->jx[k] + 0.5 * c->fx[k]) / c->rho_o[k];
            c->uy_o[k] = (c->jy[k] + 0.5 * c->fy[k]) / c->rho_o[k];
            c->sxx_div[k] = dr; /* kept for the collision below */
        }
        goto gradient;
    }
    /* 2. force density: rho g + div sigma^{t-1} (sigma_yy = 0) */
    orc_stress_divergence(lx, ly, c->sig_xx, c->sig_xy, c->sig_yy, c->fx, c->fy);
    for (int k = 0; k < N; ++k) {
        c->fx[k] += c->rho_o[k] * c->gx;
        c->fy[k] += c->rho_o[k] * c->gy;
    }
    /* 3. velocity with the half-force shift */
    for (int k = 0; k < N; ++k) {
        c->ux_o[k] = (c->jx[k] + 0.5 * c->fx[k]) / c->rho_o[k];
        c->uy_o[k] = (c->jy[k] + 0.5 * c->fy[k]) / c->rho_o[k];
    }
gradient:
    /* 4. velocity gradient and shear rates */
    orc_velocity_gradient(lx, ly, c->ux_o, c->uy_o, kxx, kxy, kyx, kyy);
    if (c->law == 2) {
        /* 5-6 replaced by the instantaneous law of the current gradient */
        for (int k = 0; k < N; ++k)
            orc_instantaneous(kxy[k], orc_shear_rate(kxx[k], kxy[k], kyx[k], kyy[k]),
                              c->g_inf, c->tau_m, c->gamma_c, &c->new_xy[k], &c->new_xx[k]);
        goto collide;
    }
    if (c->qg) {
        /* 5-6 on the quasi-logarithmic grid: push, combine, integrate */
        int cap = orc_qgrid_capacity(&c->qg[0]);
        double *t0 = zalloc(cap), *dt = zalloc(cap), *k4 = zalloc(4 * (size_t)cap),
               *st = zalloc(cap);
        for (int k = 0; k < N; ++k) {
            double kk[4] = {kxx[k], kxy[k], kyx[k], kyy[k]};
            qgrid_push(&c->qg[k], t, kk);
            int n = qgrid_walk(&c->qg[k], t0, dt, k4, st);
            qgrid_sum(n, t, t0, k4, st, c->g_inf, c->tau_m, c->gamma_c, &c->new_xy[k],
                      &c->new_xx[k]);
        }
        free(t0);
        free(dt);
        free(k4);
        free(st);
        goto collide;
    }
    if (c->ring_k) {
        /* 5-6 with the full Finger tensor: push kappa and exp(kappa dt),    */
        /* integrate over the window                                          */
        long sl = t % H;
        for (int k = 0; k < N; ++k) {
            double kk[4] = {kxx[k], kxy[k], kyx[k], kyy[k]}, f[4];
            orc_expm2(kk, f);
            for (int a = 0; a < 4; ++a) {
                c->ring_k[(sl * 4 + a) * N + k] = kk[a];
                c->ring_f[(sl * 4 + a) * N + k] = f[a];
            }
        }
        int live = (t + 1 < H) ? (int)(t + 1) : H;
        double *ka = zalloc(4 * (size_t)H), *fa = zalloc(4 * (size_t)H);
        for (int k = 0; k < N; ++k) {
            for (int a = 0; a < live; ++a) {
                long sa = (t - a) % H;
                for (int q = 0; q < 4; ++q) {
                    ka[4 * a + q] = c->ring_k[(sa * 4 + q) * N + k];
                    fa[4 * a + q] = c->ring_f[(sa * 4 + q) * N + k];
                }
            }
            double s3[3];
            orc_finger_sum(H, live, ka, fa, c->g_inf, c->tau_m, c->gamma_c, s3);
            c->new_xx[k] = s3[0];
            c->new_xy[k] = s3[1];
            c->new_yy[k] = s3[2];
        }
        free(ka);
        free(fa);
        goto collide;
    }
    /* 5. push entry t = (s_t, r_t, Gamma_t) */
    long slot = t % H;
    for (int k = 0; k < N; ++k) {
        c->ring_s[slot * N + k] = kxy[k];
        c->ring_r[slot * N + k] = orc_shear_rate(kxx[k], kxy[k], kyx[k], kyy[k]);
        c->ring_g[slot * N + k] = c->gam[k];
    }
    /* 6. history integral at every node */
    int n_live = (t + 1 < H) ? (int)(t + 1) : H;
    for (int k = 0; k < N; ++k) {
        for (int a = 0; a < n_live; ++a) {
            long sl = (t - a) % H;
            c->s_age[a] = c->ring_s[sl * N + k];
            c->r_age[a] = c->ring_r[sl * N + k];
            c->dg_age[a] = c->gam[k] - c->ring_g[sl * N + k];
        }
        if (c->law == 1)
            orc_history_sum_wm(H, n_live, c->s_age, c->r_age, c->dg_age, c->g_inf,
                               c->tau_m, c->gamma_c, &c->new_xy[k], &c->new_xx[k]);
        else
            orc_history_sum(H, n_live, c->s_age, c->r_age, c->dg_age, c->g_inf,
                            c->tau_m, c->gamma_c, &c->new_xy[k], &c->new_xx[k]);
    }
    for (int k = 0; k < N; ++k)
        c->gam[k] += kxy[k];
collide:
    /* 7. collision */
    for (int k = 0; k < N; ++k) {
        double nk[9], ns[9];
        for (int i = 0; i < 9; ++i)
            nk[i] = c->n[i * N + k];
        if (c->paper_coupling) {
            /* traceless part of sigma^{t-1}: sbar = sigma - (tr sigma / 2) I */
            double syy = c->sig_yy ? c->sig_yy[k] : 0.0;
            double sbar[3] = {0.5 * (c->sig_xx[k] - syy), c->sig_xy[k],
                              0.5 * (syy - c->sig_xx[k])};
            double neq[9], F[9];
            orc_equilibrium(c->rho_o[k], c->ux_o[k], c->uy_o[k], neq);
            orc_force_term_paper(c->tau_lb, c->ux_o[k], c->uy_o[k], c->fx[k],
                                 c->fy[k], sbar, c->sxx_div[k], F);
            for (int i = 0; i < 9; ++i)
                ns[i] = nk[i] - (nk[i] - neq[i]) / c->tau_lb + F[i];
        } else {
            orc_collide(c->tau_lb, nk, c->rho_o[k], c->ux_o[k], c->uy_o[k],
                        c->fx[k], c->fy[k], ns);
        }
        for (int i = 0; i < 9; ++i)
            c->nstar[i * N + k] = ns[i];
    }
    /* 8. streaming */
    orc_stream(lx, ly, c->nstar, c->n);
    memcpy(c->sig_xy, c->new_xy, sizeof(double) * (size_t)N);
    memcpy(c->sig_xx, c->new_xx, sizeof(double) * (size_t)N);
    if (c->sig_yy)
        memcpy(c->sig_yy, c->new_yy, sizeof(double) * (size_t)N);
    c->t = t + 1;
    c->has_out = 1;
}

void orc_step(orc_channel *c, long n_steps)
{
    for (long i = 0; i < n_steps; ++i)
        one_step(c);
}

/* Readouts refer to the last completed step; -1 before the first step and
 * after a state load (the loaded state carries no step outputs). */
int orc_fields(const orc_channel *c, double *rho, double *ux, double *uy)
{
    if (!c->has_out)
        return -1;
    size_t b = sizeof(double) * (size_t)c->N;
    if (rho) memcpy(rho, c->rho_o, b);
    if (ux) memcpy(ux, c->ux_o, b);
    if (uy) memcpy(uy, c->uy_o, b);
    return 0;
}

/* sigma_xy and the first normal-stress difference N1 = sigma_xx - sigma_yy. */
int orc_stress(const orc_channel *c, double *sxy, double *n1)
{
    if (!c->has_out)
        return -1;
    size_t b = sizeof(double) * (size_t)c->N;
    if (sxy) memcpy(sxy, c->sig_xy, b);
    if (n1) {
        memcpy(n1, c->sig_xx, b); /* sigma_yy = 0 in simple shear */
        if (c->sig_yy)
            for (int k = 0; k < c->N; ++k)
                n1[k] -= c->sig_yy[k];
    }
    return 0;
}

int orc_grad(const orc_channel *c, double *kappa)
{
    if (!c->has_out)
        return -1;
    memcpy(kappa, c->kap_o, sizeof(double) * 4 * (size_t)c->N);
    return 0;
}

/* Total mass sum_i n_i over the lattice for the current populations. */
double orc_mass(const orc_channel *c)
{
    double m = 0.0;
    for (long k = 0; k < 9L * c->N; ++k)
        m += c->n[k];
    return m;
}

/* State exchange.  Populations are n(t) after streaming, [9][ly][lx];      */
/* sig_* is sigma^{t-1}; the ring is slot-major [n_hist][N] with slot        */
/* t' mod n_hist; gam is Gamma_t.  Any pointer may be NULL (left unchanged). */
void orc_get_state(const orc_channel *c, double *n, double *sig_xy,
                   double *sig_xx, double *ring_s, double *ring_r,
                   double *ring_g, double *gam, long *t)
{
    size_t N = (size_t)c->N, R = (size_t)c->n_hist * N;
    if (n) memcpy(n, c->n, sizeof(double) * 9 * N);
    if (sig_xy) memcpy(sig_xy, c->sig_xy, sizeof(double) * N);
    if (sig_xx) memcpy(sig_xx, c->sig_xx, sizeof(double) * N);
    if (ring_s) memcpy(ring_s, c->ring_s, sizeof(double) * R);
    if (ring_r) memcpy(ring_r, c->ring_r, sizeof(double) * R);
    if (ring_g) memcpy(ring_g, c->ring_g, sizeof(double) * R);
    if (gam) memcpy(gam, c->gam, sizeof(double) * N);
    if (t) *t = c->t;
}

void orc_set_state(orc_channel *c, const double *n, const double *sig_xy,
                   const double *sig_xx, const double *ring_s,
                   const double *ring_r, const double *ring_g,
                   const double *gam, long t)
{
    size_t N = (size_t)c->N, R = (size_t)c->n_hist * N;
    if (n) memcpy(c->n, n, sizeof(double) * 9 * N);
    if (sig_xy) memcpy(c->sig_xy, sig_xy, sizeof(double) * N);
    if (sig_xx) memcpy(c->sig_xx, sig_xx, sizeof(double) * N);
    if (ring_s) memcpy(c->ring_s, ring_s, sizeof(double) * R);
    if (ring_r) memcpy(c->ring_r, ring_r, sizeof(double) * R);
    if (ring_g) memcpy(c->ring_g, ring_g, sizeof(double) * R);
    if (gam) memcpy(c->gam, gam, sizeof(double) * N);
    c->t = t;
    c->has_out = 0;
}
