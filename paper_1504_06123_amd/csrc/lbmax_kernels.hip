// lbmax_kernels.hip -- gfx950 kernels of the hybrid lattice-Boltzmann step
// with the integral nonlinear Maxwell stress (arXiv:1504.06123).
//
// One time step t is two grid-wide phases plus an optional combine:
//   k_lb      pull-stream + bounce-back, moments, force rho*g + div sigma^{t-1},
//             half-force velocity, BGK collision with the forcing term
//             (Sec. III: collision-streaming rule, Eqs. bodyforce, hydrofields)
//   history   velocity gradient, push of the shear history entry, and the
//             history integral of Eq. (gitt) with the modulus of Eq. (nlmax)
//             over the window of the last n_hist steps -> sigma^t:
//   k_hist_pass / k_hist_step: the history integral blocked in time (one
//             ring pass serves a block of steps, see below)
//   k_combine FP64 affine combination of per-chunk partial sums when a
//             channel's window is split across workgroups.
//
// Data layout (per channel, all planes [np] with node = y*lx + x):
//   populations: two buffers (step parity) x 9 planes of n_i - a_i in FP64;
//   in FP32 storage, 9 planes of FP32 remainders against the equilibrium of
//   the node's FP64 density and velocity, which two more buffers of 3 FP64
//   planes hold
//   history ring: row-major [n_hist][np]; row t' mod n_hist holds the entry
//   of step t'.  A wavefront reads one row per age: 64 consecutive nodes,
//   fully coalesced, streaming through HBM once per pass (a pass serves a
//   block of steps).  Ages are walked newest to oldest, so the accumulated
//   strain gamma_{t,t'} is a running FP64 sum of the shear rate over the
//   window (Sec. III Eq. eeval with the simple-shear reduction of the Finger
//   tensor) and no strain prefix has to be stored.
#include "lbmax_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace lbmax {

// ---------------------------------------------------------------------------
// D2Q9 (Sec. III).  Direction order of this library (opposites adjacent):
// 0 rest, 1 (+x), 2 (-x), 3 (+y), 4 (-y), 5 (+x+y), 6 (-x-y), 7 (+x-y), 8 (-x+y)
// ---------------------------------------------------------------------------
constexpr int QX[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int QY[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
constexpr int QOPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};

template <typename R>
__device__ __forceinline__ R qweight(int q)
{
    return q == 0 ? R(4) / R(9) : (q < 5 ? R(1) / R(9) : R(1) / R(36));
}

// n^eq_q - a_q = a_q [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)] (Sec. III,
// cs2 = 1/3), for direction weight w and cu = c_q.u.
template <typename P>
__device__ __forceinline__ P eq_dev(P w, P cu, P drho, P uu)
{
#pragma clang fp contract(off)
    return w * (drho + (P(1) + drho) * (P(3) * cu + P(4.5) * cu * cu - P(1.5) * uu));
}

// ---------------------------------------------------------------------------
// Window-sum accumulators.  FP32 history entries are summed in plain FP32
// partial groups (a few rows to 128 rows); each finished partial sum enters a
// Kahan-compensated FP32 total: the sum s and the compensation c, the
// negated low-order part that the additions so far have rounded away, which
// the next addition feeds back.  value() returns s - c in FP64.  FP64 entries
// are summed plainly.
// ---------------------------------------------------------------------------
template <typename R>
struct Acc {
    R s = R(0);
    __device__ __forceinline__ void add(R x) { s += x; }
    __device__ __forceinline__ double value() const { return s; }
};

template <>
struct Acc<float> {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x)
    {
        // the order of these operations is the compensation; nothing here
        // may be reassociated or contracted
#pragma clang fp contract(off) reassociate(off)
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// Rate constants of the memory decay exp(-k (1/tau + r/gamma_c)) of
// Eq. (nlmax).  FP32 keeps them scaled by log2(e) for the hardware exp2;
// FP64 keeps them plain for exp.
template <typename R>
struct Decay;

template <>
struct Decay<float> {
    float a, b;  // log2(e)/tau, log2(e)/gamma_c
    __device__ __forceinline__ explicit Decay(const ChanDev *c)
        : a((float)c->l2_tau), b((float)c->l2_gc) {}
};

template <>
struct Decay<double> {
    double a, b;  // 1/tau, 1/gamma_c
    __device__ __forceinline__ explicit Decay(const ChanDev *c)
        : a(c->inv_tau), b(c->inv_gc) {}
};

// ---------------------------------------------------------------------------
// Velocity gradient kappa_ab = d_b u_a by second-order differences
// (Sec. III): periodic central in x; central in y away from the walls; at the
// wall rows the three-point stencil through the no-slip value at the halfway
// wall, d_y u(0) = u(0) + u(1)/3 and d_y u(ly-1) = -u(ly-1) - u(ly-2)/3.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void velocity_gradient(const R *__restrict__ ux,
                                                  const R *__restrict__ uy,
                                                  int lx, int ly, int x, int y,
                                                  R &kxx, R &kxy, R &kyx,
                                                  R &kyy)
{
    const int n = y * lx + x;
    const int row = y * lx;
    const int xp = (x + 1 == lx) ? 0 : x + 1;
    const int xm = (x == 0) ? lx - 1 : x - 1;
    kxx = R(0.5) * (ux[row + xp] - ux[row + xm]);
    kyx = R(0.5) * (uy[row + xp] - uy[row + xm]);
    if (y == 0) {
        kxy = ux[n] + ux[n + lx] / R(3);
        kyy = uy[n] + uy[n + lx] / R(3);
    } else if (y == ly - 1) {
        kxy = -ux[n] - ux[n - lx] / R(3);
        kyy = -uy[n] - uy[n - lx] / R(3);
    } else {
        kxy = R(0.5) * (ux[n + lx] - ux[n - lx]);
        kyy = R(0.5) * (uy[n + lx] - uy[n - lx]);
    }
}

// |gamma_dot| = sqrt(II_D), II_D = (1/2) tr D^2, D = kappa + kappa^T (Sec. II).
template <typename R>
__device__ __forceinline__ R shear_rate(R kxx, R kxy, R kyx, R kyy)
{
    const R o = kxy + kyx;
    return sqrt(R(2) * kxx * kxx + o * o + R(2) * kyy * kyy);
}

// ---------------------------------------------------------------------------
// Initialisation: populations n*(-1) such that the first pull-stream yields
// n(0) = n^eq(1, u0) (the streaming map inverted, bounce-back included), and
// zero stress.  The moments of step -1 are rho - 1 = 0 and u = u0 (in split
// storage the remainders are taken against them).  One channel per launch.
// ---------------------------------------------------------------------------
template <typename P, typename S>
__global__ __launch_bounds__(kBlock) void k_init(char *__restrict__ ws,
                                                 const ChanDev *__restrict__ chans,
                                                 int ch,
                                                 const double *__restrict__ u0)
{
    constexpr bool kSplit = sizeof(S) < sizeof(P);
    const ChanDev *c = chans + ch;
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= c->n)
        return;
    const int lx = c->lx, ly = c->ly, np = c->np, N = c->n;
    const int y = n / lx, x = n - y * lx;
    S *pop = reinterpret_cast<S *>(ws + c->off_pop);
    S *read0 = pop + 9 * (size_t)np;  // buffer pulled from at t = 0
    const double ux0 = u0 ? u0[n] : 0.0;
    const double uy0 = u0 ? u0[N + n] : 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int yt = y + QY[q];
        int src = n, sq = QOPP[q];
        if (yt >= 0 && yt < ly) {
            int xt = x + QX[q];
            xt = xt < 0 ? xt + lx : (xt >= lx ? xt - lx : xt);
            src = yt * lx + xt;
            sq = q;
        }
        const double ux = u0 ? u0[src] : 0.0;
        const double uy = u0 ? u0[N + src] : 0.0;
        const double cu = QX[sq] * ux + QY[sq] * uy;
        const double uu = ux * ux + uy * uy;
        const double dev =
            qweight<double>(sq) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        if constexpr (kSplit) {
            const double cu_own = QX[q] * ux0 + QY[q] * uy0;
            read0[q * (size_t)np + n] =
                (S)(dev - eq_dev<double>(qweight<double>(q), cu_own, 0.0, ux0 * ux0 + uy0 * uy0));
        } else {
            read0[q * (size_t)np + n] = (S)dev;
        }
        pop[q * (size_t)np + n] = S(0);
    }
    if constexpr (kSplit) {
        P *mom = reinterpret_cast<P *>(ws + c->off_mom);
        mom[n] = P(0);
        mom[np + n] = P(0);
        mom[2 * (size_t)np + n] = P(0);
        P *m1 = mom + 3 * (size_t)np;  // step -1
        m1[n] = P(0);
        m1[np + n] = (P)ux0;
        m1[2 * (size_t)np + n] = (P)uy0;
    }
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    P *vel = reinterpret_cast<P *>(ws + c->off_vel);
    P *rho = reinterpret_cast<P *>(ws + c->off_rho);
    sig[n] = P(0);
    sig[np + n] = P(0);
    vel[n] = (P)ux0;
    vel[np + n] = (P)uy0;
    rho[n] = P(0);
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(uint4 *__restrict__ p,
                                                      size_t n16)
{
    const uint4 z = {0u, 0u, 0u, 0u};
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * kBlock)
        p[i] = z;
}

// ---------------------------------------------------------------------------
// The paper's own coupling (Sec. III, Eqs. bodyforce and hydrofields): the
// traceless stress sbar = sigma - (tr sigma / 2) I of step t-1 enters the
// second moment of the forcing term, its trace through the density rate
// dr = d_t delta rho = -(tr sigma^{t-1} - tr sigma^{t-2}) / (2 cs2);
// rho = sum n + dr / 2, the force is the external rho g only, and
//   F_q = a_q { -sbar:(c c - cs2 I) / (2 cs2^2 tau) + (1 - 1/(2 tau))
//          [dr + c.f / cs2 + (c c - cs2 I):(-dr u u + u f + f u) / (2 cs2^2)] },
// which in D2Q9 (cs2 = 1/3, sbar traceless) reads
//   a_q { -4.5 omega (sbar_xx (cx^2 - cy^2) + 2 sbar_xy cx cy)
//         + (1 - omega/2) [dr + 3 c.f + 9 (c.u)(c.f) - 3 u.f
//                          - 4.5 dr (c.u)^2 + 1.5 dr u.u] }.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void lb_collide_paper(char *__restrict__ ws, const ChanDev *c, int n,
                                                 size_t np, const R (&d)[9], R drho, R jx,
                                                 R jy, R (&out)[9], R &ux, R &uy, R &drho_out)
{
    const R *__restrict__ sxy = reinterpret_cast<const R *>(ws + c->off_sig);
    const R *__restrict__ sxx = sxy + np;
    const R syy = c->finger ? sxy[2 * np + n] : R(0);
    R *trp = reinterpret_cast<R *>(ws + c->off_trace);
    const R tr1 = sxx[n] + syy;
    const R dr = R(-1.5) * (tr1 - trp[n]);
    trp[n] = tr1;
    drho += R(0.5) * dr;
    const R rho = R(1) + drho;
    const R fx = rho * (R)c->gx, fy = rho * (R)c->gy;
    ux = (jx + R(0.5) * fx) / rho;
    uy = (jy + R(0.5) * fy) / rho;
    const R bxx = R(0.5) * (sxx[n] - syy), bxy = sxy[n];
    const R om = (R)c->omega;
    const R pf = R(1) - R(0.5) * om;
    const R uu = ux * ux + uy * uy;
    const R uf = ux * fx + uy * fy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const R cx = R(QX[q]), cy = R(QY[q]);
        const R cu = cx * ux + cy * uy;
        const R cf = cx * fx + cy * fy;
        const R w = qweight<R>(q);
        const R deq = w * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
        const R st = bxx * (cx * cx - cy * cy) + R(2) * bxy * cx * cy;
        const R F = w * (R(-4.5) * om * st +
                         pf * (dr + R(3) * (cf - uf) + R(9) * cu * cf - R(4.5) * dr * cu * cu +
                               R(1.5) * dr * uu));
        out[q] = d[q] - om * (d[q] - deq) + F;
    }
    drho_out = drho;
}

// ---------------------------------------------------------------------------
// Lattice phase of step t.
// ---------------------------------------------------------------------------
// Pull-stream of node n from the post-collision planes `src` (plane stride
// ss): n_q(x, y) = n*_q(x - c_q); through a wall, the population that left in
// the opposite direction comes back (halfway bounce-back).
template <typename R>
__device__ __forceinline__ void lb_pull(const ChanDev *c, int n, const R *__restrict__ src,
                                        size_t ss, R (&d)[9])
{
    const int lx = c->lx, ly = c->ly;
    const int y = n / lx, x = n - y * lx;
    const int xp = (x + 1 == lx) ? 0 : x + 1;
    const int xm = (x == 0) ? lx - 1 : x - 1;
    const bool lo = y > 0, hi = y < ly - 1;
    const int rowm = (y - 1) * lx, row = y * lx, rowp = (y + 1) * lx;
    d[0] = src[n];
    d[1] = src[1 * ss + row + xm];
    d[2] = src[2 * ss + row + xp];
    d[3] = lo ? src[3 * ss + rowm + x] : src[4 * ss + n];
    d[4] = hi ? src[4 * ss + rowp + x] : src[3 * ss + n];
    d[5] = lo ? src[5 * ss + rowm + xm] : src[6 * ss + n];
    d[6] = hi ? src[6 * ss + rowp + xp] : src[5 * ss + n];
    d[7] = hi ? src[7 * ss + rowp + xm] : src[8 * ss + n];
    d[8] = lo ? src[8 * ss + rowm + xp] : src[7 * ss + n];
}

// Moments of the deviations n_q - a_q: rho - 1 and j.
template <typename R>
__device__ __forceinline__ void lb_moments(const R (&d)[9], R &drho, R &jx, R &jy)
{
    drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    jx = (d[1] - d[2]) + (d[5] - d[6]) + (d[7] - d[8]);
    jy = (d[3] - d[4]) + (d[5] - d[6]) + (d[8] - d[7]);
}

// Body-force collision of node n: moments of the pulled deviations d, force
// density rho g + div sigma^{t-1} from the stress planes `sg` (plane stride
// gs: sigma_xy, sigma_xx, and sigma_yy with the full tensor), velocity with
// the half-force shift, BGK + forcing term.  Post-collision deviations in
// `out`.
template <typename R>
__device__ __forceinline__ void lb_collide_body(const ChanDev *c, int n, const R (&d)[9],
                                                const R *__restrict__ sg, size_t gs,
                                                R (&out)[9], R &ux, R &uy, R &drho)
{
    const int lx = c->lx, ly = c->ly;
    const int y = n / lx, x = n - y * lx;
    const int xp = (x + 1 == lx) ? 0 : x + 1;
    const int xm = (x == 0) ? lx - 1 : x - 1;
    const int row = y * lx;
    R jx, jy;
    lb_moments<R>(d, drho, jx, jy);
    const R rho = R(1) + drho;

    // Force density rho*g + div sigma^{t-1} (sigma_yy = 0 in the simple-shear
    // reduction, a third plane with the full tensor); d/dx periodic central,
    // d/dy central with one-sided rows at the walls.
    const R *__restrict__ sxy = sg;
    const R *__restrict__ sxx = sg + gs;
    auto ddy = [&](const R *__restrict__ f) {
        if (y == 0)
            return R(0.5) * (R(-3) * f[n] + R(4) * f[n + lx] - f[n + 2 * lx]);
        if (y == ly - 1)
            return R(0.5) * (R(3) * f[n] - R(4) * f[n - lx] + f[n - 2 * lx]);
        return R(0.5) * (f[n + lx] - f[n - lx]);
    };
    R fx = R(0.5) * (sxx[row + xp] - sxx[row + xm]) + ddy(sxy);
    R fy = R(0.5) * (sxy[row + xp] - sxy[row + xm]);
    if (c->finger)
        fy += ddy(sg + 2 * gs);
    fx += rho * (R)c->gx;
    fy += rho * (R)c->gy;

    // Velocity with the half-force shift (Eq. hydrofields).
    ux = (jx + R(0.5) * fx) / rho;
    uy = (jy + R(0.5) * fy) / rho;

    // BGK relaxation to the second-order equilibrium plus the forcing term
    // a_q (1 - 1/(2 tau_LB)) [(c - u).f / cs2 + (c.u)(c.f) / cs2^2]
    // (the f^ex part of Eq. bodyforce), all in deviation form.
    const R om = (R)c->omega;
    const R pf = R(1) - R(0.5) * om;
    const R uu = ux * ux + uy * uy;
    const R uf = ux * fx + uy * fy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const R cu = R(QX[q]) * ux + R(QY[q]) * uy;
        const R cf = R(QX[q]) * fx + R(QY[q]) * fy;
        const R w = qweight<R>(q);
        const R deq = w * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
        const R F = w * pf * (R(3) * (cf - uf) + R(9) * cu * cf);
        out[q] = d[q] - om * (d[q] - deq) + F;
    }
}

// ---------------------------------------------------------------------------
// Split population storage (LB_F32).  A post-collision population of node n
// is kept as the moments its collision used -- rho - 1, u_x, u_y in FP64,
// [2][3][np] by step parity -- and the FP32 remainder
//   r_q = n*_q - n^eq_q(rho, u),
// with n^eq the second-order equilibrium of Sec. III.  A pulled population is
// rebuilt in FP64 as n^eq_q(rho, u of the source node) + r_q.  The remainder
// is the forcing term plus (1 - 1/tau_LB) times the non-equilibrium part, some
// 1e-3 of the deviation n_q - a_q in the channels here, so FP32 rounding acts
// on that small part only, and the conserved moments carry no FP32 rounding
// from step to step.
// ---------------------------------------------------------------------------

// Population Q arriving at a node by a pull: through (the population left
// node na in direction Q) or bounced back (it left node nb in the opposite
// direction).  mom: the moment planes of the step it left (plane stride ss).
template <int Q, typename P>
__device__ __forceinline__ P pull_split_one(bool through, int na, int nb,
                                            const float *__restrict__ src,
                                            const P *__restrict__ mom, size_t ss)
{
#pragma clang fp contract(off)
    const int nd = through ? na : nb;
    const size_t plane = through ? (size_t)Q : (size_t)QOPP[Q];
    const P drho = mom[nd], ux = mom[ss + nd], uy = mom[2 * ss + nd];
    // c_opp(Q) = -c_Q
    const P cu0 = P(QX[Q]) * ux + P(QY[Q]) * uy;
    const P cu = through ? cu0 : -cu0;
    return eq_dev<P>(qweight<P>(Q), cu, drho, ux * ux + uy * uy) + (P)src[plane * ss + nd];
}

// Pull-stream of node n from split storage (the same sources as lb_pull).
template <typename P>
__device__ __forceinline__ void lb_pull_split(const ChanDev *c, int n,
                                              const float *__restrict__ src,
                                              const P *__restrict__ mom, size_t ss, P (&d)[9])
{
    const int lx = c->lx, ly = c->ly;
    const int y = n / lx, x = n - y * lx;
    const int xp = (x + 1 == lx) ? 0 : x + 1;
    const int xm = (x == 0) ? lx - 1 : x - 1;
    const bool lo = y > 0, hi = y < ly - 1;
    const int rowm = (y - 1) * lx, row = y * lx, rowp = (y + 1) * lx;
    d[0] = pull_split_one<0, P>(true, n, n, src, mom, ss);
    d[1] = pull_split_one<1, P>(true, row + xm, n, src, mom, ss);
    d[2] = pull_split_one<2, P>(true, row + xp, n, src, mom, ss);
    d[3] = pull_split_one<3, P>(lo, rowm + x, n, src, mom, ss);
    d[4] = pull_split_one<4, P>(hi, rowp + x, n, src, mom, ss);
    d[5] = pull_split_one<5, P>(lo, rowm + xm, n, src, mom, ss);
    d[6] = pull_split_one<6, P>(hi, rowp + xp, n, src, mom, ss);
    d[7] = pull_split_one<7, P>(hi, rowp + xm, n, src, mom, ss);
    d[8] = pull_split_one<8, P>(lo, rowm + xp, n, src, mom, ss);
}

// The node's own post-collision deviations n*_q - a_q rebuilt from split
// storage (for the adjoint's step record).
template <typename P>
__device__ __forceinline__ void own_split(int n, const float *__restrict__ src,
                                          const P *__restrict__ mom, size_t ss, P (&d)[9])
{
    d[0] = pull_split_one<0, P>(true, n, n, src, mom, ss);
    d[1] = pull_split_one<1, P>(true, n, n, src, mom, ss);
    d[2] = pull_split_one<2, P>(true, n, n, src, mom, ss);
    d[3] = pull_split_one<3, P>(true, n, n, src, mom, ss);
    d[4] = pull_split_one<4, P>(true, n, n, src, mom, ss);
    d[5] = pull_split_one<5, P>(true, n, n, src, mom, ss);
    d[6] = pull_split_one<6, P>(true, n, n, src, mom, ss);
    d[7] = pull_split_one<7, P>(true, n, n, src, mom, ss);
    d[8] = pull_split_one<8, P>(true, n, n, src, mom, ss);
}

// Remainders r_q = n*_q - n^eq_q(rho, u) of the post-collision deviations
// `out` of a node whose collision used (drho, ux, uy).
template <typename P>
__device__ __forceinline__ void split_remainders(const P (&out)[9], P ux, P uy, P drho,
                                                 float (&r)[9])
{
#pragma clang fp contract(off)
    const P uu = ux * ux + uy * uy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const P cu = P(QX[q]) * ux + P(QY[q]) * uy;
        r[q] = (float)(out[q] - eq_dev<P>(qweight<P>(q), cu, drho, uu));
    }
}

// Lattice update of node n at step t from and to the workspace.  S is the
// population storage type: P (plain deviations n_q - a_q) or float (split
// storage, P = double).
template <typename P, typename S>
__device__ __forceinline__ void lb_node(char *__restrict__ ws, const ChanDev *c, int n,
                                        int64_t t)
{
    constexpr bool kSplit = sizeof(S) < sizeof(P);
    const size_t np = (size_t)c->np;
    S *pop = reinterpret_cast<S *>(ws + c->off_pop);
    const S *__restrict__ src = pop + ((t + 1) & 1) * 9 * np;  // n*(t-1)
    S *__restrict__ dst = pop + (t & 1) * 9 * np;              // n*(t)
    P *mom = reinterpret_cast<P *>(ws + c->off_mom);           // split storage only
    const P *__restrict__ msrc = mom + ((t + 1) & 1) * 3 * np;
    const P *__restrict__ sig = reinterpret_cast<const P *>(ws + c->off_sig);
    if (c->rec) {
        P *rec = reinterpret_cast<P *>(c->rec) + (size_t)(t - c->rec_t0) * 10 * np;
        if constexpr (kSplit) {
            P own[9];
            own_split<P>(n, src, msrc, np, own);
#pragma unroll
            for (int q = 0; q < 9; ++q)
                rec[q * np + n] = own[q];
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q)
                rec[q * np + n] = src[q * np + n];
        }
        rec[9 * np + n] = sig[n];
    }
    P d[9];
    if constexpr (kSplit)
        lb_pull_split<P>(c, n, src, msrc, np, d);
    else
        lb_pull<P>(c, n, src, np, d);
    P out[9], ux, uy, drho;
    if (c->coupling) {
        P drho0, jx, jy;
        lb_moments<P>(d, drho0, jx, jy);
        lb_collide_paper<P>(ws, c, n, np, d, drho0, jx, jy, out, ux, uy, drho);
    } else {
        lb_collide_body<P>(c, n, d, sig, np, out, ux, uy, drho);
    }
    if constexpr (kSplit) {
        float r[9];
        split_remainders<P>(out, ux, uy, drho, r);
#pragma unroll
        for (int q = 0; q < 9; ++q)
            dst[q * np + n] = r[q];
        P *mdst = mom + (t & 1) * 3 * np;
        mdst[n] = drho;
        mdst[np + n] = ux;
        mdst[2 * np + n] = uy;
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q)
            dst[q * np + n] = out[q];
    }
    P *vel = reinterpret_cast<P *>(ws + c->off_vel);
    vel[n] = ux;
    vel[np + n] = uy;
    reinterpret_cast<P *>(ws + c->off_rho)[n] = drho;
}

// Node tile of workgroup b in a launch of n workgroups (one per tile).  The
// dispatcher deals the workgroups of a launch to the 8 XCDs in turn, so
// consecutive workgroups land in different L2 caches; giving each XCD a
// contiguous range of tiles (about n/8 of them, rows of a channel next to each
// other) keeps a stencil's neighbouring rows in the L2 that reads them.  A
// bijection of [0, n).
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int x = b % kXcds, i = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + min(x, r) + i;
}

template <typename P, typename S>
__global__ __launch_bounds__(kBlock, 5) void k_lb(char *__restrict__ ws,
                                               const ChanDev *__restrict__ chans,
                                               const NodeTile *__restrict__ tiles,
                                               const int64_t *__restrict__ tcount,
                                               int trel, int *__restrict__ tile_counters)
{
    const NodeTile tl = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    // The history pass of this step (if any) claims its tiles from these
    // counters; it runs after this kernel on the same stream.
    if (blockIdx.x == 0 && threadIdx.x < kTileCounters)
        tile_counters[threadIdx.x] = 0;
    if (n >= c->n)
        return;
    lb_node<P, S>(ws, c, n, *tcount + trel);
}

// ---------------------------------------------------------------------------
// History integral, blocked in time.
//
// Sums over the window at step t (Eq. gitt with Eq. nlmax, trapezoid weights
// w(a) = 1/2 at ages a = 0 and a = n_hist - 1, 1 inside):
//   sigma_xy(t) = G sum_e w(a) s_e E(a, r_e),
//   sigma_xx(t) = G sum_e w(a) 2 s_e gamma(t, e) E(a, r_e),
// a = t - e, E(a, r) = exp(-a (1/tau + r/gamma_c)),
// gamma(t, e) = s_e + ... + s_{t-1} (accumulated strain, Eq. eeval).
//
// Every entry but the newest is known before the step, so a pass over the
// ring at the first step t0 of a block of M steps serves all M steps: for
// m = 0..M-1 it forms, over the entries e <= t0 still in step t0+m's window,
//   A_m = sum w(k+m) s_e E(k+m, r_e),  B_m = sum w(k+m) 2 s_e gamma(t0, e) E(k+m, r_e)
// (k = t0 - e), with E(k+m) = E(k) q^m, q = exp(-(1/tau + r/gamma_c)).  At step
// t0 + m the entries pushed since t0 are added directly and, because
// gamma(t0+m, e) = gamma(t0, e) + Delta_m for every old entry with
// Delta_m = s_{t0} + ... + s_{t0+m-1},
//   sigma_xy = G (A_m + new),  sigma_xx = G (B_m + 2 Delta_m A_m + new).
//
// Pass layout: a wavefront owns 64*V consecutive nodes of one channel and one
// age range [k0, k1) (a tile; four per workgroup); lane l owns nodes
// n0 + V*l .. n0 + V*l + V-1 and reads them as one V-wide vector per ring row.  Ages are walked newest to
// oldest (the running FP64 strain gamma is a sum over the rows already
// read); rows are read in halves of U/2, the next half's loads issued before
// the current half is summed.  In FP32 the terms of F rows are added plainly
// and their sum enters a Kahan-compensated FP32 total.
// ---------------------------------------------------------------------------
template <typename R, int V>
struct alignas(sizeof(R) * V) Pack {
    R v[V];
};

// row: uniform row base; off: the lane's byte offset within the row.
template <typename R, int V>
__device__ __forceinline__ Pack<R, V> load_pack(const R *row, uint32_t off)
{
    return *reinterpret_cast<const Pack<R, V> *>(reinterpret_cast<const char *>(row) + off);
}

// Loads through a buffer resource (gfx9 raw buffer: 32-bit offsets to a
// base held in scalar registers).  A group of rows shares one resource whose
// base is the group's lowest row: the row is selected by the scalar offset (a
// multiple of the row length, the same for every group) and the lane by the
// 32-bit VGPR offset that every row shares, so neither needs a vector
// instruction per row and the scalar work per row is none.  Reads past the
// resource's `bytes` return zeros instead of touching memory.  Word 3 selects
// 32-bit raw data, the gfx9 form.
constexpr int kBufferWord3 = 0x00020000;

template <typename R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const R *base, uint32_t bytes)
{
    uint64_t a = reinterpret_cast<uint64_t>(base);
    asm volatile("" : "+s"(a));  // uniform: the resource stays in scalar registers
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(a), (short)0, (int)bytes,
                                             kBufferWord3);
}

template <typename R, int V>
__device__ __forceinline__ Pack<R, V> load_pack_rsrc(__amdgpu_buffer_rsrc_t rs, uint32_t off,
                                                     uint32_t soff)
{
    constexpr int B = (int)sizeof(R) * V;
    static_assert(B == 4 || B == 8 || B == 16 || B == 32, "pack size");
    Pack<R, V> r;
    if constexpr (B == 4) {
        const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, (int)soff, 0);
        __builtin_memcpy(&r, &x, 4);
    } else if constexpr (B == 8) {
        typedef uint32_t U2 __attribute__((ext_vector_type(2)));
        const U2 x = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, (int)soff, 0);
        __builtin_memcpy(&r, &x, 8);
    } else if constexpr (B == 16) {
        typedef uint32_t U4 __attribute__((ext_vector_type(4)));
        const U4 x = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, (int)soff, 0);
        __builtin_memcpy(&r, &x, 16);
    } else {
        typedef uint32_t U4 __attribute__((ext_vector_type(4)));
        const U4 x0 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, (int)soff, 0);
        const U4 x1 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off + 16, (int)soff, 0);
        __builtin_memcpy(&r, &x0, 16);
        __builtin_memcpy(reinterpret_cast<char *>(&r) + 16, &x1, 16);
    }
    return r;
}

// float(u) for a wave-uniform 0 <= u < 2^24 (exact), built from its bits with
// integer operations in scalar registers, so it enters the vector
// instructions as a scalar operand instead of a per-row vector conversion
// (the empty asm keeps the compiler from turning it back into one).
__device__ __forceinline__ float small_uniform_to_float(uint32_t u)
{
    const int e = 31 - __builtin_clz(u | 1u);  // u = 0 is selected below
    uint32_t bits = ((uint32_t)(e + 127) << 23) | ((u << (23 - e)) & 0x7FFFFFu);
    bits = u ? bits : 0u;
    asm volatile("" : "+s"(bits));
    return __builtin_bit_cast(float, bits);
}

__device__ __forceinline__ float fused(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fused(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R>
__device__ __forceinline__ R decay_rate(const Decay<R> &dec, R r)
{
    return fused(dec.b, r, dec.a);
}

// exp(-k * rate) in the precision's form (rate pre-scaled by log2(e) in FP32).
__device__ __forceinline__ float decay_pow(float k, float rate)
{
    return __builtin_amdgcn_exp2f(-k * rate);
}
__device__ __forceinline__ double decay_pow(double k, double rate)
{
    return exp(-k * rate);
}

// An entry whose ages touch a window end (age 0 at t0, or age k + m at the
// far end for some m): per-m weight and window membership, direct exp.
template <typename R, int M>
__device__ __forceinline__ void edge_entry(R s, R r, int k, int H, double loc,
                                           const Decay<R> &dec, Acc<R> (&A)[M],
                                           Acc<R> (&B)[M])
{
#pragma clang fp contract(off)
    const R rate = decay_rate<R>(dec, r);
    const R g = (R)loc;  // gamma; the factor 2 is applied to the finished B sums
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int a = k + m;
        if (a <= H - 1) {
            const R w = (a == 0 || a == H - 1) ? R(0.5) : R(1);
            const R se = w * s * decay_pow(R(a), rate);
            A[m].add(se);
            B[m].add(se * g);
        }
    }
}

// The same terms for an entry near the far end of the window (some k + m
// past it), into plain partial sums flushed once after the last such entry:
// E(k + m) carried as E(k) q^m.
template <typename R, int M>
__device__ __forceinline__ void tail_entry(R s, R r, int k, int H, R g, const Decay<R> &dec,
                                           R (&pa)[M], R (&pb)[M])
{
#pragma clang fp contract(off)
    const R rate = decay_rate<R>(dec, r);
    const R q = decay_pow(R(1), rate);
    R e = decay_pow(R(k), rate);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int a = k + m;
        if (a <= H - 1) {
            const R w = a == H - 1 ? R(0.5) : R(1);
            const R se = w * s * e;
            pa[m] = pa[m] + se;
            pb[m] = fused(se, g, pb[m]);
        }
        if (m + 1 < M)
            e = e * q;
    }
}

// One entry's terms for the M steps of a block: x q^m into pa[m][v] and
// x q^m g2 into pb[m][v] (g2 the entry's strain factor), m = 0..M-1 (SET: the first entry of a group sets
// them).  For M >= 16, x q^m = q^{m mod 8} (x q^{8 (m / 8)}): seven low
// powers of q, M/8 high powers carrying x and M/8 carrying x g2, one FMA
// (an add for m mod 8 = 0) per sum and step; shorter blocks carry x q^m
// along m.
template <typename R, int M, int V, bool SET>
__device__ __forceinline__ void add_powers(R x, R q, R g2, R (&pa)[M][V], R (&pb)[M][V],
                                           int v)
{
#pragma clang fp contract(off)
    if constexpr (M >= 16 && M % 8 == 0) {
        constexpr int MH = M / 8;
        R lo[8], hx[MH], hg[MH];
        lo[1] = q;
#pragma unroll
        for (int i = 2; i < 8; ++i)
            lo[i] = lo[i - 1] * q;
        const R q8 = lo[4] * lo[4];
        hx[0] = x;
#pragma unroll
        for (int j = 1; j < MH; ++j)
            hx[j] = hx[j - 1] * q8;
#pragma unroll
        for (int j = 0; j < MH; ++j)
            hg[j] = hx[j] * g2;
#pragma unroll
        for (int j = 0; j < MH; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int m = 8 * j + i;
                if (SET) {
                    pa[m][v] = i == 0 ? hx[j] : lo[i] * hx[j];
                    pb[m][v] = i == 0 ? hg[j] : lo[i] * hg[j];
                } else {
                    pa[m][v] = i == 0 ? pa[m][v] + hx[j] : fused(lo[i], hx[j], pa[m][v]);
                    pb[m][v] = i == 0 ? pb[m][v] + hg[j] : fused(lo[i], hg[j], pb[m][v]);
                }
            }
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (SET) {
                pa[m][v] = x;
                pb[m][v] = x * g2;
            } else {
                pa[m][v] += x;
                pb[m][v] = fused(x, g2, pb[m][v]);
            }
            if (m + 1 < M)
                x *= q;
        }
    }
}

// Loads of U ring rows, slots slot, slot - 1, ..., slot - U + 1 (all >= 0),
// at the lane's byte offset `off`.  The rows lie (U - 1 - u) row lengths above
// the group's lowest row; the host limits channels so that U rows of a ring
// plane span less than 4 GiB.
template <typename R, int V, int U, bool HAS_R>
__device__ __forceinline__ void load_rows(const R *__restrict__ ring_s,
                                          const R *__restrict__ ring_r, size_t np,
                                          uint32_t off, int slot, Pack<R, V> (&sv)[U],
                                          Pack<R, V> (&rv)[U])
{
    static_assert(U <= 8, "the channel size limit keeps 8 rows of a plane below 4 GiB");
    const uint32_t row_bytes = (uint32_t)(np * sizeof(R));
    const size_t low = (size_t)(slot - (U - 1)) * np;
    const __amdgpu_buffer_rsrc_t rs = row_rsrc<R>(ring_s + low, (uint32_t)U * row_bytes);
    __amdgpu_buffer_rsrc_t rr = rs;
    if (HAS_R)
        rr = row_rsrc<R>(ring_r + low, (uint32_t)U * row_bytes);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t soff = (uint32_t)(U - 1 - u) * row_bytes;
        sv[u] = load_pack_rsrc<R, V>(rs, off, soff);
        if (HAS_R)
            rv[u] = load_pack_rsrc<R, V>(rr, off, soff);
    }
}

// The terms of U loaded rows of interior ages kf0, kf0 + 1, ...: the plain
// partial sums pa, pb take x = s E(k+m) (carried along m by the per-entry
// factor q) and x * gamma; FIRST starts them from these rows.
template <typename R, int V, int M, int U, bool HAS_R, bool FIRST>
__device__ __forceinline__ void sum_rows(const Pack<R, V> (&sv)[U], const Pack<R, V> (&rv)[U],
                                         int kf0, const Decay<R> &dec, R (&pa)[M][V],
                                         R (&pb)[M][V], double (&loc)[V])
{
    // No implicit contraction: every lane width and group size rounds the
    // same operations the same way (the FMAs are written out).
#pragma clang fp contract(off)
#pragma unroll
    for (int u = 0; u < U; ++u) {
        // ages stay below 2^24 in FP32 histories (the window is limited to
        // that), where the scalar construction equals the vector conversion
        const R kf = sizeof(R) == 4
                         ? R(small_uniform_to_float((uint32_t)__builtin_amdgcn_readfirstlane(kf0 + u)))
                         : R(kf0 + u);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R s = sv[u].v[v];
            const R rate = decay_rate<R>(dec, HAS_R ? rv[u].v[v] : fabs(s));
            loc[v] += (double)s;
            // gamma (not 2 gamma): doubling the finished B sums is exact
            const R g = (R)loc[v];
            R x = s * decay_pow(kf, rate);
            R q = R(1);
            if (M > 1)
                q = decay_pow(R(1), rate);
            if (FIRST && u == 0)
                add_powers<R, M, V, true>(x, q, g, pa, pb, v);
            else
                add_powers<R, M, V, false>(x, q, g, pa, pb, v);
        }
    }
}

// U rows of interior ages: entry k + j0 + u sits at ring slot `slot - j0 - u`.
template <typename R, int V, int M, int U, bool HAS_R, bool FIRST>
__device__ __forceinline__ void pass_rows(const R *__restrict__ ring_s,
                                          const R *__restrict__ ring_r, size_t np,
                                          uint32_t lane_off, int slot, int kf0,
                                          const Decay<R> &dec, R (&pa)[M][V], R (&pb)[M][V],
                                          double (&loc)[V])
{
    Pack<R, V> sv[U], rv[U];
    load_rows<R, V, U, HAS_R>(ring_s, ring_r, np, lane_off, slot, sv, rv);
    sum_rows<R, V, M, U, HAS_R, FIRST>(sv, rv, kf0, dec, pa, pb, loc);
}

template <typename R, int V, int M>
__device__ __forceinline__ void flush(const R (&pa)[M][V], const R (&pb)[M][V],
                                      Acc<R> (&A)[M][V], Acc<R> (&B)[M][V])
{
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            A[m][v].add(pa[m][v]);
            B[m][v].add(pb[m][v]);
        }
}

// Interior ages [k, kend) of one chunk: every m has weight 1 and is in the
// window.  Rows are visited newest to oldest, wrapping at row 0.  The plain
// partial sums enter the compensated totals every F rows (F a multiple of
// U), then every U/2 (or U) rows near the end of a run, then row by row.
// In the F-row blocks the rows go in two halves of U/2 that alternate: the
// loads of one half are issued before the terms of the other are summed, so
// the load latency is hidden behind the arithmetic of the wavefront itself
// (the register cost is that of U rows).  The half after a run's last F-row
// block is loaded from clamped, in-bounds rows and not used.
template <typename R, int V, int M, int U, int F, bool HAS_R>
__device__ __forceinline__ void pass_bulk(const R *__restrict__ ring_s,
                                          const R *__restrict__ ring_r, size_t np,
                                          uint32_t lane_off, int H, int p, int k, int kend,
                                          const Decay<R> &dec, Acc<R> (&A)[M][V],
                                          Acc<R> (&B)[M][V], double (&loc)[V])
{
    static_assert(F % U == 0, "flush length must be a multiple of the row group");
    constexpr int U2 = U / 2;
    int slot = p - k;
    if (slot < 0)
        slot += H;
    while (k < kend) {
        const int run = min(kend - k, slot + 1);  // rows down to 0 without wrap
        int j = 0;
        R pa[M][V], pb[M][V];
        if constexpr (F > U && U % 2 == 0) {
            const uint32_t off = lane_off;
            Pack<R, V> as[U2], ar[U2], bs[U2], br[U2];
            if (run >= F)
                load_rows<R, V, U2, HAS_R>(ring_s, ring_r, np, off, slot, as, ar);
            for (; j + F <= run; j += F) {
                // inside the block every row index is >= slot - run + 1 >= 0
                load_rows<R, V, U2, HAS_R>(ring_s, ring_r, np, off, slot - j - U2, bs,
                                           br);
                sum_rows<R, V, M, U2, HAS_R, true>(as, ar, k + j, dec, pa, pb, loc);
                for (int g = U2; g < F; g += U) {
                    // the next rows: past the block's end they belong to the
                    // next block, or to no block (clamped to rows U2 - 1 .. 0)
                    load_rows<R, V, U2, HAS_R>(ring_s, ring_r, np, off,
                                               max(slot - j - g - U2, U2 - 1), as, ar);
                    sum_rows<R, V, M, U2, HAS_R, false>(bs, br, k + j + g, dec, pa, pb, loc);
                    if (g + U2 < F) {
                        load_rows<R, V, U2, HAS_R>(ring_s, ring_r, np, off,
                                                   slot - j - g - U, bs, br);
                        sum_rows<R, V, M, U2, HAS_R, false>(as, ar, k + j + g + U2, dec, pa,
                                                            pb, loc);
                    }
                }
                flush<R, V, M>(pa, pb, A, B);
            }
        }
        // the rest of the run in groups of UR rows (the half group where the
        // blocks above alternate halves: no more registers than they use)
        constexpr int UR = (F > U && U % 2 == 0) ? U2 : U;
        for (; j + UR <= run; j += UR) {
            pass_rows<R, V, M, UR, HAS_R, true>(ring_s, ring_r, np, lane_off, slot - j, k + j,
                                                dec, pa, pb, loc);
            flush<R, V, M>(pa, pb, A, B);
        }
        for (; j < run; ++j) {
            pass_rows<R, V, M, 1, HAS_R, true>(ring_s, ring_r, np, lane_off, slot - j, k + j,
                                               dec, pa, pb, loc);
            flush<R, V, M>(pa, pb, A, B);
        }
        k += run;
        slot = H - 1;
    }
}

template <typename P, typename R, int V, int M, int U, int F, bool HAS_R>
__device__ __forceinline__ void pass_tile(char *__restrict__ ws, const ChanDev *c,
                                          const HistTile &tl, int64_t t)
{
    const int H = c->n_hist;
    const size_t np = (size_t)c->np;
    const int first = tl.n0 + (int)(threadIdx.x % kWave) * V;  // lane's first node
    // A lane past the channel end shadows the last vector of the channel (in
    // bounds, results discarded); nodes past the end inside a vector read the
    // zero padding of the ring.
    const int lane_node = first < c->n ? first : ((c->n - 1) / V) * V;
    const uint32_t lane_off = (uint32_t)lane_node * (uint32_t)sizeof(R);
    const int p = (int)(t % H);
    R *ring_s = reinterpret_cast<R *>(ws + c->off_ring_s);
    R *ring_r = reinterpret_cast<R *>(ws + c->off_ring_r);
    const Decay<R> dec(c);
    Acc<R> A[M][V], B[M][V];
    double loc[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
        loc[v] = 0.0;
    int k = tl.k0;
    if (k == 0) {
        // Newest entry, age 0: gradient of this step's velocity, push it.
        const P *vel = reinterpret_cast<const P *>(ws + c->off_vel);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int node = first + v;
            R s = R(0), r = R(0);
            if (node < c->n) {
                const int y = node / c->lx, x = node - y * c->lx;
                P kxx, kxy, kyx, kyy;
                velocity_gradient<P>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx,
                                     kyy);
                s = (R)kxy;
                r = HAS_R ? (R)shear_rate<P>(kxx, kxy, kyx, kyy) : fabs(s);
                ring_s[(size_t)p * np + node] = s;
                if (HAS_R)
                    ring_r[(size_t)p * np + node] = r;
            }
            Acc<R> a1[M], b1[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                a1[m] = A[m][v];
                b1[m] = B[m][v];
            }
            edge_entry<R, M>(s, r, 0, H, 0.0, dec, a1, b1);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                A[m][v] = a1[m];
                B[m][v] = b1[m];
            }
        }
        k = 1;
    }
    // Interior ages, then the ages whose k + m reaches the window end.
    const int tail0 = max(k, H - M);
    pass_bulk<R, V, M, U, F, HAS_R>(ring_s, ring_r, np, lane_off, H, p, k, min(tl.k1, tail0),
                                 dec, A, B, loc);
    if (max(k, tail0) < tl.k1) {
        R ta[V][M], tb[V][M];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int m = 0; m < M; ++m)
                ta[v][m] = tb[v][m] = R(0);
        for (int kk = max(k, tail0); kk < tl.k1; ++kk) {
            int slot = p - kk;
            if (slot < 0)
                slot += H;
            const size_t row = (size_t)slot * np;
            const Pack<R, V> sv = load_pack<R, V>(ring_s + row, lane_off);
            Pack<R, V> rv;
            if (HAS_R)
                rv = load_pack<R, V>(ring_r + row, lane_off);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const R s = sv.v[v];
                loc[v] += (double)s;
                tail_entry<R, M>(s, HAS_R ? rv.v[v] : fabs(s), kk, H, (R)loc[v], dec, ta[v],
                                 tb[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                A[m][v].add(ta[v][m]);
                B[m][v].add(tb[v][m]);
            }
    }
    if (first >= c->n)
        return;
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    double *part = reinterpret_cast<double *>(ws + c->off_part);
    double *blk = reinterpret_cast<double *>(ws + c->off_blk);
    const size_t pplane = (size_t)c->max_chunks * np;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int node = first + v;
        if (node >= c->n)
            break;
        // B was summed with gamma for 2 gamma: doubling is exact
        if (c->nchunks == 1) {
            sig[node] = (P)(c->g_inf * A[0][v].value());
            sig[np + node] = (P)(c->g_inf * (2.0 * B[0][v].value()));
#pragma unroll
            for (int m = 1; m < M; ++m) {
                blk[m * np + node] = A[m][v].value();
                blk[(kPlaneB + m) * np + node] = 2.0 * B[m][v].value();
            }
        } else {
            const size_t at = (size_t)tl.chunk * np + node;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                part[m * pplane + at] = A[m][v].value();
                part[(kPlaneB + m) * pplane + at] = 2.0 * B[m][v].value();
            }
            part[kPlaneT * pplane + at] = loc[v];
        }
    }
}

// One launch per (lane width V, block length M): the tiles of the channels
// whose lane width is V, one wavefront per tile (64 V nodes), so channels
// narrower than a workgroup leave no wavefront idle.  Plain form: the four
// wavefronts of workgroup b take tiles 4b .. 4b + 3.
// FP32 histories fit two wavefronts per SIMD at 32 steps per pass (the bound
// is needed to get there) and three at 16; FP64 ones keep the default.
template <typename R, int M>
constexpr int pass_waves_per_simd()
{
    return sizeof(R) == 4 ? (M <= 16 ? 3 : 2) : 1;
}

template <typename P, typename R, int V, int M, int U, int F>
__global__ __launch_bounds__(kBlock, (pass_waves_per_simd<R, M>())) void k_hist_pass(char *__restrict__ ws,
                                                      const ChanDev *__restrict__ chans,
                                                      const HistTile *__restrict__ tiles,
                                                      int n_tiles,
                                                      const int64_t *__restrict__ tcount,
                                                      int trel)
{
    // wave-uniform, so the tile and channel fields stay in scalar registers
    const int i = (int)blockIdx.x * (kBlock / kWave) +
                  __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (i >= n_tiles)
        return;  // the last workgroup's spare wavefronts
    const HistTile tl = tiles[i];
    const ChanDev *c = chans + tl.ch;
    const int64_t t = *tcount + trel;
    if (c->has_r)
        pass_tile<P, R, V, M, U, F, true>(ws, c, tl, t);
    else
        pass_tile<P, R, V, M, U, F, false>(ws, c, tl, t);
}

// Persistent form: as many workgroups as fit on the chip at once; each
// wavefront claims the next tile of the list (longest first) from a counter
// until the list is exhausted.  The counter was zeroed by the lattice kernel
// of this step.
template <typename P, typename R, int V, int M, int U, int F>
__global__ __launch_bounds__(kBlock, (pass_waves_per_simd<R, M>())) void k_hist_pass_persistent(
    char *__restrict__ ws, const ChanDev *__restrict__ chans,
    const HistTile *__restrict__ tiles, int n_tiles, const int64_t *__restrict__ tcount,
    int trel, int *__restrict__ counter)
{
    const int64_t t = *tcount + trel;
    const bool leader = threadIdx.x % kWave == 0;
    for (;;) {
        int i = 0;
        if (leader)
            i = atomicAdd(counter, 1);
        i = __builtin_amdgcn_readfirstlane(i);  // the claim of the first lane, wave-uniform
        if (i >= n_tiles)
            break;  // uniform across the wavefront
        const HistTile tl = tiles[i];
        const ChanDev *c = chans + tl.ch;
        if (c->has_r)
            pass_tile<P, R, V, M, U, F, true>(ws, c, tl, t);
        else
            pass_tile<P, R, V, M, U, F, false>(ws, c, tl, t);
    }
}

// ---------------------------------------------------------------------------
// Full-tensor Finger path (Eq. gitt with -d_t'B = E kappa E^T + transpose,
// E(t, t') the ordered product of exp(kappa dt), Eq. eeval).
//
// Ring of a full-tensor channel: 8 planes [8][n_hist][np] -- kappa_xx,
// kappa_xy, kappa_yx, kappa_yy of the entry, then g = exp(kappa dt) - I
// row-major (formed once, in FP64, when the entry is pushed; kept apart from
// the identity so FP32 storage keeps its precision).
// Walking ages newest to oldest, E_k = E_{k-1} (I + g_k) in FP64 (E_0 = I:
// the newest entry contributes no factor), and the entry's term is
// P_k = E_k kappa_k E_k^T + transpose (symmetric: xx, xy, yy).  With the
// damping unchanged, a pass at t0 forms for m = 0..M-1
//   S_m = sum w(k+m) P_k E(k+m, r_k)
// (E the damping factor as in the reduced path), and step t0 + m has
//   sigma = G (E_m S_m E_m^T + terms of the entries pushed since t0),
// E_m = E(t0 + m, t0): the deformation since the pass is a common left
// factor of every older entry's deformation, so the blocking carries over.
// A window split into age ranges keeps, per range, its sums and its total
// product T_c; the combine forms sum_c O_c S_c O_c^T with O_c = T_0 ... T_{c-1}.
// ---------------------------------------------------------------------------
struct Mat2 {
    double a, b, c, d;  // [[a, b], [c, d]]
};

__device__ __forceinline__ Mat2 mat_mul(const Mat2 &x, const Mat2 &y)
{
    return {fma(x.a, y.a, x.b * y.c), fma(x.a, y.b, x.b * y.d), fma(x.c, y.a, x.d * y.c),
            fma(x.c, y.b, x.d * y.d)};
}

// E (I + g) = E + E g
__device__ __forceinline__ Mat2 step_deformation(const Mat2 &E, double g00, double g01,
                                                 double g10, double g11)
{
    return {fma(E.a, g00, fma(E.b, g10, E.a)), fma(E.a, g01, fma(E.b, g11, E.b)),
            fma(E.c, g00, fma(E.d, g10, E.c)), fma(E.c, g01, fma(E.d, g11, E.d))};
}

// P = E k E^T + (E k E^T)^T as (xx, xy, yy)
__device__ __forceinline__ void finger_term(const Mat2 &E, double kxx, double kxy, double kyx,
                                            double kyy, double &pxx, double &pxy,
                                            double &pyy)
{
    const double ea = fma(E.a, kxx, E.b * kyx), eb = fma(E.a, kxy, E.b * kyy);
    const double ec = fma(E.c, kxx, E.d * kyx), ed = fma(E.c, kxy, E.d * kyy);
    pxx = 2.0 * fma(ea, E.a, eb * E.b);
    pxy = fma(ea, E.c, eb * E.d) + fma(ec, E.a, ed * E.b);
    pyy = 2.0 * fma(ec, E.c, ed * E.d);
}

// S -> O S O^T for symmetric S = (xx, xy, yy)
__device__ __forceinline__ void congruence(const Mat2 &O, double &sxx, double &sxy,
                                           double &syy)
{
    const double xa = fma(O.a, sxx, O.b * sxy), xb = fma(O.a, sxy, O.b * syy);
    const double xc = fma(O.c, sxx, O.d * sxy), xd = fma(O.c, sxy, O.d * syy);
    const double nxx = fma(xa, O.a, xb * O.b);
    const double nxy = fma(xa, O.c, xb * O.d);
    const double nyy = fma(xc, O.c, xd * O.d);
    sxx = nxx;
    sxy = nxy;
    syy = nyy;
}

// g = exp(K) - I for a 2x2 K (the velocity gradient of one step), formed
// when an entry is pushed.
// Cayley-Hamilton: with s = tr K / 2, h = (K_xx - K_yy)/2 and
// q^2 = h^2 + K_xy K_yx (the eigenvalues are s +- q),
//   exp(K) = e^s [cosh(q) I + sinh(q)/q (K - s I)],
// so g_xx = e^s (c + S h) - 1, g_yy = e^s (c - S h) - 1, g_xy = e^s S K_xy,
// g_yx = e^s S K_yx with c = cosh q, S = sinh(q)/q as even series in q^2 and
// e^s - 1 as a series in s (no cancellation near K = 0).  The series cover
// |s| <= 1/8 and |q^2| <= 1/64 to the working precision; a larger K is
// halved j times first and the result squared back, g <- g (2 I + g).
template <typename R>
struct ExpTerms;
template <>
struct ExpTerms<float> {
    static constexpr int kS = 7, kQ = 4;
};
template <>
struct ExpTerms<double> {
    static constexpr int kS = 13, kQ = 7;
};

template <typename R>
__device__ __forceinline__ void expm1_2x2(R kxx, R kxy, R kyx, R kyy, R (&g)[4])
{
    R s = R(0.5) * (kxx + kyy), h = R(0.5) * (kxx - kyy);
    R q2 = fused(h, h, kxy * kyx);
    // halvings j with 64 max(s^2, |q^2|) 4^-j <= 1: with 64 max(..) < 2^e,
    // j = ceil(e / 2) suffices
    int j = 0;
    const R m2 = R(64) * fmax(s * s, fabs(q2));
    if (m2 > R(1)) {
        int e;
        (void)frexp(m2, &e);
        j = (e + 1) >> 1;
        const R sc = ldexp(R(1), -j);
        s *= sc;
        h *= sc;
        kxy *= sc;
        kyx *= sc;
        q2 *= sc * sc;
    }
    // c - 1 = sum_{n>=1} q^{2n}/(2n)!,  S = sum_{n>=0} q^{2n}/(2n+1)!
    R cm1 = R(0), S = R(1);
    {
        R tc = R(1), ts = R(1);
#pragma unroll
        for (int n = 1; n <= ExpTerms<R>::kQ; ++n) {
            tc = tc * q2 * R(1.0 / ((2 * n - 1) * (2 * n)));
            ts = ts * q2 * R(1.0 / ((2 * n) * (2 * n + 1)));
            cm1 += tc;
            S += ts;
        }
    }
    // e^s - 1 = s (1 + s/2 (1 + s/3 (1 + ...)))
    R em1 = R(1);
#pragma unroll
    for (int n = ExpTerms<R>::kS; n >= 2; --n)
        em1 = fused(em1, s * R(1.0 / n), R(1));
    em1 *= s;
    const R es = em1 + R(1), sh = S * h;
    // e^s (c +- S h) - 1 = em1 (c +- S h) + (c - 1) +- S h
    g[0] = fused(em1, (cm1 + R(1)) + sh, cm1 + sh);
    g[3] = fused(em1, (cm1 + R(1)) - sh, cm1 - sh);
    g[1] = es * S * kxy;
    g[2] = es * S * kyx;
    for (; j > 0; --j) {
        // (I + g)^2 - I = g (2 I + g)
        const R a = g[0], b = g[1], c = g[2], d = g[3];
        g[0] = fused(a, a, fused(b, c, R(2) * a));
        g[1] = fused(b, a + d, R(2) * b);
        g[2] = fused(c, a + d, R(2) * c);
        g[3] = fused(d, d, fused(b, c, R(2) * d));
    }
}

template <typename R>
__device__ __forceinline__ R finger_rate(R kxx, R kxy, R kyx, R kyy)
{
    const R o = kxy + kyx;
    return sqrt(R(2) * kxx * kxx + o * o + R(2) * kyy * kyy);
}

// An entry whose ages touch a window end: per-m weight and window membership.
template <typename R, int M>
__device__ __forceinline__ void finger_edge(double pxx, double pxy, double pyy, R rate, int k,
                                            int H, Acc<R> (&X)[M], Acc<R> (&Y)[M],
                                            Acc<R> (&Z)[M])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int a = k + m;
        if (a <= H - 1) {
            const R w = (a == 0 || a == H - 1) ? R(0.5) : R(1);
            const R e = w * decay_pow(R(a), rate);
            X[m].add(e * (R)pxx);
            Y[m].add(e * (R)pxy);
            Z[m].add(e * (R)pyy);
        }
    }
}

// U interior rows starting at ring slot `slot`, age kf0: advance E, add the
// terms into the FP32 partials (FIRST starts them).
template <typename R, int M, int U, bool FIRST>
__device__ __forceinline__ void finger_rows(const R *__restrict__ ring, size_t hplane, size_t np,
                                            int node, int slot, int kf0, const Decay<R> &dec,
                                            Mat2 &E, R (&px)[M], R (&py)[M], R (&pz)[M])
{
#pragma clang fp contract(off)
    R v[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t row = (size_t)(slot - u) * np + node;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[u][q] = ring[q * hplane + row];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        E = step_deformation(E, (double)v[u][4], (double)v[u][5], (double)v[u][6],
                             (double)v[u][7]);
        double pxx, pxy, pyy;
        finger_term(E, (double)v[u][0], (double)v[u][1], (double)v[u][2], (double)v[u][3], pxx,
                    pxy, pyy);
        const R rate = decay_rate<R>(dec, finger_rate<R>(v[u][0], v[u][1], v[u][2], v[u][3]));
        R x = decay_pow(R(kf0 + u), rate);
        R q = R(1);
        if (M > 1)
            q = decay_pow(R(1), rate);
        const R fx = (R)pxx, fy = (R)pxy, fz = (R)pyy;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (FIRST && u == 0) {
                px[m] = x * fx;
                py[m] = x * fy;
                pz[m] = x * fz;
            } else {
                px[m] = fused(x, fx, px[m]);
                py[m] = fused(x, fy, py[m]);
                pz[m] = fused(x, fz, pz[m]);
            }
            if (m + 1 < M)
                x *= q;
        }
    }
}

template <typename R, int M>
__device__ __forceinline__ void finger_flush(const R (&px)[M], const R (&py)[M],
                                             const R (&pz)[M], Acc<R> (&X)[M], Acc<R> (&Y)[M],
                                             Acc<R> (&Z)[M])
{
#pragma unroll
    for (int m = 0; m < M; ++m) {
        X[m].add(px[m]);
        Y[m].add(py[m]);
        Z[m].add(pz[m]);
    }
}

// Gradient of this step at a node and its push into the full-tensor ring.
template <typename P, typename R>
__device__ __forceinline__ void finger_push(char *__restrict__ ws, const ChanDev *c, int node,
                                            int slot, P &kxx, P &kxy, P &kyx, P &kyy)
{
    const size_t np = (size_t)c->np;
    const P *vel = reinterpret_cast<const P *>(ws + c->off_vel);
    const int y = node / c->lx, x = node - y * c->lx;
    velocity_gradient<P>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);
    R *ring = reinterpret_cast<R *>(ws + c->off_ring_s);
    const size_t hplane = (size_t)c->n_hist * np, row = (size_t)slot * np + node;
    double g[4];
    expm1_2x2<double>((double)kxx, (double)kxy, (double)kyx, (double)kyy, g);
    ring[0 * hplane + row] = (R)kxx;
    ring[1 * hplane + row] = (R)kxy;
    ring[2 * hplane + row] = (R)kyx;
    ring[3 * hplane + row] = (R)kyy;
    for (int q = 0; q < 4; ++q)
        ring[(4 + q) * hplane + row] = (R)g[q];
}

// One tile of a full-tensor channel: 256 nodes (one per lane), ages [k0, k1).
template <typename P, typename R, int M, int U, int F>
__device__ __forceinline__ void finger_tile(char *__restrict__ ws, const ChanDev *c,
                                            const HistTile &tl, int64_t t)
{
    static_assert(F % U == 0, "flush length must be a multiple of the row group");
    const int H = c->n_hist;
    const size_t np = (size_t)c->np, hplane = (size_t)H * np;
    const int first = tl.n0 + (int)threadIdx.x;
    const int node = first < c->n ? first : c->n - 1;  // shadow lanes past the end
    const int p = (int)(t % H);
    const R *ring = reinterpret_cast<const R *>(ws + c->off_ring_s);
    const Decay<R> dec(c);
    Acc<R> X[M], Y[M], Z[M];
    Mat2 E = {1.0, 0.0, 0.0, 1.0};
    int k = tl.k0;
    if (k == 0) {
        P kxx = P(0), kxy = P(0), kyx = P(0), kyy = P(0);
        if (first < c->n)
            finger_push<P, R>(ws, c, node, p, kxx, kxy, kyx, kyy);
        // age 0: E = I, P = kappa + kappa^T
        const R rate = decay_rate<R>(dec, finger_rate<R>((R)kxx, (R)kxy, (R)kyx, (R)kyy));
        finger_edge<R, M>(2.0 * (double)(R)kxx, (double)(R)kxy + (double)(R)kyx,
                          2.0 * (double)(R)kyy, rate, 0, H, X, Y, Z);
        k = 1;
    }
    // interior ages, then those whose k + m reaches the window end
    const int tail0 = max(k, H - M);
    const int kend = min(tl.k1, tail0);
    int slot = p - k;
    if (slot < 0)
        slot += H;
    R px[M], py[M], pz[M];
    while (k < kend) {
        const int run = min(kend - k, slot + 1);
        int j = 0;
        for (; j + F <= run; j += F) {
            finger_rows<R, M, U, true>(ring, hplane, np, node, slot - j, k + j, dec, E, px, py,
                                       pz);
            for (int gq = U; gq < F; gq += U)
                finger_rows<R, M, U, false>(ring, hplane, np, node, slot - j - gq, k + j + gq,
                                            dec, E, px, py, pz);
            finger_flush<R, M>(px, py, pz, X, Y, Z);
        }
        for (; j < run; ++j) {
            finger_rows<R, M, 1, true>(ring, hplane, np, node, slot - j, k + j, dec, E, px, py,
                                       pz);
            finger_flush<R, M>(px, py, pz, X, Y, Z);
        }
        k += run;
        slot = H - 1;
    }
    for (int kk = max(k, tail0); kk < tl.k1; ++kk) {
        int sl = p - kk;
        if (sl < 0)
            sl += H;
        const size_t row = (size_t)sl * np + node;
        R v[8];
        for (int q = 0; q < 8; ++q)
            v[q] = ring[q * hplane + row];
        E = step_deformation(E, (double)v[4], (double)v[5], (double)v[6], (double)v[7]);
        double pxx, pxy, pyy;
        finger_term(E, (double)v[0], (double)v[1], (double)v[2], (double)v[3], pxx, pxy, pyy);
        const R rate = decay_rate<R>(dec, finger_rate<R>(v[0], v[1], v[2], v[3]));
        finger_edge<R, M>(pxx, pxy, pyy, rate, kk, H, X, Y, Z);
    }
    if (first >= c->n)
        return;
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    double *part = reinterpret_cast<double *>(ws + c->off_part);
    double *blk = reinterpret_cast<double *>(ws + c->off_blk);
    if (c->nchunks == 1) {
        sig[first] = (P)(c->g_inf * Y[0].value());
        sig[np + first] = (P)(c->g_inf * X[0].value());
        sig[2 * np + first] = (P)(c->g_inf * Z[0].value());
#pragma unroll
        for (int m = 1; m < M; ++m) {
            blk[m * np + first] = X[m].value();
            blk[(kMaxBlock + m) * np + first] = Y[m].value();
            blk[(2 * kMaxBlock + m) * np + first] = Z[m].value();
        }
    } else {
        const size_t pplane = (size_t)c->max_chunks * np, at = (size_t)tl.chunk * np + first;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            part[m * pplane + at] = X[m].value();
            part[(kMaxBlock + m) * pplane + at] = Y[m].value();
            part[(2 * kMaxBlock + m) * pplane + at] = Z[m].value();
        }
        part[(3 * kMaxBlock + 0) * pplane + at] = E.a;
        part[(3 * kMaxBlock + 1) * pplane + at] = E.b;
        part[(3 * kMaxBlock + 2) * pplane + at] = E.c;
        part[(3 * kMaxBlock + 3) * pplane + at] = E.d;
    }
}

template <typename P, typename R, int M, int U, int F>
__global__ __launch_bounds__(kBlock) void k_finger_pass(char *__restrict__ ws,
                                                        const ChanDev *__restrict__ chans,
                                                        const HistTile *__restrict__ tiles,
                                                        const int64_t *__restrict__ tcount,
                                                        int trel)
{
    const HistTile tl = tiles[blockIdx.x];
    const ChanDev *c = chans + tl.ch;
    if (tl.n0 + (int)(threadIdx.x & ~63u) >= c->n)
        return;
    finger_tile<P, R, M, U, F>(ws, c, tl, *tcount + trel);
}

template <typename P, typename R, int M, int U, int F>
__global__ __launch_bounds__(kBlock) void k_finger_pass_persistent(
    char *__restrict__ ws, const ChanDev *__restrict__ chans,
    const HistTile *__restrict__ tiles, int n_tiles, const int64_t *__restrict__ tcount,
    int trel, int *__restrict__ counter)
{
    __shared__ int claimed;
    const int64_t t = *tcount + trel;
    for (;;) {
        if (threadIdx.x == 0)
            claimed = atomicAdd(counter, 1);
        __syncthreads();
        const int i = claimed;
        __syncthreads();
        if (i >= n_tiles)
            break;
        const HistTile tl = tiles[i];
        const ChanDev *c = chans + tl.ch;
        if (tl.n0 + (int)(threadIdx.x & ~63u) < c->n)
            finger_tile<P, R, M, U, F>(ws, c, tl, t);
    }
}

// In-block step m of a full-tensor channel (called from k_hist_step).
template <typename P, typename R>
__device__ __forceinline__ void finger_step(char *__restrict__ ws, const ChanDev *c, int n,
                                            int64_t t, int m)
{
    const int H = c->n_hist;
    const size_t np = (size_t)c->np, hplane = (size_t)H * np;
    const int p = (int)(t % H);
    P kxx, kxy, kyx, kyy;
    finger_push<P, R>(ws, c, n, p, kxx, kxy, kyx, kyy);
    const R *ring = reinterpret_cast<const R *>(ws + c->off_ring_s);
    const Decay<R> dec(c);
    // newest entry: age 0, weight 1/2, E = I
    double sxx = (double)(R)kxx, sxy = 0.5 * ((double)(R)kxy + (double)(R)kyx),
           syy = (double)(R)kyy;
    Mat2 E = {1.0, 0.0, 0.0, 1.0};
    int slot = p;
    for (int a = 1; a <= m; ++a) {
        slot = slot == 0 ? H - 1 : slot - 1;
        const size_t row = (size_t)slot * np + n;
        R v[8];
        for (int q = 0; q < 8; ++q)
            v[q] = ring[q * hplane + row];
        E = step_deformation(E, (double)v[4], (double)v[5], (double)v[6], (double)v[7]);
        if (a < m && a <= H - 1) {
            double pxx, pxy, pyy;
            finger_term(E, (double)v[0], (double)v[1], (double)v[2], (double)v[3], pxx, pxy,
                        pyy);
            const R rate = decay_rate<R>(dec, finger_rate<R>(v[0], v[1], v[2], v[3]));
            const double w = (a == H - 1) ? 0.5 : 1.0;
            const double e = w * (double)decay_pow(R(a), rate);
            sxx += e * pxx;
            sxy += e * pxy;
            syy += e * pyy;
        }
    }
    // E is now E(t, t0): carry the pass's sums forward
    const double *blk = reinterpret_cast<const double *>(ws + c->off_blk);
    double bxx = blk[m * np + n], bxy = blk[(kMaxBlock + m) * np + n],
           byy = blk[(2 * kMaxBlock + m) * np + n];
    congruence(E, bxx, bxy, byy);
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    sig[n] = (P)(c->g_inf * (sxy + bxy));
    sig[np + n] = (P)(c->g_inf * (sxx + bxx));
    sig[2 * np + n] = (P)(c->g_inf * (syy + byy));
}

// ---------------------------------------------------------------------------
// Accumulated-strain damping (the White-Metzner-type variant of Sec. II):
//   G(t, t') = G exp(-(t - t')/tau - R(t, t')/gamma_c),
// R(t, t') = sum of |gamma_dot| over the steps t', ..., t - 1 (the steps of
// the strain gamma).  The damping factorises over time: at step t0 + m an
// entry's factor is its factor at t0 times c_m = exp(-m/tau - dR_m/gamma_c)
// with dR_m the |gamma_dot| pushed since the pass.  So a pass at t0 needs a
// single sum over the entries that stay inside the window with weight 1 for
// the whole block (ages 1 .. H-M-1), plus per-step terms for the few ages at
// the window's ends; the step t0 + m scales the result by c_m.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R wm_damping(const Decay<R> &dec, R k, double racc)
{
    return decay_pow(R(1), fused(dec.b, (R)racc, dec.a * k));
}

template <typename P, typename R, int M>
__device__ __forceinline__ void wm_tile(char *__restrict__ ws, const ChanDev *c,
                                        const HistTile &tl, int64_t t)
{
#pragma clang fp contract(off)
    const int H = c->n_hist;
    const size_t np = (size_t)c->np;
    const int first = tl.n0 + (int)threadIdx.x;
    const int node = first < c->n ? first : c->n - 1;
    const int p = (int)(t % H);
    R *ring_s = reinterpret_cast<R *>(ws + c->off_ring_s);
    R *ring_r = reinterpret_cast<R *>(ws + c->off_ring_r);
    const bool has_r = c->has_r != 0;
    const Decay<R> dec(c);
    Acc<R> bulkA, bulkB;
    // newest entry: gradient, push, age 0
    R s0 = R(0), r0 = R(0);
    {
        const P *vel = reinterpret_cast<const P *>(ws + c->off_vel);
        if (first < c->n) {
            const int y = node / c->lx, x = node - y * c->lx;
            P kxx, kxy, kyx, kyy;
            velocity_gradient<P>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);
            s0 = (R)kxy;
            r0 = has_r ? (R)shear_rate<P>(kxx, kxy, kyx, kyy) : fabs(s0);
            ring_s[(size_t)p * np + node] = s0;
            if (has_r)
                ring_r[(size_t)p * np + node] = r0;
        }
    }
    double loc = 0.0, racc = 0.0;  // strain and accumulated |gamma_dot| since age 0
    // per-step sums of the few entries at the window's ends (at most M + 1
    // terms each: plain sums in the history precision)
    R A[M], B[M];
    auto edge = [&](R s, int k, R e, double gam) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int a = k + m;
            if (a <= H - 1) {
                const R w = (a == 0 || a == H - 1) ? R(0.5) : R(1);
                const R x = w * s * e;
                A[m] = A[m] + x;
                B[m] = B[m] + x * R(2) * (R)gam;
            }
        }
    };
    const int kb = max(1, H - M);  // ages [1, kb) stay inside with weight 1
    int slot = p;
    // bulk ages: one sum, FP32 partials of 32 rows into the compensated total; rows
    // are loaded 8 at a time before any is used (same order of operations)
    int k = 1;
    while (k < kb) {
        const int kend = min(kb, k + 32);
        R pa = R(0), pb = R(0);
        for (; k + 8 <= kend; k += 8) {
            R sv[8], rv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                slot = slot == 0 ? H - 1 : slot - 1;
                const size_t row = (size_t)slot * np + node;
                sv[u] = ring_s[row];
                rv[u] = has_r ? ring_r[row] : R(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const R s = sv[u];
                const R r = has_r ? rv[u] : fabs(s);
                loc += (double)s;
                racc += (double)r;
                const R x = s * wm_damping<R>(dec, R(k + u), racc);
                pa = pa + x;
                pb = fused(x, R(2) * (R)loc, pb);
            }
        }
        for (; k < kend; ++k) {
            slot = slot == 0 ? H - 1 : slot - 1;
            const size_t row = (size_t)slot * np + node;
            const R s = ring_s[row];
            const R r = has_r ? ring_r[row] : fabs(s);
            loc += (double)s;
            racc += (double)r;
            const R x = s * wm_damping<R>(dec, R(k), racc);
            pa = pa + x;
            pb = fused(x, R(2) * (R)loc, pb);
        }
        bulkA.add(pa);
        bulkB.add(pb);
    }
    // the newest entry (age 0, no strain, no damping), then the ages whose
    // k + m reaches the window end: per-step weights
#pragma unroll
    for (int m = 0; m < M; ++m)
        A[m] = B[m] = R(0);
    edge(s0, 0, R(1), 0.0);
    for (; k < H; ++k) {
        slot = slot == 0 ? H - 1 : slot - 1;
        const size_t row = (size_t)slot * np + node;
        const R s = ring_s[row];
        const R r = has_r ? ring_r[row] : fabs(s);
        loc += (double)s;
        racc += (double)r;
        edge(s, k, wm_damping<R>(dec, R(k), racc), loc);
    }
    if (first >= c->n)
        return;
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    double *blk = reinterpret_cast<double *>(ws + c->off_blk);
    sig[first] = (P)(c->g_inf * (bulkA.value() + (double)A[0]));
    sig[np + first] = (P)(c->g_inf * (bulkB.value() + (double)B[0]));
#pragma unroll
    for (int m = 1; m < M; ++m) {
        blk[m * np + first] = bulkA.value() + (double)A[m];
        blk[(kPlaneB + m) * np + first] = bulkB.value() + (double)B[m];
    }
}

template <typename P, typename R, int M>
__global__ __launch_bounds__(kBlock) void k_wm_pass(char *__restrict__ ws,
                                                    const ChanDev *__restrict__ chans,
                                                    const HistTile *__restrict__ tiles,
                                                    const int64_t *__restrict__ tcount, int trel)
{
    const HistTile tl = tiles[blockIdx.x];
    const ChanDev *c = chans + tl.ch;
    if (tl.n0 + (int)(threadIdx.x & ~63u) >= c->n)
        return;
    wm_tile<P, R, M>(ws, c, tl, *tcount + trel);
}

// In-block step m of an accumulated-strain channel (called from k_hist_step).
template <typename P, typename R>
__device__ __forceinline__ void wm_step(char *__restrict__ ws, const ChanDev *c, int n,
                                        int64_t t, int m)
{
    const int H = c->n_hist;
    const size_t np = (size_t)c->np;
    const int p = (int)(t % H);
    R *ring_s = reinterpret_cast<R *>(ws + c->off_ring_s);
    R *ring_r = reinterpret_cast<R *>(ws + c->off_ring_r);
    const bool has_r = c->has_r != 0;
    const P *vel = reinterpret_cast<const P *>(ws + c->off_vel);
    const int y = n / c->lx, x = n - y * c->lx;
    P kxx, kxy, kyx, kyy;
    velocity_gradient<P>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);
    const R s_new = (R)kxy;
    ring_s[(size_t)p * np + n] = s_new;
    if (has_r)
        ring_r[(size_t)p * np + n] = (R)shear_rate<P>(kxx, kxy, kyx, kyy);
    const Decay<R> dec(c);
    double sxy = 0.5 * (double)s_new, sxx = 0.0, gam = 0.0, racc = 0.0;
    int slot = p;
    // the m rows pushed since the pass, newest first, loaded 8 at a time
    // before any is used (same order of operations)
    for (int a0 = 1; a0 <= m; a0 += 8) {
        R sv[8], rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sv[u] = rv[u] = R(0);
            if (a0 + u <= m) {
                slot = slot == 0 ? H - 1 : slot - 1;
                sv[u] = ring_s[(size_t)slot * np + n];
                if (has_r)
                    rv[u] = ring_r[(size_t)slot * np + n];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int a = a0 + u;
            if (a > m)
                break;
            const R s = sv[u];
            const R r = has_r ? rv[u] : fabs(s);
            gam += (double)s;
            racc += (double)r;
            if (a < m && a <= H - 1) {
                const double w = (a == H - 1) ? 0.5 : 1.0;
                const double se = w * (double)(s * wm_damping<R>(dec, R(a), racc));
                sxy += se;
                sxx += 2.0 * gam * se;
            }
        }
    }
    // the pass's sums carried to this step: factor c_m
    const double cm = (double)wm_damping<R>(dec, R(m), racc);
    const double *blk = reinterpret_cast<const double *>(ws + c->off_blk);
    const double A = blk[m * np + n], B = blk[(kPlaneB + m) * np + n];
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    sig[n] = (P)(c->g_inf * (sxy + cm * A));
    sig[np + n] = (P)(c->g_inf * (sxx + cm * (B + 2.0 * gam * A)));
}

// Instantaneous law (Eq. inlM read at time t): sigma_xy = G tau_M s,
// sigma_xx = 2 G tau_M^2 s^2, tau_M = 1/(1/tau + |gamma_dot|/gamma_c).
template <typename P>
__global__ __launch_bounds__(kBlock) void k_inst_step(char *__restrict__ ws,
                                                      const ChanDev *__restrict__ chans,
                                                      const NodeTile *__restrict__ tiles)
{
    const NodeTile tl = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    if (c->law != 2 || n >= c->n)
        return;
    const size_t np = (size_t)c->np;
    const P *vel = reinterpret_cast<const P *>(ws + c->off_vel);
    const int y = n / c->lx, x = n - y * c->lx;
    P kxx, kxy, kyx, kyy;
    velocity_gradient<P>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);
    const double r = (double)shear_rate<P>(kxx, kxy, kyx, kyy);
    const double taum = 1.0 / (c->inv_tau + c->inv_gc * r);
    const double s = (double)kxy;
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    sig[n] = (P)(c->g_inf * taum * s);
    sig[np + n] = (P)(2.0 * c->g_inf * taum * taum * s * s);
}

// ---------------------------------------------------------------------------
// FP64 combine of the per-chunk partials of a split window, newest chunk
// first: A_m = sum_c A_{m,c}, B_m = sum_c (2 O_c A_{m,c} + B_{m,c}), where
// O_c = sum of the strain totals T of the newer chunks (the accumulated
// strain at the chunk's start).  One thread per node and step m of the block
// (grid: node tiles x block); m = 0 writes sigma of the pass step, m > 0 the
// block sums for the following steps.
// ---------------------------------------------------------------------------
template <typename P>
__global__ __launch_bounds__(kBlock) void k_combine(char *__restrict__ ws,
                                                    const ChanDev *__restrict__ chans,
                                                    const NodeTile *__restrict__ tiles)
{
    const NodeTile tl = tiles[blockIdx.x];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    const int m = blockIdx.y;
    if (c->nchunks == 1 || n >= c->n)
        return;
    const size_t np = (size_t)c->np;
    const size_t pplane = (size_t)c->max_chunks * np;
    const double *part = reinterpret_cast<const double *>(ws + c->off_part);
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    double *blk = reinterpret_cast<double *>(ws + c->off_blk);
    if (c->finger) {
        // sum_c O_c S_c O_c^T, O_0 = I, O_{c+1} = O_c T_c
        double X = 0.0, Y = 0.0, Z = 0.0;
        Mat2 O = {1.0, 0.0, 0.0, 1.0};
        for (int k = 0; k < c->nchunks; ++k) {
            const size_t at = (size_t)k * np + n;
            double sx = part[m * pplane + at], sy = part[(kMaxBlock + m) * pplane + at],
                   sz = part[(2 * kMaxBlock + m) * pplane + at];
            congruence(O, sx, sy, sz);
            X += sx;
            Y += sy;
            Z += sz;
            const Mat2 T = {part[(3 * kMaxBlock + 0) * pplane + at],
                            part[(3 * kMaxBlock + 1) * pplane + at],
                            part[(3 * kMaxBlock + 2) * pplane + at],
                            part[(3 * kMaxBlock + 3) * pplane + at]};
            O = mat_mul(O, T);
        }
        if (m == 0) {
            sig[n] = (P)(c->g_inf * Y);
            sig[np + n] = (P)(c->g_inf * X);
            sig[2 * np + n] = (P)(c->g_inf * Z);
        } else {
            blk[m * np + n] = X;
            blk[(kMaxBlock + m) * np + n] = Y;
            blk[(2 * kMaxBlock + m) * np + n] = Z;
        }
        return;
    }
    double A = 0.0, B = 0.0, O = 0.0;
    for (int k = 0; k < c->nchunks; ++k) {
        const size_t at = (size_t)k * np + n;
        const double a = part[m * pplane + at];
        A += a;
        B += 2.0 * O * a + part[(kPlaneB + m) * pplane + at];
        O += part[kPlaneT * pplane + at];
    }
    if (m == 0) {
        sig[n] = (P)(c->g_inf * A);
        sig[np + n] = (P)(c->g_inf * B);
    } else {
        blk[m * np + n] = A;
        blk[(kPlaneB + m) * np + n] = B;
    }
}

// ---------------------------------------------------------------------------
// Step t = t0 + m of a block (1 <= m < M): gradient and push of entry t, then
// sigma from the block sums plus the entries t0+1 .. t pushed since the pass.
// Walking ages a = 0..m from the new entry back to entry t0 accumulates the
// strain gamma(t, t - a); at a = m it is Delta_m.
// ---------------------------------------------------------------------------
template <typename P, typename R>
__device__ __forceinline__ void hist_step_node(char *__restrict__ ws, const ChanDev *c, int n,
                                               int64_t t, int m)
{
    if (c->finger) {
        finger_step<P, R>(ws, c, n, t, m);
        return;
    }
    if (c->law == 1) {
        wm_step<P, R>(ws, c, n, t, m);
        return;
    }
    if (c->law == 2)
        return;  // instantaneous channels step in k_inst_step
    const int H = c->n_hist;
    const size_t np = (size_t)c->np;
    const int p = (int)(t % H);
    R *ring_s = reinterpret_cast<R *>(ws + c->off_ring_s);
    R *ring_r = reinterpret_cast<R *>(ws + c->off_ring_r);
    const P *vel = reinterpret_cast<const P *>(ws + c->off_vel);
    const int y = n / c->lx, x = n - y * c->lx;
    P kxx, kxy, kyx, kyy;
    velocity_gradient<P>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);
    const R s_new = (R)kxy;
    ring_s[(size_t)p * np + n] = s_new;
    if (c->has_r)
        ring_r[(size_t)p * np + n] = (R)shear_rate<P>(kxx, kxy, kyx, kyy);

    const double *blk = reinterpret_cast<const double *>(ws + c->off_blk);
    const double A = blk[m * np + n];
    const double B = blk[(kPlaneB + m) * np + n];
    // newest entry: age 0, weight 1/2, E = 1, gamma = 0
    // The decay of these few entries is taken in the history precision, as
    // in the pass.
    const Decay<R> dec(c);
    double sxy = 0.5 * (double)s_new, sxx = 0.0, gam = 0.0;
    // entries at ages 1..m (the one at age m only adds its strain), read
    // kLoads rows ahead of their use
    constexpr int kLoads = 8;
    int slot = p;
    for (int a0 = 1; a0 <= m; a0 += kLoads) {
        R sv[kLoads], rv[kLoads];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int a = a0 + u;
            if (a <= m) {
                slot = slot == 0 ? H - 1 : slot - 1;
                const size_t o = (size_t)slot * np + n;
                sv[u] = ring_s[o];
                rv[u] = (c->has_r && a < m) ? ring_r[o] : fabs(sv[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int a = a0 + u;
            if (a <= m) {
                const R s = sv[u];
                gam += (double)s;
                if (a < m && a <= H - 1) {
                    const double w = (a == H - 1) ? 0.5 : 1.0;
                    const double se =
                        w * (double)(s * decay_pow(R(a), decay_rate<R>(dec, rv[u])));
                    sxy += se;
                    sxx += 2.0 * gam * se;
                }
            }
        }
    }
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    sig[n] = (P)(c->g_inf * (A + sxy));
    sig[np + n] = (P)(c->g_inf * (B + 2.0 * gam * A + sxx));
}

template <typename P, typename R>
__global__ __launch_bounds__(kBlock) void k_hist_step(char *__restrict__ ws,
                                                      const ChanDev *__restrict__ chans,
                                                      const NodeTile *__restrict__ tiles,
                                                      const int64_t *__restrict__ tcount,
                                                      int trel, int m)
{
    const NodeTile tl = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    if (c->qb != 0 || n >= c->n)
        return;  // grid channels step in k_grid_step
    hist_step_node<P, R>(ws, c, n, *tcount + trel, m);
}

// Steps m0 .. m0 + count - 1 of a block (all after its pass) for handles whose
// channels each fit one workgroup: workgroup b runs channel b's lattice phase
// and in-block history phase for every step, with a workgroup barrier where
// the unfused path has a kernel boundary (every node a stencil of the channel
// reads belongs to the workgroup).  Same per-node arithmetic as k_lb and
// k_hist_step, so results are identical.
template <typename P, typename R, typename S>
__global__ __launch_bounds__(kFuseThreads) void k_fused_steps(char *__restrict__ ws,
                                                            const ChanDev *__restrict__ chans,
                                                            const int64_t *__restrict__ tcount,
                                                            int trel, int m0, int count)
{
    const ChanDev *c = chans + blockIdx.x;
    const int64_t t0 = *tcount + trel;
    for (int k = 0; k < count; ++k) {
        const int64_t t = t0 + k;
        for (int n = threadIdx.x; n < c->n; n += kFuseThreads)
            lb_node<P, S>(ws, c, n, t);
        __syncthreads();
        for (int n = threadIdx.x; n < c->n; n += kFuseThreads)
            hist_step_node<P, R>(ws, c, n, t, m0 + k);
        __syncthreads();
    }
}

// Steps m0 .. m0 + count - 1 of a block with the channel's lattice state in
// the workgroup, for handles in split population storage whose channels all
// take the simple-shear integral law with the body-force coupling on a
// uniform window (and fit one workgroup).  LDS holds the post-collision
// remainders, the moments (rho - 1, u) and the stress of the channel, so the
// neighbours a stencil reads come from LDS; each thread keeps the history rows
// of its node pushed since the pass in registers.  Every result still goes to
// the workspace (remainders and moments of both parities, velocity, rho,
// stress, ring rows) as the separate launches write it, and the arithmetic is
// the same operations in the same order, so the results are identical.
//
// In-block history of one node at step t0 + m from the rows in registers
// (entry j pushed at t0 + j, s_new this step's): the ring walk of
// hist_step_node, ages a = 1..m in the same order.
template <typename R, bool HAS_R>
__device__ __forceinline__ void hist_regs(const ChanDev *c, const Decay<R> &dec, int m, R s_new,
                                          const R (&hs)[kMaxBlock], const R (&hr)[kMaxBlock],
                                          double &sxy_out, double &sxx_out, double &gam_out)
{
    const int H = c->n_hist;
    double sxy = 0.5 * (double)s_new, sxx = 0.0, gam = 0.0;
#pragma unroll
    for (int j = kMaxBlock - 1; j >= 0; --j) {
        if (j < m) {
            const int a = m - j;
            const R s = hs[j];
            gam += (double)s;
            if (a < m && a <= H - 1) {
                const double w = (a == H - 1) ? 0.5 : 1.0;
                const R r = HAS_R ? hr[j] : fabs(s);
                const double se = w * (double)(s * decay_pow(R(a), decay_rate<R>(dec, r)));
                sxy += se;
                sxx += 2.0 * gam * se;
            }
        }
    }
    sxy_out = sxy;
    sxx_out = sxx;
    gam_out = gam;
}

// Remainders r_q = (float)(out_q - n^eq_q) of a collision, as
// split_remainders forms them, and the populations a pull rebuilds from them,
// n^eq_q + r_q (the same operations as pull_split_one, so bit for bit what a
// neighbour pulling from split storage obtains).
template <typename P>
__device__ __forceinline__ void split_and_rebuild(const P (&out)[9], P ux, P uy, P drho,
                                                  float (&r)[9], P (&full)[9])
{
#pragma clang fp contract(off)
    const P uu = ux * ux + uy * uy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const P cu = P(QX[q]) * ux + P(QY[q]) * uy;
        const P e = eq_dev<P>(qweight<P>(q), cu, drho, uu);
        r[q] = (float)(out[q] - e);
        full[q] = e + (P)r[q];
    }
}

// LDS of the span: the channel's pulled-from populations as FP64 deviations
// rebuilt from split storage ([9][K]), its velocity ([2][K]) and stress
// ([2][K]); pulls read them without arithmetic.
template <typename P, typename R, bool HAS_R>
__device__ __forceinline__ void fused_span_lds(char *__restrict__ ws, const ChanDev *c,
                                               int64_t t0s, int m0, int count, P *s_full,
                                               P *s_vel, P *s_sig)
{
    constexpr int K = kFuseThreads;  // LDS plane stride
    const int n = threadIdx.x;
    const bool own = n < c->n;
    const size_t np = (size_t)c->np;
    const int H = c->n_hist;
    const int64_t tb = t0s - m0;  // step of the block's pass
    float *pop = reinterpret_cast<float *>(ws + c->off_pop);
    P *mom = reinterpret_cast<P *>(ws + c->off_mom);
    P *vel = reinterpret_cast<P *>(ws + c->off_vel);
    P *rhop = reinterpret_cast<P *>(ws + c->off_rho);
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    R *ring_s = reinterpret_cast<R *>(ws + c->off_ring_s);
    R *ring_r = reinterpret_cast<R *>(ws + c->off_ring_r);
    const double *blk = reinterpret_cast<const double *>(ws + c->off_blk);
    const Decay<R> dec(c);
    // state of step t0s - 1, and the rows pushed since the pass
    R hs[kMaxBlock], hr[kMaxBlock];
    if (own) {
        const float *src = pop + ((t0s + 1) & 1) * 9 * np;
        const P *msrc = mom + ((t0s + 1) & 1) * 3 * np;
        P full[9];
        own_split<P>(n, src, msrc, np, full);
#pragma unroll
        for (int q = 0; q < 9; ++q)
            s_full[q * K + n] = full[q];
        s_sig[n] = sig[n];
        s_sig[K + n] = sig[np + n];
#pragma unroll
        for (int j = 0; j < kMaxBlock; ++j) {
            hs[j] = hr[j] = R(0);
            if (j < m0) {
                const size_t o = (size_t)((tb + j) % H) * np + n;
                hs[j] = ring_s[o];
                if (HAS_R)
                    hr[j] = ring_r[o];
            }
        }
    }
    __syncthreads();
    for (int k = 0; k < count; ++k) {
        const int64_t t = t0s + k;
        const int m = m0 + k;
        double A = 0.0, B = 0.0;
        P full[9];
        P ux = P(0), uy = P(0);
        if (own) {
            A = blk[m * np + n];  // issued before the lattice phase
            B = blk[(kPlaneB + m) * np + n];
            if (c->rec) {
                P *rec = reinterpret_cast<P *>(c->rec) + (size_t)(t - c->rec_t0) * 10 * np;
#pragma unroll
                for (int q = 0; q < 9; ++q)
                    rec[q * np + n] = s_full[q * K + n];
                rec[9 * np + n] = s_sig[n];
            }
            P d[9], out[9], drho;
            lb_pull<P>(c, n, s_full, K, d);
            lb_collide_body<P>(c, n, d, s_sig, K, out, ux, uy, drho);
            float r[9];
            split_and_rebuild<P>(out, ux, uy, drho, r, full);
            // The workspace state of the span's last step (nothing here is read
            // in the span, and the next step reads only the last one); every
            // step's while the lattice inputs are being recorded.
            if (k == count - 1 || c->rec) {
                float *dst = pop + (t & 1) * 9 * np;
                P *mdst = mom + (t & 1) * 3 * np;
#pragma unroll
                for (int q = 0; q < 9; ++q)
                    dst[q * np + n] = r[q];
                mdst[n] = drho;
                mdst[np + n] = ux;
                mdst[2 * np + n] = uy;
                vel[n] = ux;
                vel[np + n] = uy;
                rhop[n] = drho;
            }
        }
        __syncthreads();  // every stencil read of the old state and stress is done
        if (own) {
#pragma unroll
            for (int q = 0; q < 9; ++q)
                s_full[q * K + n] = full[q];
            s_vel[n] = ux;
            s_vel[K + n] = uy;
        }
        __syncthreads();  // this step's velocities are in LDS
        if (own) {
            const int y = n / c->lx, x = n - y * c->lx;
            P kxx, kxy, kyx, kyy;
            velocity_gradient<P>(s_vel, s_vel + K, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);
            const R s_new = (R)kxy;
            const size_t o = (size_t)(t % H) * np + n;
            ring_s[o] = s_new;
            R r_new = R(0);
            if (HAS_R) {
                r_new = (R)shear_rate<P>(kxx, kxy, kyx, kyy);
                ring_r[o] = r_new;
            }
            double sxy, sxx, gam;
            hist_regs<R, HAS_R>(c, dec, m, s_new, hs, hr, sxy, sxx, gam);
#pragma unroll
            for (int j = 0; j < kMaxBlock; ++j)
                if (j == m) {
                    hs[j] = s_new;
                    if (HAS_R)
                        hr[j] = r_new;
                }
            const P sxy_p = (P)(c->g_inf * (A + sxy));
            const P sxx_p = (P)(c->g_inf * (B + 2.0 * gam * A + sxx));
            if (k == count - 1 || c->rec) {
                sig[n] = sxy_p;
                sig[np + n] = sxx_p;
            }
            s_sig[n] = sxy_p;
            s_sig[K + n] = sxx_p;
        }
        __syncthreads();  // this step's stress is in LDS
    }
}

template <typename P, typename R>
__global__ __launch_bounds__(kFuseThreads) void k_fused_steps_lds(
    char *__restrict__ ws, const ChanDev *__restrict__ chans, const int64_t *__restrict__ tcount,
    int trel, int m0, int count)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    P *s_full = reinterpret_cast<P *>(lds_raw);  // [9][kFuseThreads]
    P *s_vel = s_full + 9 * kFuseThreads;        // [2][kFuseThreads]
    P *s_sig = s_vel + 2 * kFuseThreads;         // [2][kFuseThreads]
    const ChanDev *c = chans + blockIdx.x;
    const int64_t t0s = *tcount + trel;
    // unidirectional channels only (|gamma_dot| = |s|: one row per entry in
    // registers); the host selects this form only then
    fused_span_lds<P, R, false>(ws, c, t0s, m0, count, s_full, s_vel, s_sig);
}

// ---------------------------------------------------------------------------
// Quasi-logarithmic history grid (Sec. III), one node per thread, every step.
//
// Block b = 1..B (index bi = b - 1, 0 the oldest) has the step 2^(B-b).  Its
// i-th entry (i counts the C zero entries it starts with) lives in row
// bi*C + (i mod C) and starts at t0 = 2^(B-b) i - (2^(B-b+1) - 1) C.  With
// the C zero entries present before t = 0, block b has received
// floor(t / 2^(B-b)) + 1 entries after step t (one per step for block B,
// one per combination of block b + 1 otherwise) and combined
// floor(t / 2^(B-b+1)) + 1 pairs, so at step t it combines its pair j = t /
// 2^(B-b+1) -- entries 2j, 2j+1 -- exactly when 2^(B-b+1) divides t, into
// entry C + j of block b - 1.  Blocks are combined oldest first, each before
// it receives, so a block never holds more than C entries.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R rate_of_d(R dxx, R dxy, R dyy)
{
    // sqrt(II_D), II_D = tr(D^2) / 2 for D = kappa + kappa^T (Sec. II)
    return sqrt(R(0.5) * (dxx * dxx + R(2) * dxy * dxy + dyy * dyy));
}

// Entry bookkeeping of block bi (lg = B - 1 - bi, step 2^lg): the newest
// and oldest entry it holds after the combinations and the push of step t,
// and the age at step t of its i-th entry.
__device__ __forceinline__ int64_t grid_newest(int64_t t, int lg, int C)
{
    return C + (t >> lg);
}
__device__ __forceinline__ int64_t grid_oldest(int64_t t, int lg)
{
    return 2 * ((t >> (lg + 1)) + 1);
}
__device__ __forceinline__ int64_t grid_age(int64_t t, int64_t i, int lg, int C)
{
    const int64_t step = int64_t(1) << lg;
    return t - (step * i - (2 * step - 1) * (int64_t)C);
}

// The combinations due at step t, oldest block first, then the push of step
// t's entry (node n; the velocity of step t is in place).
template <typename P, typename R>
__device__ __forceinline__ void grid_update(char *__restrict__ ws, const ChanDev *c, int n,
                                            int64_t t)
{
    const int B = c->qb, C = c->qc;
    const size_t np = (size_t)c->np;
    const size_t dplane = (size_t)B * C * np;
    const bool has_r = c->has_r != 0;
    R *gs = reinterpret_cast<R *>(ws + c->off_grid_s);
    R *gr = reinterpret_cast<R *>(ws + c->off_grid_r);
    R *gd = reinterpret_cast<R *>(ws + c->off_grid_d);
    auto row = [&](int bi, int slot) { return ((size_t)bi * C + slot) * np + n; };

    const P *vel = reinterpret_cast<const P *>(ws + c->off_vel);
    const int y = n / c->lx, x = n - y * c->lx;
    P kxx, kxy, kyx, kyy;
    velocity_gradient<P>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);

    for (int bi = 0; bi < B; ++bi) {
        const int sh = B - bi;  // log2 of the block's combination period
        if ((t & ((int64_t(1) << sh) - 1)) != 0)
            continue;
        const int64_t j = t >> sh;
        const int s0 = (int)((2 * j) % C), s1 = s0 + 1 == C ? 0 : s0 + 1;
        const size_t o0 = row(bi, s0), o1 = row(bi, s1);
        const R ms = R(0.5) * (gs[o0] + gs[o1]);
        R md[3] = {R(0), R(0), R(0)}, mr = R(0);
        if (has_r) {
            for (int q = 0; q < 3; ++q)
                md[q] = R(0.5) * (gd[q * dplane + o0] + gd[q * dplane + o1]);
            mr = rate_of_d<R>(md[0], md[1], md[2]);
        }
        if (bi > 0) {
            const size_t d = row(bi - 1, (int)(j % C));
            gs[d] = ms;
            if (has_r) {
                gr[d] = mr;
                for (int q = 0; q < 3; ++q)
                    gd[q * dplane + d] = md[q];
            }
        }
    }
    const size_t d = row(B - 1, (int)(t % C));
    gs[d] = (R)kxy;
    if (has_r) {
        const R dd[3] = {(R)(P(2) * kxx), (R)(kxy + kyx), (R)(P(2) * kyy)};
        for (int q = 0; q < 3; ++q)
            gd[q * dplane + d] = dd[q];
        gr[d] = (R)shear_rate<P>(kxx, kxy, kyx, kyy);
    }
}

// Running state of Eq. gitt on the grid, entries visited newest first:
// trapezoid weights from the neighbours' ages, strain gamma = sum of (mean
// s) x (step) over the entries from the newest-but-one down to the current.
// Ages fit in 32 bits: the grid spans fewer than (C + 2) 2^B <= 2^30 + 2^21
// steps.
struct GridSums {
    double sxy = 0.0, sxx = 0.0, gam = 0.0;
    int a_prev = 0;
    bool first = true;
};

// Visit an entry of block bi (time step `step`) of age `age` at the current
// step, with shear rate sv and |gamma_dot| rv; `has_next`: the block holds an
// older entry.  Returns its decay rate and E(age) in the history precision.
// Without `direct` the entry's trapezoid terms are left to the caller.
template <typename R>
__device__ __forceinline__ void grid_visit(R sv, R rv, int bi, int step, int age, bool has_next,
                                           const Decay<R> &dec, GridSums &g, R &rate, R &e,
                                           bool direct = true)
{
    // the older neighbour: the next entry of the block, or the newest of
    // block bi - 1 (2 steps back), or none for the oldest entry of all
    const int a_next = has_next ? age + step : (bi > 0 ? age + 2 * step : age);
    if (!g.first)
        g.gam += (double)sv * (double)step;
    rate = decay_rate<R>(dec, rv);
    e = decay_pow((R)age, rate);
    if (direct) {
        const double xw = 0.5 * (double)(a_next - g.a_prev) * (double)(sv * e);
        g.sxy += xw;
        g.sxx += 2.0 * g.gam * xw;
    }
    g.a_prev = age;
    g.first = false;
}

// Visit entries hi, hi - 1, ..., lo of block bi (newest first), loading L
// entries ahead of their use; fn(i, sv, rate, e) after each visit.  Entries
// sk_lo..sk_hi are visited without their trapezoid terms.  The row of entry
// i is bi C + (i mod C): the slot and the age (which grows by the block's
// step from one entry to the next older one) are carried along the range,
// so that no entry needs a 64-bit division.
template <typename R, int L, typename Fn>
__device__ __forceinline__ void grid_range(const R *__restrict__ gs, const R *__restrict__ gr,
                                           bool has_r, const ChanDev *c, int n, int bi, int lg,
                                           int64_t hi, int64_t lo, int64_t i_old, int64_t t,
                                           const Decay<R> &dec, GridSums &g, Fn &&fn,
                                           int64_t sk_lo = 1, int64_t sk_hi = 0)
{
    if (hi < lo)
        return;
    const int C = c->qc;
    const size_t np = (size_t)c->np;
    const int step = 1 << lg;
    const int count = (int)(hi - lo + 1);
    const R *bs = gs + (size_t)bi * C * np;
    const R *br = gr + (size_t)bi * C * np;
    int slot = (int)(hi % C);
    int age = (int)grid_age(t, hi, lg, C);
    for (int k = 0; k < count; k += L) {
        R sv[L], rv[L];
#pragma unroll
        for (int u = 0; u < L; ++u) {
            if (k + u < count) {
                const size_t o = (size_t)slot * np + n;
                sv[u] = bs[o];
                rv[u] = has_r ? br[o] : fabs(sv[u]);
            }
            slot = slot == 0 ? C - 1 : slot - 1;
        }
#pragma unroll
        for (int u = 0; u < L; ++u)
            if (k + u < count) {
                const int64_t i = hi - (k + u);
                R rate, e;
                grid_visit<R>(sv[u], rv[u], bi, step, age + u * step, i > i_old, dec, g, rate, e,
                              i < sk_lo || i > sk_hi);
                fn(i, sv[u], rate, e);
            }
        age += L * step;
    }
}

// Temporal blocking on the grid.  The grid takes blocks of M = min(steps per
// pass, kMaxGridBlock) steps: per step it reads 1/M of its entries in the
// pass, plus the entries outside the interior (below), whose count grows
// with M.  For a block of steps t0..t1 = t0 + M - 1, entry i of block bi
// with grid_oldest(t1) < i < grid_newest(t0) is held at every step of the
// block with the same neighbours, so its trapezoid weight
// stays `step`, its decay is E(age(t0)) q^m at step t0 + m, and its strain
// grows by the same Delta_m (the strain of the entries pushed since t0) as
// every older entry: combinations only regroup the strain of newer entries.
// These interior entries enter the block sums A_m, B_m of the pass at t0
// exactly as the window entries do; the other entries (the newest ones,
// received since t0 and the one newest at t0, and the oldest ones, combined
// away during the block and the oldest kept) are visited every step.  The two
// sets are disjoint when C >= M + 2.
__host__ __device__ constexpr bool grid_blockable(int C, int M) { return M > 1 && C >= M + 2; }

// The full walk at step t.  With M > 1 it also forms, for m = 1..M-1, the
// block sums of the interior entries of the block t..t+M-1 (blk planes m and
// kPlaneB + m) and, per grid block, their strain (plane kPlaneGrid + bi).
template <typename P, typename R, int M>
__device__ __forceinline__ void grid_walk(char *__restrict__ ws, const ChanDev *c, int n,
                                          int64_t t)
{
#pragma clang fp contract(off)
    constexpr int F = 64;  // FP32 partial sums enter the totals every F entries
    const int B = c->qb, C = c->qc;
    const size_t np = (size_t)c->np;
    const bool has_r = c->has_r != 0;
    const R *gs = reinterpret_cast<const R *>(ws + c->off_grid_s);
    const R *gr = reinterpret_cast<const R *>(ws + c->off_grid_r);
    double *blk = reinterpret_cast<double *>(ws + c->off_blk);
    const Decay<R> dec(c);
    GridSums g;
    R pa[M][1], pb[M][1];
    Acc<R> A[M][1], Bs[M][1];
    int cnt = 0;
    const int64_t t1 = t + M - 1;
    for (int bi = B - 1; bi >= 0; --bi) {
        const int lg = B - 1 - bi;
        const int64_t step = int64_t(1) << lg;
        const int64_t i_new = grid_newest(t, lg, C), i_old = grid_oldest(t, lg);
        const int64_t in_hi = i_new - 1, in_lo = grid_oldest(t1, lg) + 1;
        double strain = 0.0;
        constexpr int L = M == 1 ? 4 : 8;  // entries loaded ahead
        grid_range<R, L>(gs, gr, has_r, c, n, bi, lg, i_new, i_old, i_old, t, dec, g,
                      [&](int64_t i, R sv, R rate, R e) {
                          if (M > 1 && i >= in_lo && i <= in_hi) {
                              strain += (double)sv * (double)step;
                              const R x = (R)step * (sv * e);
                              const R q = decay_pow(R(1), rate);
                              const R g2 = R(2) * (R)g.gam;
                              if (cnt == 0)
                                  add_powers<R, M, 1, true>(x, q, g2, pa, pb, 0);
                              else
                                  add_powers<R, M, 1, false>(x, q, g2, pa, pb, 0);
                              if (++cnt == F) {
                                  flush<R, 1, M>(pa, pb, A, Bs);
                                  cnt = 0;
                              }
                          }
                      },
                      in_lo, M > 1 ? in_hi : in_lo - 1);
        if (M > 1)
            blk[(kPlaneGrid + bi) * np + n] = strain;
    }
    // the interior's terms of step t are its m = 0 block sums
    double a0 = 0.0, b0 = 0.0;
    if (M > 1) {
        if (cnt > 0)
            flush<R, 1, M>(pa, pb, A, Bs);
        a0 = A[0][0].value();
        b0 = Bs[0][0].value();
    }
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    sig[n] = (P)(c->g_inf * (g.sxy + a0));
    sig[np + n] = (P)(c->g_inf * (g.sxx + b0));
    if (M > 1) {
#pragma unroll
        for (int m = 1; m < M; ++m) {
            blk[m * np + n] = A[m][0].value();
            blk[(kPlaneB + m) * np + n] = Bs[m][0].value();
        }
    }
}

// Step t0 + m (0 < m < M) of a block: the entries outside the interior
// directly, the interior through the pass's sums and strains.
template <typename P, typename R>
__device__ __forceinline__ void grid_edges(char *__restrict__ ws, const ChanDev *c, int n,
                                           int64_t t, int m, int M)
{
    const int B = c->qb, C = c->qc;
    const size_t np = (size_t)c->np;
    const bool has_r = c->has_r != 0;
    const R *gs = reinterpret_cast<const R *>(ws + c->off_grid_s);
    const R *gr = reinterpret_cast<const R *>(ws + c->off_grid_r);
    const double *blk = reinterpret_cast<const double *>(ws + c->off_blk);
    const Decay<R> dec(c);
    const int64_t t0 = t - m, t1 = t0 + M - 1;
    GridSums g;
    double delta = 0.0;
    auto none = [](int64_t, R, R, R) {};
    for (int bi = B - 1; bi >= 0; --bi) {
        const int lg = B - 1 - bi;
        const int64_t i_new = grid_newest(t, lg, C), i_new0 = grid_newest(t0, lg, C);
        const int64_t i_old = grid_oldest(t, lg), i_old1 = grid_oldest(t1, lg);
        grid_range<R, 4>(gs, gr, has_r, c, n, bi, lg, i_new, i_new0, i_old, t, dec, g, none);
        if (bi == B - 1)
            delta = g.gam;  // entries C + t0 .. C + t - 1: the shear rates of steps t0..t-1
        if (i_old1 + 1 <= i_new0 - 1) {
            g.gam += blk[(kPlaneGrid + bi) * np + n];
            g.a_prev = (int)grid_age(t, i_old1 + 1, lg, C);
        }
        grid_range<R, 4>(gs, gr, has_r, c, n, bi, lg, i_old1, i_old, i_old, t, dec, g, none);
    }
    const double A = blk[m * np + n], Bm = blk[(kPlaneB + m) * np + n];
    P *sig = reinterpret_cast<P *>(ws + c->off_sig);
    sig[n] = (P)(c->g_inf * (A + g.sxy));
    sig[np + n] = (P)(c->g_inf * (Bm + 2.0 * delta * A + g.sxx));
}

// Unblocked grid step (M = 1): update and full walk every step.
template <typename P, typename R>
__global__ __launch_bounds__(kBlock) void k_grid_step(char *__restrict__ ws,
                                                      const ChanDev *__restrict__ chans,
                                                      const NodeTile *__restrict__ tiles,
                                                      const int64_t *__restrict__ tcount,
                                                      int trel)
{
    const NodeTile tl = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    if (c->qb == 0 || n >= c->n)
        return;
    const int64_t t = *tcount + trel;
    grid_update<P, R>(ws, c, n, t);
    grid_walk<P, R, 1>(ws, c, n, t);
}

// First step of a block of M: update, full walk and the interior sums.
// Channels too short for blocking (C < M + 2) take the full walk only.
template <typename P, typename R, int M>
__global__ __launch_bounds__(kBlock) void k_grid_pass(char *__restrict__ ws,
                                                      const ChanDev *__restrict__ chans,
                                                      const NodeTile *__restrict__ tiles,
                                                      const int64_t *__restrict__ tcount,
                                                      int trel)
{
    const NodeTile tl = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    if (c->qb == 0 || n >= c->n)
        return;
    const int64_t t = *tcount + trel;
    grid_update<P, R>(ws, c, n, t);
    if (grid_blockable(c->qc, M))
        grid_walk<P, R, M>(ws, c, n, t);
    else
        grid_walk<P, R, 1>(ws, c, n, t);
}

// Step m (0 < m < M) of a block: update and the edge walk.
template <typename P, typename R>
__global__ __launch_bounds__(kBlock) void k_grid_edges(char *__restrict__ ws,
                                                       const ChanDev *__restrict__ chans,
                                                       const NodeTile *__restrict__ tiles,
                                                       const int64_t *__restrict__ tcount,
                                                       int trel, int m, int M)
{
    const NodeTile tl = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    if (c->qb == 0 || n >= c->n)
        return;
    const int64_t t = *tcount + trel;
    grid_update<P, R>(ws, c, n, t);
    if (grid_blockable(c->qc, M))
        grid_edges<P, R>(ws, c, n, t, m, M);
    else
        grid_walk<P, R, 1>(ws, c, n, t);
}

__global__ void k_tick(int64_t *tcount, int64_t add)
{
    if (threadIdx.x == 0)
        tcount[0] += add;
}

__global__ void k_set_force(ChanDev *chans, int ch, double gx, double gy)
{
    if (threadIdx.x == 0) {
        chans[ch].gx = gx;
        chans[ch].gy = gy;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_readout(int which, const char *__restrict__ ws,
                                                    const ChanDev *__restrict__ chans,
                                                    int ch, double *__restrict__ out)
{
    const ChanDev *c = chans + ch;
    const int n = blockIdx.x * kBlock + threadIdx.x;
    const int N = c->n;
    if (n >= N)
        return;
    const size_t np = (size_t)c->np;
    if (which == 0) {
        const R *rho = reinterpret_cast<const R *>(ws + c->off_rho);
        const R *vel = reinterpret_cast<const R *>(ws + c->off_vel);
        out[n] = 1.0 + (double)rho[n];
        out[N + n] = (double)vel[n];
        out[2 * N + n] = (double)vel[np + n];
    } else if (which == 1) {
        const R *sig = reinterpret_cast<const R *>(ws + c->off_sig);
        out[n] = (double)sig[n];
        // N1 = sigma_xx - sigma_yy (sigma_yy = 0 in the simple-shear reduction)
        out[N + n] = (double)sig[np + n] - (c->finger ? (double)sig[2 * np + n] : 0.0);
    } else {
        const R *vel = reinterpret_cast<const R *>(ws + c->off_vel);
        const int y = n / c->lx, x = n - y * c->lx;
        R kxx, kxy, kyx, kyy;
        velocity_gradient<R>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx, kyy);
        out[n] = (double)kxx;
        out[N + n] = (double)kxy;
        out[2 * N + n] = (double)kyx;
        out[3 * N + n] = (double)kyy;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

// Precision codes: 0 FP64 lattice + FP64 history, 1 split population storage
// (FP32 remainders, FP64 moments) + FP32 history, 2 FP64 lattice + FP32
// history.  P is the lattice arithmetic and plane type, H the history type,
// S the population storage type.
#define LBMAX_BY_PREC(prec, BODY)                                                \
    do {                                                                         \
        if ((prec) == 0) {                                                       \
            typedef double P;                                                    \
            typedef double H;                                                    \
            typedef double S;                                                    \
            BODY;                                                                \
        } else if ((prec) == 1) {                                                \
            typedef double P;                                                    \
            typedef float H;                                                     \
            typedef float S;                                                     \
            BODY;                                                                \
        } else {                                                                 \
            typedef double P;                                                    \
            typedef float H;                                                     \
            typedef double S;                                                    \
            BODY;                                                                \
        }                                                                        \
    } while (0)

void launch_init(int prec, char *ws, const ChanDev *chans, int ch, const NodeTile *,
                 int n_tiles, const double *u0_dev, hipStream_t st)
{
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_init<P, S>), dim3(n_tiles), dim3(kBlock), 0, st, ws,
                                           chans, ch, u0_dev));
}

void launch_fill_zero(void *p, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0)
        return;
    size_t blocks = (n16 + kBlock - 1) / kBlock;
    if (blocks > 8192)
        blocks = 8192;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                       reinterpret_cast<uint4 *>(p), n16);
}

void launch_lb(int prec, char *ws, const ChanDev *chans, const NodeTile *tiles, int n_tiles,
               const int64_t *tcount, int trel, int *tile_counters, hipStream_t st)
{
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_lb<P, S>), dim3(n_tiles), dim3(kBlock), 0, st, ws,
                                           chans, tiles, tcount, trel, tile_counters));
}

// Shapes of the history pass: (nodes per lane V, steps per pass M, rows
// loaded per group U, rows per partial sum F) for each block length and
// requested lane width.  Blocked passes use one node per lane (the M
// accumulator pairs fill the registers); longer partial sums save
// compensated additions where the pass is bound by vector-ALU issue.  In the
// F-row blocks the rows go in halves of U/2, the loads of one half issued
// before the other half is summed.
#define LBMAX_PASS_SHAPE_TABLE(block, vec, X)                                    \
    do {                                                                         \
        if (block == 1) {                                                        \
            if (vec == 4)                                                        \
                X(4, 1, 4, 32);                                                    \
            else if (vec == 2)                                                   \
                X(2, 1, 8, 32);                                                    \
            else                                                                 \
                X(1, 1, 8, 32);                                                    \
        } else if (block == 2) {                                                 \
            if (vec == 1)                                                        \
                X(1, 2, 8, 32);                                                    \
            else                                                                 \
                X(2, 2, 4, 32);                                                    \
        } else if (block == 4) {                                                 \
            if (vec == 1)                                                        \
                X(1, 4, 8, 32);                                                    \
            else                                                                 \
                X(2, 4, 4, 32);                                                    \
        } else if (block == 8) {                                                 \
            X(1, 8, 8, 32);                                                      \
        } else if (block == 16) {                                                \
            X(1, 16, 8, 32);                                                     \
        } else {                                                                 \
            X(1, 32, (sizeof(H) == 4 ? 16 : 8), 128);                               \
        }                                                                        \
    } while (0)

void launch_hist_pass(int prec, int vec, int block, char *ws, const ChanDev *chans,
                      const HistTile *tiles, int n_tiles, const int64_t *tcount, int trel,
                      int persistent_grid, int *counter, hipStream_t st)
{
    if (n_tiles <= 0)
        return;
    const int per_group = kBlock / kWave;  // one tile per wavefront
    const int groups = (n_tiles + per_group - 1) / per_group;
    const int grid = persistent_grid > 0 ? std::min(persistent_grid, groups) : groups;
#define LBMAX_PASS(V, M, U, F)                                                    \
    do {                                                                         \
        if (persistent_grid > 0)                                                 \
            hipLaunchKernelGGL((k_hist_pass_persistent<P, H, V, M, U, F>), dim3(grid), \
                               dim3(kBlock), 0, st, ws, chans, tiles, n_tiles,   \
                               tcount, trel, counter);                           \
        else                                                                     \
            hipLaunchKernelGGL((k_hist_pass<P, H, V, M, U, F>), dim3(grid),         \
                               dim3(kBlock), 0, st, ws, chans, tiles, n_tiles,   \
                               tcount, trel);                                    \
    } while (0)
#define LBMAX_PASS_SHAPES LBMAX_PASS_SHAPE_TABLE(block, vec, LBMAX_PASS)
    LBMAX_BY_PREC(prec, LBMAX_PASS_SHAPES);
#undef LBMAX_PASS_SHAPES
#undef LBMAX_PASS
}

// Workgroups of the persistent pass that are resident on one compute unit.
int hist_pass_blocks_per_cu(int prec, int vec, int block)
{
    int n = 0;
    hipError_t e = hipSuccess;
#define LBMAX_OCC(V, M, U, F)                                                         \
    do {                                                                             \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                            \
            &n, reinterpret_cast<const void *>(&k_hist_pass_persistent<P, H, V, M, U, F>), \
            kBlock, 0);                                                              \
    } while (0)
#define LBMAX_OCC_SHAPES LBMAX_PASS_SHAPE_TABLE(block, vec, LBMAX_OCC)
    LBMAX_BY_PREC(prec, LBMAX_OCC_SHAPES);
#undef LBMAX_OCC_SHAPES
#undef LBMAX_OCC
    return (e == hipSuccess && n > 0) ? n : 1;
}

// Shapes of the full-tensor pass: (steps per pass M, rows per group U, rows
// per partial sum F); three sums per step limit the block to 16 steps.
#define LBMAX_FINGER_SHAPE_TABLE(block, X)                                      \
    do {                                                                         \
        if (block == 1)                                                          \
            X(1, 8, 8);                                                          \
        else if (block == 2)                                                     \
            X(2, 4, 8);                                                          \
        else if (block == 4)                                                     \
            X(4, 4, 8);                                                          \
        else if (block == 8)                                                     \
            X(8, 4, 16);                                                         \
        else                                                                     \
            X(16, 4, 16);                                                        \
    } while (0)

void launch_finger_pass(int prec, int block, char *ws, const ChanDev *chans,
                        const HistTile *tiles, int n_tiles, const int64_t *tcount, int trel,
                        int persistent_grid, int *counter, hipStream_t st)
{
    if (n_tiles <= 0)
        return;
    const int grid = persistent_grid > 0 ? std::min(persistent_grid, n_tiles) : n_tiles;
#define LBMAX_FPASS(M, U, F)                                                     \
    do {                                                                         \
        if (persistent_grid > 0)                                                 \
            hipLaunchKernelGGL((k_finger_pass_persistent<P, H, M, U, F>), dim3(grid), \
                               dim3(kBlock), 0, st, ws, chans, tiles, n_tiles,   \
                               tcount, trel, counter);                           \
        else                                                                     \
            hipLaunchKernelGGL((k_finger_pass<P, H, M, U, F>), dim3(grid),       \
                               dim3(kBlock), 0, st, ws, chans, tiles, tcount,    \
                               trel);                                            \
    } while (0)
#define LBMAX_FPASS_SHAPES LBMAX_FINGER_SHAPE_TABLE(block, LBMAX_FPASS)
    LBMAX_BY_PREC(prec, LBMAX_FPASS_SHAPES);
#undef LBMAX_FPASS_SHAPES
#undef LBMAX_FPASS
}

int finger_pass_blocks_per_cu(int prec, int block)
{
    int n = 0;
    hipError_t e = hipSuccess;
#define LBMAX_FOCC(M, U, F)                                                          \
    do {                                                                             \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                            \
            &n, reinterpret_cast<const void *>(&k_finger_pass_persistent<P, H, M, U, F>), \
            kBlock, 0);                                                              \
    } while (0)
#define LBMAX_FOCC_SHAPES LBMAX_FINGER_SHAPE_TABLE(block, LBMAX_FOCC)
    LBMAX_BY_PREC(prec, LBMAX_FOCC_SHAPES);
#undef LBMAX_FOCC_SHAPES
#undef LBMAX_FOCC
    return (e == hipSuccess && n > 0) ? n : 1;
}

void launch_wm_pass(int prec, int block, char *ws, const ChanDev *chans, const HistTile *tiles,
                    int n_tiles, const int64_t *tcount, int trel, hipStream_t st)
{
    if (n_tiles <= 0)
        return;
#define LBMAX_WM(MM) hipLaunchKernelGGL((k_wm_pass<P, H, MM>), dim3(n_tiles), dim3(kBlock), 0, \
                                        st, ws, chans, tiles, tcount, trel)
#define LBMAX_WM_SHAPES                                                          \
    do {                                                                         \
        if (block == 1)                                                          \
            LBMAX_WM(1);                                                         \
        else if (block == 2)                                                     \
            LBMAX_WM(2);                                                         \
        else if (block == 4)                                                     \
            LBMAX_WM(4);                                                         \
        else if (block == 8)                                                     \
            LBMAX_WM(8);                                                         \
        else if (block == 16)                                                    \
            LBMAX_WM(16);                                                        \
        else                                                                     \
            LBMAX_WM(32);                                                        \
    } while (0)
    LBMAX_BY_PREC(prec, LBMAX_WM_SHAPES);
#undef LBMAX_WM_SHAPES
#undef LBMAX_WM
}

void launch_inst_step(int prec, char *ws, const ChanDev *chans, const NodeTile *tiles,
                      int n_tiles, const int64_t *, int, hipStream_t st)
{
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL(k_inst_step<P>, dim3(n_tiles), dim3(kBlock), 0, st,
                                           ws, chans, tiles));
}

void launch_combine(int prec, int block, char *ws, const ChanDev *chans, const NodeTile *tiles,
                    int n_tiles, hipStream_t st)
{
    if (n_tiles <= 0 || block <= 0)
        return;
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL(k_combine<P>, dim3(n_tiles, block), dim3(kBlock), 0,
                                           st, ws, chans, tiles));
}

void launch_fused_steps(int prec, bool lds, char *ws, const ChanDev *chans, int n_ch,
                        const int64_t *tcount, int trel, int m0, int count, hipStream_t st)
{
    if (n_ch <= 0 || count <= 0)
        return;
    if (!lds) {
        LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_fused_steps<P, H, S>), dim3(n_ch),
                                               dim3(kFuseThreads), 0, st, ws, chans, tcount,
                                               trel, m0, count));
        return;
    }
    if (prec == 1)
        hipLaunchKernelGGL((k_fused_steps_lds<double, float>), dim3(n_ch), dim3(kFuseThreads),
                           fused_lds_bytes(prec), st, ws, chans, tcount, trel, m0, count);
}

// Rebuilt populations, velocity and stress: 13 FP64 planes.
size_t fused_lds_bytes(int prec)
{
    return prec == 1 ? (size_t)kFuseThreads * 13 * sizeof(double) : 0;
}

int prepare_fused_lds(int prec)
{
    // Split storage only: with FP64 populations the state would not fit
    if (prec != 1)
        return -1;
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused_steps_lds<double, float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)fused_lds_bytes(prec));
    return e == hipSuccess ? 0 : -1;
}

void launch_hist_step(int prec, int m, char *ws, const ChanDev *chans, const NodeTile *tiles,
                      int n_tiles, const int64_t *tcount, int trel, hipStream_t st)
{
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_hist_step<P, H>), dim3(n_tiles), dim3(kBlock), 0,
                                           st, ws, chans, tiles, tcount, trel, m));
}

void launch_grid_step(int prec, int block, int m, char *ws, const ChanDev *chans,
                      const NodeTile *tiles, int n_tiles, const int64_t *tcount, int trel,
                      hipStream_t st)
{
    block = block < kMaxGridBlock ? block : kMaxGridBlock;
    m %= block;
    if (block <= 1) {
        LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_grid_step<P, H>), dim3(n_tiles),
                                               dim3(kBlock), 0, st, ws, chans, tiles, tcount,
                                               trel));
    } else if (m > 0) {
        LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_grid_edges<P, H>), dim3(n_tiles),
                                               dim3(kBlock), 0, st, ws, chans, tiles, tcount,
                                               trel, m, block));
    } else {
#define LBMAX_GRID_PASS(MM)                                                                   \
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_grid_pass<P, H, MM>), dim3(n_tiles), dim3(kBlock), \
                                           0, st, ws, chans, tiles, tcount, trel))
        switch (block) {
        case 2: LBMAX_GRID_PASS(2); break;
        case 4: LBMAX_GRID_PASS(4); break;
        case 8: LBMAX_GRID_PASS(8); break;
        default: LBMAX_GRID_PASS(16); break;
        }
#undef LBMAX_GRID_PASS
    }
}

void launch_tick(int64_t *tcount, int64_t add, hipStream_t st)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, tcount, add);
}

void launch_set_force(ChanDev *chans, int ch, double gx, double gy, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_force, dim3(1), dim3(64), 0, st, chans, ch, gx, gy);
}

void launch_readout(int prec, int which, char *ws, const ChanDev *chans, int ch,
                    int n_nodes, double *stage, hipStream_t st)
{
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL(k_readout<P>, dim3(blocks_for(n_nodes)),
                                           dim3(kBlock), 0, st, which, ws, chans, ch, stage));
}


// ===========================================================================
// Discrete adjoint of the step for unidirectional channels (lx = 1: d/dx
// vanishes, sigma_xx never reaches the force, |gamma_dot| = |s|).  The
// reverse sweep runs t = T-1 .. 0; per step two kernels:
//   k_adj_a(t): sigma_bar^t = Dy^T fbar(t+1) pushed into the adjoint ring,
//     nbar(t) = streaming^T dbar(t+1), and the history transpose, a gather
//     over the future adjoint stresses:
//       S0 = sum_j w_j sigma_bar^{t+j} E_j,  S1 = sum_j w_j sigma_bar^{t+j} E_j j,
//       E_j = exp(-j (1/tau + |s_t|/gamma_c)),
//       sbar_t = G (S0 - |s_t| S1 / gamma_c)
//     (d/ds of s E_j(|s|) is E_j (1 - j |s| / gamma_c)), plus the parameter
//     terms dL/dG += s_t S0, dL/dtau += G s_t S1 / tau^2,
//     dL/dgamma_c += G s_t |s_t| S1 / gamma_c^2.
//   k_adj_b(t): the step's collision, moments and force recomputed from the
//     recorded n*(t-1), sigma^{t-1}; their transposes give dbar(t), fbar(t),
//     and dL/dg_x += fbar_x rho.
// Per-node FP64 accumulators; no atomics, fixed order.
// ===========================================================================

// d s(y) / d u(yp) of the velocity-gradient stencil in y.
template <typename R>
__device__ __forceinline__ R coef_grad(int y, int yp, int ly)
{
    if (y == 0)
        return yp == 0 ? R(1) : (yp == 1 ? R(1) / R(3) : R(0));
    if (y == ly - 1)
        return yp == ly - 1 ? R(-1) : (yp == ly - 2 ? R(-1) / R(3) : R(0));
    return yp == y + 1 ? R(0.5) : (yp == y - 1 ? R(-0.5) : R(0));
}

// d f(y) / d sigma(yp) of the stress-divergence stencil in y.
template <typename R>
__device__ __forceinline__ R coef_div(int y, int yp, int ly)
{
    if (y == 0)
        return yp == 0 ? R(-1.5) : (yp == 1 ? R(2) : (yp == 2 ? R(-0.5) : R(0)));
    if (y == ly - 1)
        return yp == ly - 1 ? R(1.5) : (yp == ly - 2 ? R(-2) : (yp == ly - 3 ? R(0.5) : R(0)));
    return yp == y + 1 ? R(0.5) : (yp == y - 1 ? R(-0.5) : R(0));
}

// sigma_bar^t of node y (the divergence stencil's transpose applied to
// fbar(t+1)) into ring slot p = t mod n_hist of the adjoint ring, and nbar(t)
// (the pull-stream's transpose, the push map, applied to dbar(t+1)).
template <typename R>
__device__ __forceinline__ R adj_push(const ChanDev *c, const AdjChan *a, char *aws, int p,
                                      int y)
{
    const int ly = c->ly;
    const size_t np = (size_t)c->np;
    R *sring = reinterpret_cast<R *>(aws + a->off_sbar_ring);
    const R *fbar = reinterpret_cast<const R *>(aws + a->off_fbar);
    const R *dbar = reinterpret_cast<const R *>(aws + a->off_dbar);
    R *nbar = reinterpret_cast<R *>(aws + a->off_nbar);
    R sb = R(0);
    for (int yy = max(0, y - 2); yy <= min(ly - 1, y + 2); ++yy)
        sb += coef_div<R>(yy, y, ly) * fbar[yy];
    sring[(size_t)p * np + y] = sb;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int yt = y + QY[q];
        nbar[q * np + y] = (yt >= 0 && yt < ly) ? dbar[q * np + yt] : dbar[QOPP[q] * np + y];
    }
    return sb;
}

// Workgroup of k_adj_a: kAdjNodes nodes x kAdjChunks age ranges of one of
// kAdjGroups parts of the adjoint window; thread = node + kAdjNodes * range,
// so each wavefront reads kAdjNodes consecutive nodes of 64 / kAdjNodes
// ranges.  The kAdjGroups x kAdjChunks ranges split [0, n_hist) with rounded-up
// bounds, so the first range always holds age 0 (the entry pushed by the same
// workgroup).
constexpr int kAdjNodes = 16;
constexpr int kAdjChunks = 64;
constexpr int kAdjRanges = kAdjGroups * kAdjChunks;

// Adjoint of the pushed shear rate at node y (the history transpose of step
// t combined over the kAdjGroups partial sums in group order) and the two
// sums themselves; s_t from the step's record (recs: the segment slot's row).
template <typename RH>
__device__ __forceinline__ double adj_sbar(const RH *recs, const ChanDev *c, const double *part,
                                           int y, double &S0, double &S1, double &s)
{
    const size_t np = (size_t)c->np;
    S0 = 0.0;
    S1 = 0.0;
#pragma unroll
    for (int g = 0; g < kAdjGroups; ++g) {
        S0 += part[(size_t)(2 * g) * np + y];
        S1 += part[(size_t)(2 * g + 1) * np + y];
    }
    s = (double)recs[y];
    return c->g_inf * (S0 - fabs(s) * S1 * c->inv_gc);
}

template <typename R, typename RH>
__global__ __launch_bounds__(kAdjNodes * kAdjChunks) void k_adj_a(const ChanDev *__restrict__ chans,
                                                              const NodeTile *__restrict__ tiles,
                                                              char *__restrict__ aws,
                                                              const AdjChan *__restrict__ achans,
                                                              const int64_t *__restrict__ t0,
                                                              int slot, int buf)
{
    const int64_t t = *t0 + slot;
    __shared__ double part[2][kAdjChunks][kAdjNodes];
    constexpr int kSub = kBlock / kAdjNodes;  // node groups per node tile
    const int grp = (int)(blockIdx.x % kAdjGroups);
    const int sub = (int)(blockIdx.x / kAdjGroups);
    const NodeTile tl = tiles[sub / kSub];
    const ChanDev *c = chans + tl.ch;
    const AdjChan *a = achans + tl.ch;
    const int lane = (int)(threadIdx.x % kAdjNodes), chunk = (int)(threadIdx.x / kAdjNodes);
    // lx = 1: node index = y
    const int y = tl.n0 + (sub % kSub) * kAdjNodes + lane;
    const int ly = c->ly;
    const bool own = y < ly;
    const size_t np = (size_t)c->np;
    const int H = c->n_hist;
    const int p = (int)(t % H);
    const R *sring = reinterpret_cast<const R *>(aws + a->off_sbar_ring);

    if (own && chunk == 0 && grp == 0)
        adj_push<R>(c, a, aws, p, y);
    __syncthreads();  // sigma_bar^t is in the ring before any range reads age 0

    // History transpose for the entry of step t over the ages j of this
    // wavefront's range [j0, j1): S0 = sum w_j sbar^{t+j} E_j,
    // S1 = sum w_j sbar^{t+j} E_j j, E_j = q^j with q = exp(-rate) carried from
    // E_{j0} = exp(-j0 rate); the ranges combine in FP64 below.
    R s = R(0);
    double rate = 0.0, S0 = 0.0, S1 = 0.0;
    const int64_t rg = (int64_t)grp * kAdjChunks + chunk;
    const int j0 = (int)(((int64_t)H * rg + kAdjRanges - 1) / kAdjRanges);
    const int j1 = (int)(((int64_t)H * (rg + 1) + kAdjRanges - 1) / kAdjRanges);
    if (own && j0 < j1) {
        s = (R)reinterpret_cast<const RH *>(aws + a->off_recs[buf])[(size_t)slot * np + y];
        rate = c->inv_tau + c->inv_gc * (double)fabs(s);
        const double q = exp(-rate);
        double e = exp(-(double)j0 * rate);
        int slot = p + j0;
        if (slot >= H)
            slot -= H;
        constexpr int L = 8;  // ring rows loaded ahead
        for (int jb = j0; jb < j1; jb += L) {
            R v[L];
#pragma unroll
            for (int u = 0; u < L; ++u) {
                int sl = slot + u;
                if (sl >= H)
                    sl -= H;
                v[u] = jb + u < j1 ? sring[(size_t)sl * np + y] : R(0);
            }
#pragma unroll
            for (int u = 0; u < L; ++u) {
                const int j = jb + u;
                if (j < j1) {
                    const double w = (j == 0 || j == H - 1) ? 0.5 : 1.0;
                    const double x = w * (double)v[u] * e;
                    S0 += x;
                    S1 += x * (double)j;
                    e *= q;
                }
            }
            slot += L;
            if (slot >= H)
                slot -= H;
        }
    }
    part[0][chunk][lane] = S0;
    part[1][chunk][lane] = S1;
    __syncthreads();
    if (!own || chunk != 0)
        return;
    S0 = 0.0;
    S1 = 0.0;
    for (int k = 0; k < kAdjChunks; ++k) {
        S0 += part[0][k][lane];
        S1 += part[1][k][lane];
    }
    // this group's sums; k_adj_b combines the groups in group order
    double *gpart = reinterpret_cast<double *>(aws + a->off_part);
    gpart[(size_t)(2 * grp) * np + y] = S0;
    gpart[(size_t)(2 * grp + 1) * np + y] = S1;
}

// The lattice part of reverse step `slot` at node y: the step's moments,
// force and collision recomputed from the recorded n*(t-1) and sigma^{t-1}
// in the order and arithmetic of k_lb, their transposes (dbar(t), fbar(t)),
// the loss, the velocity-gradient transpose of the pushed shear rates of y
// and its neighbours (sbar_of(yy, S0, S1, s) gives sbar at node yy, and at yy
// = y also the history sums and s for the parameter terms), and the parameter
// gradients' per-node accumulators.  Split into the loads of the step's
// records (adj_load_step), which do not depend on the sweep, and the
// arithmetic (adj_lattice_core), which takes nbar(t) as A, adds to the
// accumulators through acc_add(k, v) and hands out dbar(t) and fbar(t)
// through put(q, v) (q = 9: fbar).
template <typename R>
struct AdjStepIn {
    R d[9];     // pulled populations n*(t-1) at node y
    R sg[3];    // sigma^{t-1} of the divergence stencil at node y
    double dldu;  // dL/du_x(t) at node y
};

template <typename R>
__device__ __forceinline__ void adj_load_step(const ChanDev *c, const AdjChan *a, const char *aws,
                                              int slot, int buf, int y, AdjStepIn<R> &in)
{
    const int ly = c->ly;
    const size_t np = (size_t)c->np;
    const R *rec = reinterpret_cast<const R *>(aws + a->off_rec[buf]) + (size_t)slot * 10 * np;
    const R *sig = rec + 9 * np;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ys = y - QY[q];
        in.d[q] = (ys >= 0 && ys < ly) ? rec[q * np + ys] : rec[QOPP[q] * np + y];
    }
    // stencil nodes: (0, 1, 2) at the first node, (y, y - 1, y - 2) at the
    // last, (y + 1, y - 1, -) inside; every load is issued (indices selected
    // and clamped to the channel), so the loads of a step stay in one
    // sequence for the wait counters
    const int i0 = y == 0 ? 0 : (y == ly - 1 ? y : y + 1);
    const int i1 = y == 0 ? min(1, ly - 1) : y - 1;
    const int i2 = y == 0 ? min(2, ly - 1) : (y == ly - 1 ? max(y - 2, 0) : y);
    in.sg[0] = sig[i0];
    in.sg[1] = sig[i1];
    in.sg[2] = sig[i2];
    in.dldu = reinterpret_cast<const double *>(aws + a->off_dldu[buf])[(size_t)slot * np + y];
}

template <typename R, typename SbarOf, typename AccAdd, typename Put>
__device__ __forceinline__ void adj_lattice_core(const ChanDev *c, int y, const AdjStepIn<R> &in,
                                                 const R (&A)[9], SbarOf &&sbar_of,
                                                 AccAdd &&acc_add, Put &&put)
{
    const int ly = c->ly;
    const R *d = in.d;
    const R drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const R jx = (d[1] - d[2]) + (d[5] - d[6]) + (d[7] - d[8]);
    const R jy = (d[3] - d[4]) + (d[5] - d[6]) + (d[8] - d[7]);
    const R rho = R(1) + drho;
    R dys;
    if (y == 0)
        dys = R(0.5) * (R(-3) * in.sg[0] + R(4) * in.sg[1] - in.sg[2]);
    else if (y == ly - 1)
        dys = R(0.5) * (R(3) * in.sg[0] - R(4) * in.sg[1] + in.sg[2]);
    else
        dys = R(0.5) * (in.sg[0] - in.sg[1]);
    const R gx = (R)c->gx;
    const R fx = dys + rho * gx;
    const R ux = (jx + R(0.5) * fx) / rho;
    const R uy = jy / rho;
    const R om = (R)c->omega;
    const R pf = R(1) - R(0.5) * om;

    // collision + forcing transpose
    R drho_b = R(0), ux_b = R(0), uy_b = R(0), fx_b = R(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const R cx = R(QX[q]), cy = R(QY[q]);
        const R w = qweight<R>(q);
        const R cu = cx * ux + cy * uy;
        const R P = R(3) * cu + R(4.5) * cu * cu - R(1.5) * (ux * ux + uy * uy);
        drho_b += om * A[q] * w * (R(1) + P);
        ux_b += om * A[q] * w * rho * (R(3) * cx + R(9) * cu * cx - R(3) * ux) +
                A[q] * w * pf * (R(-3) * fx + R(9) * cx * cx * fx);
        uy_b += om * A[q] * w * rho * (R(3) * cy + R(9) * cu * cy - R(3) * uy) +
                A[q] * w * pf * R(9) * cy * cx * fx;
        fx_b += A[q] * w * pf * (R(3) * (cx - ux) + R(9) * cu * cx);
    }
    // the loss and the velocity-gradient transpose
    ux_b += (R)in.dldu;
    for (int yy = max(0, y - 1); yy <= min(ly - 1, y + 1); ++yy) {
        double S0, S1, s;
        const R sbar = (R)sbar_of(yy, S0, S1, s);
        ux_b += coef_grad<R>(yy, y, ly) * sbar;
        if (yy == y) {
            // parameter terms of the history transpose at this node
            const double G = c->g_inf, as = fabs(s);
            acc_add(0, s * S0);
            acc_add(1, G * s * S1 * c->inv_tau * c->inv_tau);
            acc_add(2, G * s * as * S1 * c->inv_gc * c->inv_gc);
        }
    }
    // u = (j + f/2) / rho
    const R jx_b = ux_b / rho;
    const R jy_b = uy_b / rho;
    fx_b += ux_b / (R(2) * rho);
    drho_b -= (ux * ux_b + uy * uy_b) / rho;
    // f_x = Dy sigma + rho g_x
    drho_b += fx_b * gx;
    acc_add(3, (double)fx_b * (double)rho);
    // moments of the pulled populations
#pragma unroll
    for (int q = 0; q < 9; ++q)
        put(q, (R(1) - om) * A[q] + drho_b + R(QX[q]) * jx_b + R(QY[q]) * jy_b);
    put(9, fx_b);
}

template <typename R, typename RH, typename SbarOf>
__device__ __forceinline__ void adj_lattice(const ChanDev *c, const AdjChan *a, char *aws,
                                            int slot, int buf, int y, SbarOf &&sbar_of)
{
    const size_t np = (size_t)c->np;
    AdjStepIn<R> in;
    adj_load_step<R>(c, a, aws, slot, buf, y, in);
    const R *nbar = reinterpret_cast<const R *>(aws + a->off_nbar);
    R A[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
        A[q] = nbar[q * np + y];
    double *acc = reinterpret_cast<double *>(aws + a->off_acc);
    R *dbar = reinterpret_cast<R *>(aws + a->off_dbar);
    R *fbar = reinterpret_cast<R *>(aws + a->off_fbar);
    adj_lattice_core<R>(c, y, in, A, sbar_of,
                        [&](int k, double v) { acc[k * np + y] += v; },
                        [&](int q, R v) {
                            if (q < 9)
                                dbar[q * np + y] = v;
                            else
                                fbar[y] = v;
                        });
}

template <typename R, typename RH>
__global__ __launch_bounds__(kBlock) void k_adj_b(const ChanDev *__restrict__ chans,
                                                  const NodeTile *__restrict__ tiles,
                                                  char *__restrict__ aws,
                                                  const AdjChan *__restrict__ achans,
                                                  const int64_t *__restrict__ t0, int slot,
                                                  int buf)
{
    (void)t0;
    const NodeTile tl = tiles[blockIdx.x];
    const ChanDev *c = chans + tl.ch;
    const AdjChan *a = achans + tl.ch;
    const int y = tl.n0 + threadIdx.x;
    if (y >= c->ly)
        return;
    const RH *recs = reinterpret_cast<const RH *>(aws + a->off_recs[buf]) + (size_t)slot * c->np;
    const double *part = reinterpret_cast<const double *>(aws + a->off_part);
    adj_lattice<R, RH>(c, a, aws, slot, buf, y,
                       [&](int yy, double &S0, double &S1, double &s) {
                           return adj_sbar<RH>(recs, c, part, yy, S0, S1, s);
                       });
}

// Blocked reverse sweep.  The history transpose of the entry pushed at step
// t sums over the ages j of the window in fixed parts: the near ages [0,
// kAdjMaxBlock) in order, then the far ages [kAdjMaxBlock, n_hist) as
// kAdjBulkRanges ranges, each in order, whose sums are added in range order
// and then to the near sum.  For a block of reverse steps t = t0 + slot, slot
// = slot_hi, slot_hi - 1, ..., slot_hi - count + 1 (count <= kAdjMaxBlock),
// the far ages reach adjoint stresses of steps after the block, all in the
// ring before the block starts: k_adj_bulk sums them for the whole block in
// one launch, and a span kernel runs the block's steps one by one with the
// near ages.  The parts do not depend on the block or the segment a step
// falls in, so the gradients do not depend on the block size or the segment
// length; the per-step kernels above split the window in another way and
// agree up to the order of the FP64 sums.
//
// k_adj_bulk: workgroup = kAdjBulkNodes nodes x kAdjBulkRanges far ranges of
// one entry of the block; thread = node + kAdjBulkNodes * range.  Each thread
// sums its range, B0 = sum w_j sbar^{t+j} E_j and B1 = sum w_j sbar^{t+j} E_j
// j with E_j = q^j carried from one exp at the range's first age; the
// ranges combine through LDS in range order.
constexpr int kAdjBulkNodes = 16;
static_assert(kAdjBulkNodes * kAdjBulkRanges == kBlock, "bulk workgroup shape");

template <typename R, typename RH>
__global__ __launch_bounds__(kBlock) void k_adj_bulk(const ChanDev *__restrict__ chans,
                                                     const NodeTile *__restrict__ tiles,
                                                     int n_tiles, char *__restrict__ aws,
                                                     const AdjChan *__restrict__ achans,
                                                     const int64_t *__restrict__ t0, int slot_hi,
                                                     int count, int buf)
{
    __shared__ double part[2][kAdjBulkRanges][kAdjBulkNodes];
    constexpr int kSub = kBlock / kAdjBulkNodes;  // node groups per node tile
    const NodeTile tl = tiles[blockIdx.x % n_tiles];
    const int sub = (int)((blockIdx.x / n_tiles) % kSub);
    const int m = (int)(blockIdx.x / (n_tiles * kSub));
    const ChanDev *c = chans + tl.ch;
    const AdjChan *a = achans + tl.ch;
    const int y0 = tl.n0 + sub * kAdjBulkNodes;
    if (y0 >= c->ly || m >= count)
        return;  // whole workgroup
    const int lane = (int)(threadIdx.x % kAdjBulkNodes), r = (int)(threadIdx.x / kAdjBulkNodes);
    const int y = y0 + lane;
    const bool own = y < c->ly;
    const size_t np = (size_t)c->np;
    const int H = c->n_hist;
    const int slot = slot_hi - m;
    const int64_t t = *t0 + slot;
    // far range r: ages [ja, jb)
    const int lo = min(kAdjMaxBlock, H);
    const int ja = lo + (int)((int64_t)(H - lo) * r / kAdjBulkRanges);
    const int jb = lo + (int)((int64_t)(H - lo) * (r + 1) / kAdjBulkRanges);
    double S0 = 0.0, S1 = 0.0;
    if (own && ja < jb) {
        const R *sring = reinterpret_cast<const R *>(aws + a->off_sbar_ring);
        const R s = (R)reinterpret_cast<const RH *>(aws + a->off_recs[buf])[(size_t)slot * np + y];
        const double rate = c->inv_tau + c->inv_gc * (double)fabs(s);
        const double q = exp(-rate);
        double e = exp(-(double)ja * rate);
        int sl = (int)((t + ja) % H);
        constexpr int L = 8;  // ring rows loaded ahead
        for (int j0 = ja; j0 < jb; j0 += L) {
            R v[L];
#pragma unroll
            for (int u = 0; u < L; ++u) {
                int su = sl + u;
                if (su >= H)
                    su -= H;
                v[u] = j0 + u < jb ? sring[(size_t)su * np + y] : R(0);
            }
#pragma unroll
            for (int u = 0; u < L; ++u) {
                const int j = j0 + u;
                if (j < jb) {
                    const double w = j == H - 1 ? 0.5 : 1.0;
                    const double x = w * (double)v[u] * e;
                    S0 += x;
                    S1 += x * (double)j;
                    e *= q;
                }
            }
            sl += L;
            if (sl >= H)
                sl -= H;
        }
    }
    part[0][r][lane] = S0;
    part[1][r][lane] = S1;
    __syncthreads();
    if (!own || r != 0)
        return;
    S0 = 0.0;
    S1 = 0.0;
#pragma unroll
    for (int k = 0; k < kAdjBulkRanges; ++k) {
        S0 += part[0][k][lane];
        S1 += part[1][k][lane];
    }
    double *bulk = reinterpret_cast<double *>(aws + a->off_bulk);
    bulk[(size_t)(2 * m) * np + y] = S0;
    bulk[(size_t)(2 * m + 1) * np + y] = S1;
}

// Near sum of the entry at node y: S0 = sum_{j <= jn} w_j sbar^{t+j} E_j,
// S1 = sum w_j sbar^{t+j} E_j j in age order with E_j = q^j (w = 1/2 at the
// window's ends); near(j) gives sbar^{t+j}.
template <typename Near>
__device__ __forceinline__ void adj_near_sum(int jn, int H, double q, Near &&near, double &S0,
                                             double &S1)
{
    S0 = 0.0;
    S1 = 0.0;
    double e = 1.0;
    if (H > kAdjMaxBlock) {
        // every near age, the window's end beyond them: no bound to test
#pragma unroll
        for (int j = 0; j < kAdjMaxBlock; ++j) {
            const double w = j == 0 ? 0.5 : 1.0;
            const double x = w * near(j) * e;
            S0 += x;
            S1 += x * (double)j;
            e *= q;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < kAdjMaxBlock; ++j) {
        if (j <= jn) {
            const double w = (j == 0 || j == H - 1) ? 0.5 : 1.0;
            const double x = w * near(j) * e;
            S0 += x;
            S1 += x * (double)j;
            e *= q;
        }
    }
}

// k_adj_span: one workgroup per channel runs the block's steps in reverse
// order; per step, for every node, the push of sigma_bar^t and nbar(t), the
// near sum plus the far sum of the bulk pass, with sbar_t and the node's
// sums into LDS; a barrier; the lattice part with the neighbours' sbar from
// LDS; and a barrier before the next step reads dbar and fbar.
// kAdjSpanThreads threads loop over the channel's nodes (the lattice part
// needs about 180 registers a lane); the near ages come from the adjoint
// ring and the adjoint state from device memory.
constexpr int kAdjSpanThreads = 256;

template <typename R, typename RH>
__global__ __launch_bounds__(kAdjSpanThreads) void k_adj_span(const ChanDev *__restrict__ chans,
                                                              char *__restrict__ aws,
                                                              const AdjChan *__restrict__ achans,
                                                              const int64_t *__restrict__ t0,
                                                              int slot_hi, int count, int buf)
{
    __shared__ double s_sbar[kFuseThreads], s_S0[kFuseThreads], s_S1[kFuseThreads],
        s_s[kFuseThreads];
    const ChanDev *c = chans + blockIdx.x;
    const AdjChan *a = achans + blockIdx.x;
    const int ly = c->ly;
    const size_t np = (size_t)c->np;
    const int H = c->n_hist;
    const int jn = min(kAdjMaxBlock, H) - 1;  // last near age
    const R *sring = reinterpret_cast<const R *>(aws + a->off_sbar_ring);
    const RH *recs = reinterpret_cast<const RH *>(aws + a->off_recs[buf]);
    const double *bulk = reinterpret_cast<const double *>(aws + a->off_bulk);
    const int64_t t_hi = *t0 + slot_hi;
    for (int m = 0; m < count; ++m) {
        const int64_t t = t_hi - m;
        const int p = (int)(t % H);
        for (int y = threadIdx.x; y < ly; y += kAdjSpanThreads) {
            // loads that do not wait for this step's push
            const double s = (double)recs[(size_t)(slot_hi - m) * np + y];
            const double b0 = bulk[(size_t)(2 * m) * np + y];
            const double b1 = bulk[(size_t)(2 * m + 1) * np + y];
            adj_push<R>(c, a, aws, p, y);
            const double q = exp(-(c->inv_tau + c->inv_gc * fabs(s)));
            double S0, S1;
            adj_near_sum(jn, H, q,
                         [&](int j) {
                             int sl = p + j;
                             if (sl >= H)
                                 sl -= H;
                             return (double)sring[(size_t)sl * np + y];
                         },
                         S0, S1);
            S0 += b0;
            S1 += b1;
            s_S0[y] = S0;
            s_S1[y] = S1;
            s_s[y] = s;
            s_sbar[y] = c->g_inf * (S0 - fabs(s) * S1 * c->inv_gc);
        }
        __syncthreads();  // every node's sbar_t is in LDS
        for (int y = threadIdx.x; y < ly; y += kAdjSpanThreads)
            adj_lattice<R, RH>(c, a, aws, slot_hi - m, buf, y,
                               [&](int yy, double &S0, double &S1, double &s) {
                                   S0 = s_S0[yy];
                                   S1 = s_S1[yy];
                                   s = s_s[yy];
                                   return s_sbar[yy];
                               });
        __syncthreads();  // dbar(t), fbar(t) written before the next step reads them
    }
}

// k_adj_span_lds: the same steps for channels of at most kAdjSpanLdsNodes
// nodes, one thread per node, with the whole adjoint state of the block on
// chip: dbar and fbar in LDS (read from device memory at the start, written
// back at the end), nbar(t) in registers from the push to the lattice part,
// the parameter accumulators in registers, and the near ages in an LDS ring
// of kAdjNearRows rows indexed by step (filled from the adjoint ring at the
// start and by each push: the block's entries reach from kAdjMaxBlock - 1
// steps after the block to its first step; the block's pushes go to the
// adjoint ring at the end).  Each step's records are loaded one step ahead,
// so a step waits on no device memory.  Same values in the same order as
// k_adj_span.
constexpr int kAdjSpanLdsNodes = 128;
constexpr int kAdjNearRows = 2 * kAdjMaxBlock;
static_assert((kAdjNearRows & (kAdjNearRows - 1)) == 0, "the near ring is indexed with a mask");

template <typename R, typename RH>
__global__ __launch_bounds__(kAdjSpanLdsNodes) void k_adj_span_lds(
    const ChanDev *__restrict__ chans, char *__restrict__ aws, const AdjChan *__restrict__ achans,
    const int64_t *__restrict__ t0, int slot_hi, int count, int buf)
{
    constexpr int N = kAdjSpanLdsNodes;
    __shared__ double s_sbar[N], s_S0[N], s_S1[N], s_s[N];
    __shared__ R s_near[kAdjNearRows][N];
    __shared__ R s_fbar[N], s_dbar[9][N];
    const ChanDev *c = chans + blockIdx.x;
    const AdjChan *a = achans + blockIdx.x;
    const int ly = c->ly;
    if (ly > N)
        return;  // whole workgroup; the launcher takes this kernel only when no channel is wider
    const size_t np = (size_t)c->np;
    const int H = c->n_hist;
    const int jn = min(kAdjMaxBlock, H) - 1;  // last near age
    const int y = threadIdx.x;
    const bool own = y < ly;
    R *sring = reinterpret_cast<R *>(aws + a->off_sbar_ring);
    const RH *recs = reinterpret_cast<const RH *>(aws + a->off_recs[buf]);
    const double *bulk = reinterpret_cast<const double *>(aws + a->off_bulk);
    R *g_fbar = reinterpret_cast<R *>(aws + a->off_fbar);
    R *g_dbar = reinterpret_cast<R *>(aws + a->off_dbar);
    double *g_acc = reinterpret_cast<double *>(aws + a->off_acc);
    const int64_t t_hi = *t0 + slot_hi;

    // steps t_hi + 1 .. t_hi + jn, pushed before the block
    for (int i = threadIdx.x; i < jn * ly; i += N) {
        const int k = 1 + i / ly, yy = i % ly;
        const int64_t u = t_hi + k;
        s_near[u % kAdjNearRows][yy] = sring[(size_t)(u % H) * np + yy];
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (own) {
        s_fbar[y] = g_fbar[y];
#pragma unroll
        for (int q = 0; q < 9; ++q)
            s_dbar[q][y] = g_dbar[q * np + y];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            acc[k] = g_acc[k * np + y];
    }
    // A step's inputs: records, s (converted where used, so that its load
    // stays in flight) and the far sums.
    struct In {
        AdjStepIn<R> rec;
        RH s;
        double b0, b1;
    };
    const auto load = [&](int m, In &in) {
        const int slot = slot_hi - m;
        adj_load_step<R>(c, a, aws, slot, buf, y, in.rec);
        in.s = recs[(size_t)slot * np + y];
        in.b0 = bulk[(size_t)(2 * m) * np + y];
        in.b1 = bulk[(size_t)(2 * m + 1) * np + y];
    };
    // Step m with its inputs in `cur`; the next step's go to `nxt` while
    // this one runs.
    const auto run_step = [&](int m, const In &cur, In &nxt) {
        const int64_t t = t_hi - m;
        const int r0 = (int)(t % kAdjNearRows);  // this step's row of the near ring
        R A[9];
        if (own) {
            // push: sigma_bar^t = Dy^T fbar(t+1), nbar(t) = push map of dbar(t+1)
            R sb = R(0);
            for (int yy = max(0, y - 2); yy <= min(ly - 1, y + 2); ++yy)
                sb += coef_div<R>(yy, y, ly) * s_fbar[yy];
            s_near[r0][y] = sb;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int yt = y + QY[q];
                A[q] = (yt >= 0 && yt < ly) ? s_dbar[q][yt] : s_dbar[QOPP[q]][y];
            }
            const double s = (double)cur.s;
            const double q = exp(-(c->inv_tau + c->inv_gc * fabs(s)));
            double S0, S1;
            adj_near_sum(jn, H, q,
                         [&](int j) { return (double)s_near[(r0 + j) & (kAdjNearRows - 1)][y]; },
                         S0, S1);
            S0 += cur.b0;
            S1 += cur.b1;
            s_S0[y] = S0;
            s_S1[y] = S1;
            s_s[y] = s;
            s_sbar[y] = c->g_inf * (S0 - fabs(s) * S1 * c->inv_gc);
        }
        __syncthreads();  // every node's sbar_t is in LDS; every push has read dbar, fbar
        if (own) {
            // unconditional (the last step reloads its own inputs), so the
            // loads of every step stay in one sequence for the wait counters
            load(min(m + 1, count - 1), nxt);
            adj_lattice_core<R>(c, y, cur.rec, A,
                                [&](int yy, double &S0, double &S1, double &ss) {
                                    S0 = s_S0[yy];
                                    S1 = s_S1[yy];
                                    ss = s_s[yy];
                                    return s_sbar[yy];
                                },
                                [&](int k, double v) { acc[k] += v; },
                                [&](int q, R v) {
                                    if (q < 9)
                                        s_dbar[q][y] = v;
                                    else
                                        s_fbar[y] = v;
                                });
        }
        __syncthreads();  // dbar(t), fbar(t) in LDS before the next push reads them
    };
    In in0, in1;
    if (own)
        load(0, in0);
    __syncthreads();
    // two steps per trip, so that the inputs in flight stay in their registers
    for (int m = 0; m < count; m += 2) {
        run_step(m, in0, in1);
        if (m + 1 < count)
            run_step(m + 1, in1, in0);
    }
    if (own) {
        for (int m = 0; m < count; ++m) {
            const int64_t t = t_hi - m;
            sring[(size_t)(t % H) * np + y] = s_near[t % kAdjNearRows][y];
        }
        g_fbar[y] = s_fbar[y];
#pragma unroll
        for (int q = 0; q < 9; ++q)
            g_dbar[q * np + y] = s_dbar[q][y];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            g_acc[k * np + y] = acc[k];
    }
}

// Sum the per-node parameter gradients of every channel in node order.
__global__ void k_adj_reduce(const ChanDev *__restrict__ chans, int n_ch,
                             const char *__restrict__ aws, const AdjChan *__restrict__ achans,
                             double *__restrict__ out)
{
    const int ch = blockIdx.x;
    if (ch >= n_ch || threadIdx.x >= 4)
        return;
    const ChanDev *c = chans + ch;
    const double *acc = reinterpret_cast<const double *>(aws + achans[ch].off_acc) +
                        (size_t)threadIdx.x * c->np;
    double sum = 0.0;
    for (int n = 0; n < c->n; ++n)
        sum += acc[n];
    out[ch * 4 + threadIdx.x] = sum;
}

__global__ void k_set_params(ChanDev *chans, int ch, double g_inf, double tau_m, double gamma_c)
{
    if (threadIdx.x == 0) {
        ChanDev *c = chans + ch;
        c->g_inf = g_inf;
        c->inv_tau = 1.0 / tau_m;
        c->inv_gc = isinf(gamma_c) ? 0.0 : 1.0 / gamma_c;
        c->l2_tau = 1.4426950408889634 * c->inv_tau;
        c->l2_gc = 1.4426950408889634 * c->inv_gc;
    }
}

void launch_adj_a(int prec, const ChanDev *chans, const NodeTile *tiles, int n_tiles, char *aws,
                  const AdjChan *achans, const int64_t *t0, int slot, int buf, hipStream_t st)
{
    // workgroups of kAdjNodes nodes x kAdjChunks age ranges: kBlock / kAdjNodes node
    // groups per node tile, kAdjGroups parts of the window per node group
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_adj_a<P, H>),
                                           dim3(n_tiles * (kBlock / kAdjNodes) * kAdjGroups),
                                           dim3(kAdjNodes * kAdjChunks), 0, st, chans, tiles,
                                           aws, achans, t0, slot, buf));
}

void launch_adj_b(int prec, const ChanDev *chans, const NodeTile *tiles, int n_tiles, char *aws,
                  const AdjChan *achans, const int64_t *t0, int slot, int buf, hipStream_t st)
{
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_adj_b<P, H>), dim3(n_tiles), dim3(kBlock), 0, st,
                                           chans, tiles, aws, achans, t0, slot, buf));
}

void launch_adj_bulk(int prec, const ChanDev *chans, const NodeTile *tiles, int n_tiles,
                     char *aws, const AdjChan *achans, const int64_t *t0, int slot_hi,
                     int count, int buf, hipStream_t st)
{
    // node tiles x groups of kAdjBulkNodes nodes x entries of the block
    LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_adj_bulk<P, H>),
                                           dim3(n_tiles * (kBlock / kAdjBulkNodes) * count),
                                           dim3(kBlock), 0, st, chans, tiles, n_tiles, aws,
                                           achans, t0, slot_hi, count, buf));
}

void launch_adj_span(int prec, const ChanDev *chans, int n_ch, int max_ly, char *aws,
                     const AdjChan *achans, const int64_t *t0, int slot_hi, int count,
                     int buf, hipStream_t st)
{
    if (max_ly <= kAdjSpanLdsNodes)
        LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_adj_span_lds<P, H>), dim3(n_ch),
                                               dim3(kAdjSpanLdsNodes), 0, st, chans, aws,
                                               achans, t0, slot_hi, count, buf));
    else
        LBMAX_BY_PREC(prec, hipLaunchKernelGGL((k_adj_span<P, H>), dim3(n_ch),
                                               dim3(kAdjSpanThreads), 0, st, chans, aws, achans,
                                               t0, slot_hi, count, buf));
}

__global__ void k_store_i64(int64_t *p, int64_t v)
{
    if (threadIdx.x == 0)
        p[0] = v;
}

void launch_store_i64(int64_t *p, int64_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_store_i64, dim3(1), dim3(64), 0, st, p, v);
}

// Step records on (aws: each channel's record area of buffer buf, from step
// t0) or off (aws = nullptr) in the device channel table.
__global__ void k_set_record(ChanDev *chans, const AdjChan *achans, int n_ch, char *aws, int buf,
                             int64_t t0)
{
    const int ci = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (ci >= n_ch)
        return;
    chans[ci].rec = aws ? (int64_t)(uintptr_t)(aws + achans[ci].off_rec[buf]) : 0;
    chans[ci].rec_t0 = aws ? t0 : 0;
}

void launch_set_record(ChanDev *chans, const AdjChan *achans, int n_ch, char *aws, int buf,
                       int64_t t0, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_record, dim3((n_ch + 63) / 64), dim3(64), 0, st, chans, achans,
                       n_ch, aws, buf, t0);
}

void launch_adj_reduce(const ChanDev *chans, int n_ch, char *aws, const AdjChan *achans,
                       double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_reduce, dim3(n_ch), dim3(64), 0, st, chans, n_ch, aws, achans,
                       out);
}

void launch_set_params(ChanDev *chans, int ch, double g_inf, double tau_m, double gamma_c,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_set_params, dim3(1), dim3(64), 0, st, chans, ch, g_inf, tau_m,
                       gamma_c);
}

}  // namespace lbmax
