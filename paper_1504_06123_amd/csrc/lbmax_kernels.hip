// lbmax_kernels.hip -- gfx950 kernels of the hybrid lattice-Boltzmann step
// with the integral nonlinear Maxwell stress (arXiv:1504.06123).
//
// One time step t is two grid-wide phases plus an optional combine:
//   k_lb      pull-stream + bounce-back, moments, force rho*g + div sigma^{t-1},
//             half-force velocity, BGK collision with the forcing term
//             (Sec. III: collision-streaming rule, Eqs. bodyforce, hydrofields)
//   k_hist    velocity gradient, push of the shear history entry, and the
//             history integral of Eq. (gitt) with the modulus of Eq. (nlmax)
//             over the window of the last n_hist steps -> sigma^t
//   k_combine FP64 affine combination of per-chunk partial sums when a
//             channel's window is split across workgroups.
//
// Data layout (per channel, all planes [np] with node = y*lx + x):
//   populations: two buffers (step parity) x 9 planes of n_i - a_i
//   history ring: row-major [n_hist][np]; row t' mod n_hist holds the entry
//   of step t'.  A wavefront reads one row per age: 64 consecutive nodes,
//   fully coalesced, streaming through HBM once per step.  Ages are walked
//   newest to oldest, so the accumulated strain gamma_{t,t'} is a running
//   FP64 sum of the shear rate over the window (Sec. III Eq. eeval with the
//   simple-shear reduction of the Finger tensor) and no strain prefix has to
//   be stored.
#include "lbmax_internal.h"

#include <hip/hip_runtime.h>

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

// ---------------------------------------------------------------------------
// Compensated accumulation.  FP32 sums use Kahan's compensation; FP64 sums
// are plain.  value() returns the compensated sum in FP64.
// ---------------------------------------------------------------------------
template <typename R>
struct Acc {
    R s = R(0);
    __device__ __forceinline__ void add(R x) { s += x; }
    __device__ __forceinline__ double value() const { return (double)s; }
};

template <>
struct Acc<float> {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x)
    {
        float y = x - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const
    {
        return (double)s - (double)c;
    }
};

// Memory decay exp(-k (1/tau + r/gamma_c)) of Eq. (nlmax).  FP32: hardware
// exp2 with the log2(e)-scaled rates; FP64: libm-grade exp.
template <typename R>
struct Decay;

template <>
struct Decay<float> {
    float a, b;  // log2(e)/tau, log2(e)/gamma_c
    __device__ __forceinline__ explicit Decay(const ChanDev *c)
        : a((float)c->l2_tau), b((float)c->l2_gc) {}
    __device__ __forceinline__ float operator()(float k, float r) const
    {
        return __builtin_amdgcn_exp2f(-k * __builtin_fmaf(b, r, a));
    }
};

template <>
struct Decay<double> {
    double a, b;  // 1/tau, 1/gamma_c
    __device__ __forceinline__ explicit Decay(const ChanDev *c)
        : a(c->inv_tau), b(c->inv_gc) {}
    __device__ __forceinline__ double operator()(double k, double r) const
    {
        return exp(-k * (a + b * r));
    }
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
// zero stress / moments.  One channel per launch.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_init(char *__restrict__ ws,
                                                 const ChanDev *__restrict__ chans,
                                                 int ch,
                                                 const double *__restrict__ u0)
{
    const ChanDev *c = chans + ch;
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= c->n)
        return;
    const int lx = c->lx, ly = c->ly, np = c->np, N = c->n;
    const int y = n / lx, x = n - y * lx;
    R *pop = reinterpret_cast<R *>(ws + c->off_pop);
    R *read0 = pop + 9 * (size_t)np;  // buffer pulled from at t = 0
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
        read0[q * (size_t)np + n] = (R)dev;
        pop[q * (size_t)np + n] = R(0);
    }
    R *sig = reinterpret_cast<R *>(ws + c->off_sig);
    R *vel = reinterpret_cast<R *>(ws + c->off_vel);
    R *rho = reinterpret_cast<R *>(ws + c->off_rho);
    sig[n] = R(0);
    sig[np + n] = R(0);
    vel[n] = R(0);
    vel[np + n] = R(0);
    rho[n] = R(0);
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
// Lattice phase of step t.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_lb(char *__restrict__ ws,
                                               const ChanDev *__restrict__ chans,
                                               const NodeTile *__restrict__ tiles,
                                               const int64_t *__restrict__ tcount,
                                               int trel)
{
    const NodeTile tl = tiles[blockIdx.x];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    if (n >= c->n)
        return;
    const int lx = c->lx, ly = c->ly;
    const size_t np = (size_t)c->np;
    const int64_t t = *tcount + trel;
    R *pop = reinterpret_cast<R *>(ws + c->off_pop);
    const R *__restrict__ src = pop + ((t + 1) & 1) * 9 * np;  // n*(t-1)
    R *__restrict__ dst = pop + (t & 1) * 9 * np;              // n*(t)
    const int y = n / lx, x = n - y * lx;
    const int xp = (x + 1 == lx) ? 0 : x + 1;
    const int xm = (x == 0) ? lx - 1 : x - 1;
    const bool lo = y > 0, hi = y < ly - 1;
    const int rowm = (y - 1) * lx, row = y * lx, rowp = (y + 1) * lx;

    // Pull-stream: n_q(x, y) = n*_q(x - c_q); through a wall, the population
    // that left in the opposite direction comes back (halfway bounce-back).
    R d[9];
    d[0] = src[n];
    d[1] = src[1 * np + row + xm];
    d[2] = src[2 * np + row + xp];
    d[3] = lo ? src[3 * np + rowm + x] : src[4 * np + n];
    d[4] = hi ? src[4 * np + rowp + x] : src[3 * np + n];
    d[5] = lo ? src[5 * np + rowm + xm] : src[6 * np + n];
    d[6] = hi ? src[6 * np + rowp + xp] : src[5 * np + n];
    d[7] = hi ? src[7 * np + rowp + xm] : src[8 * np + n];
    d[8] = lo ? src[8 * np + rowm + xp] : src[7 * np + n];

    // Moments of the deviations n_q - a_q: rho - 1 and j.
    const R drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const R jx = (d[1] - d[2]) + (d[5] - d[6]) + (d[7] - d[8]);
    const R jy = (d[3] - d[4]) + (d[5] - d[6]) + (d[8] - d[7]);
    const R rho = R(1) + drho;

    // Force density rho*g + div sigma^{t-1} (sigma_yy = 0 in simple shear);
    // d/dx periodic central, d/dy central with one-sided rows at the walls.
    const R *__restrict__ sxy = reinterpret_cast<const R *>(ws + c->off_sig);
    const R *__restrict__ sxx = sxy + np;
    R dys;
    if (y == 0)
        dys = R(0.5) * (R(-3) * sxy[n] + R(4) * sxy[n + lx] - sxy[n + 2 * lx]);
    else if (y == ly - 1)
        dys = R(0.5) * (R(3) * sxy[n] - R(4) * sxy[n - lx] + sxy[n - 2 * lx]);
    else
        dys = R(0.5) * (sxy[n + lx] - sxy[n - lx]);
    R fx = R(0.5) * (sxx[row + xp] - sxx[row + xm]) + dys;
    R fy = R(0.5) * (sxy[row + xp] - sxy[row + xm]);
    fx += rho * (R)c->gx;
    fy += rho * (R)c->gy;

    // Velocity with the half-force shift (Eq. hydrofields).
    const R ux = (jx + R(0.5) * fx) / rho;
    const R uy = (jy + R(0.5) * fy) / rho;

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
        dst[q * np + n] = d[q] - om * (d[q] - deq) + F;
    }
    R *vel = reinterpret_cast<R *>(ws + c->off_vel);
    vel[n] = ux;
    vel[np + n] = uy;
    reinterpret_cast<R *>(ws + c->off_rho)[n] = drho;
}

// ---------------------------------------------------------------------------
// History integral.
//
// A workgroup owns kBlock*V consecutive nodes of one channel and one age
// range [k0, k1) of their window; lane l owns nodes n0 + V*l .. n0 + V*l + V-1
// and reads them as one V-wide vector per ring row.  Ages are walked newest
// to oldest; U rows are loaded before any is used so each wavefront keeps U
// (2U with |gamma_dot|) vector reads in flight.  Row addresses are uniform
// across the workgroup, so a load is a scalar row base plus the lane's
// 32-bit node offset.
//   A += w s E,  B += w 2 s gamma E,  gamma = FP64 running strain (loc),
// w = 1 inside the window; the end weights 1/2 are applied by the caller's
// peeled first (age 0) and last (age n_hist-1) entries.
// ---------------------------------------------------------------------------
template <typename R, int V>
struct alignas(sizeof(R) * V) Pack {
    R v[V];
};

// row: uniform row base; off: the lane's byte offset within the row (32-bit,
// so the load is a scalar base plus an unsigned vector offset).
template <typename R, int V>
__device__ __forceinline__ Pack<R, V> load_pack(const R *row, uint32_t off)
{
    return *reinterpret_cast<const Pack<R, V> *>(reinterpret_cast<const char *>(row) + off);
}

template <typename R>
__device__ __forceinline__ void accumulate(R s, R r, R k, const Decay<R> &dec,
                                           Acc<R> &A, Acc<R> &B, double &loc)
{
    loc += (double)s;
    const R se = s * dec(k, r);
    A.add(se);
    B.add(R(2) * se * (R)loc);
}

template <typename R, int V, int U, bool HAS_R>
__device__ __forceinline__ void hist_range(const R *__restrict__ ring_s,
                                           const R *__restrict__ ring_r,
                                           size_t np, uint32_t lane_off, int H, int p,
                                           int k0, int k1, const Decay<R> &dec,
                                           Acc<R> (&A)[V], Acc<R> (&B)[V],
                                           double (&loc)[V])
{
    int k = k0;
    int slot = p - k;
    if (slot < 0)
        slot += H;
    while (k < k1) {
        // contiguous run of rows going down without wrapping
        const int run = min(k1 - k, slot + 1);
        int j = 0;
        for (; j + U <= run; j += U) {
            Pack<R, V> sv[U], rv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t row = (size_t)(slot - j - u) * np;
                sv[u] = load_pack<R, V>(ring_s + row, lane_off);
                if (HAS_R)
                    rv[u] = load_pack<R, V>(ring_r + row, lane_off);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const R kf = R(k + j + u);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const R s = sv[u].v[v];
                    accumulate<R>(s, HAS_R ? rv[u].v[v] : fabs(s), kf, dec, A[v], B[v],
                                  loc[v]);
                }
            }
        }
        for (; j < run; ++j) {
            const size_t row = (size_t)(slot - j) * np;
            const Pack<R, V> sv = load_pack<R, V>(ring_s + row, lane_off);
            Pack<R, V> rv;
            if (HAS_R)
                rv = load_pack<R, V>(ring_r + row, lane_off);
            const R kf = R(k + j);
#pragma unroll
            for (int v = 0; v < V; ++v)
                accumulate<R>(sv.v[v], HAS_R ? rv.v[v] : fabs(sv.v[v]), kf, dec, A[v],
                              B[v], loc[v]);
        }
        k += run;
        slot = H - 1;
    }
}

template <typename R, int V, int U, bool HAS_R>
__device__ __forceinline__ void hist_tile(char *__restrict__ ws, const ChanDev *c,
                                          const HistTile &tl, int64_t t)
{
    const int H = c->n_hist;
    const size_t np = (size_t)c->np;
    const int first = tl.n0 + (int)threadIdx.x * V;  // lane's first node
    // A lane past the channel end shadows the last vector of the channel (in
    // bounds, results discarded); nodes past the end inside a vector read the
    // zero padding of the ring.
    const int lane_node = first < c->n ? first : ((c->n - 1) / V) * V;
    const uint32_t lane_off = (uint32_t)lane_node * (uint32_t)sizeof(R);
    const int p = (int)(t % H);
    R *ring_s = reinterpret_cast<R *>(ws + c->off_ring_s);
    R *ring_r = reinterpret_cast<R *>(ws + c->off_ring_r);
    const Decay<R> dec(c);
    Acc<R> A[V], B[V];
    double loc[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
        loc[v] = 0.0;
    int k = tl.k0;
    if (k == 0) {
        // Newest entry, age 0: gradient of this step's velocity, push it, and
        // add it with the trapezoid weight 1/2 (E = 1, gamma = 0).
        const R *vel = reinterpret_cast<const R *>(ws + c->off_vel);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int node = first + v;
            R s = R(0);
            if (node < c->n) {
                const int y = node / c->lx, x = node - y * c->lx;
                R kxx, kxy, kyx, kyy;
                velocity_gradient<R>(vel, vel + np, c->lx, c->ly, x, y, kxx, kxy, kyx,
                                     kyy);
                s = kxy;
                ring_s[(size_t)p * np + node] = s;
                if (HAS_R)
                    ring_r[(size_t)p * np + node] = shear_rate<R>(kxx, kxy, kyx, kyy);
            }
            A[v].add(R(0.5) * s);
        }
        k = 1;
    }
    const bool oldest = tl.k1 == H;
    hist_range<R, V, U, HAS_R>(ring_s, ring_r, np, lane_off, H, p, k,
                               oldest ? H - 1 : tl.k1, dec, A, B, loc);
    if (oldest) {
        // Oldest entry, age H-1, trapezoid weight 1/2.
        int slot = p + 1;
        if (slot >= H)
            slot -= H;
        const size_t row = (size_t)slot * np;
        const Pack<R, V> sv = load_pack<R, V>(ring_s + row, lane_off);
        Pack<R, V> rv;
        if (HAS_R)
            rv = load_pack<R, V>(ring_r + row, lane_off);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R s = sv.v[v];
            loc[v] += (double)s;
            const R se = R(0.5) * s * dec(R(H - 1), HAS_R ? rv.v[v] : fabs(s));
            A[v].add(se);
            B[v].add(R(2) * se * (R)loc[v]);
        }
    }
    if (first >= c->n)
        return;
    R *sig = reinterpret_cast<R *>(ws + c->off_sig);
    double *part = reinterpret_cast<double *>(ws + c->off_part);
    const size_t plane = (size_t)c->max_chunks * np;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int node = first + v;
        if (node >= c->n)
            break;
        if (c->nchunks == 1) {
            sig[node] = (R)(c->g_inf * A[v].value());
            sig[np + node] = (R)(c->g_inf * B[v].value());
        } else {
            const size_t at = (size_t)tl.chunk * np + node;
            part[at] = A[v].value();
            part[plane + at] = B[v].value();
            part[2 * plane + at] = loc[v];
        }
    }
}

// One launch per lane width V: the tiles of channels with c->vec == V.
template <typename R, int V, int U>
__global__ __launch_bounds__(kBlock) void k_hist(char *__restrict__ ws,
                                                 const ChanDev *__restrict__ chans,
                                                 const HistTile *__restrict__ tiles,
                                                 const int64_t *__restrict__ tcount,
                                                 int trel)
{
    const HistTile tl = tiles[blockIdx.x];
    const ChanDev *c = chans + tl.ch;
    // A wavefront whose nodes all lie past the channel has nothing to do.
    if (tl.n0 + (int)(threadIdx.x & ~63u) * V >= c->n)
        return;
    const int64_t t = *tcount + trel;
    if (c->has_r)
        hist_tile<R, V, U, true>(ws, c, tl, t);
    else
        hist_tile<R, V, U, false>(ws, c, tl, t);
}

// ---------------------------------------------------------------------------
// FP64 combine of the per-chunk partials of a split window, newest chunk
// first: sigma_xy = G sum_c A_c, sigma_xx = G sum_c (2 O_c A_c + B_c), where
// O_c = sum of the strain totals T of the newer chunks (the accumulated
// strain at the chunk's start).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_combine(char *__restrict__ ws,
                                                    const ChanDev *__restrict__ chans,
                                                    const NodeTile *__restrict__ tiles)
{
    const NodeTile tl = tiles[blockIdx.x];
    const ChanDev *c = chans + tl.ch;
    const int n = tl.n0 + threadIdx.x;
    if (c->nchunks == 1 || n >= c->n)
        return;
    const size_t np = (size_t)c->np;
    const size_t plane = (size_t)c->max_chunks * np;
    const double *part = reinterpret_cast<const double *>(ws + c->off_part);
    double O = 0.0, sxy = 0.0, sxx = 0.0;
    for (int k = 0; k < c->nchunks; ++k) {
        const double A = part[k * np + n];
        const double B = part[plane + k * np + n];
        const double T = part[2 * plane + k * np + n];
        sxy += A;
        sxx += 2.0 * O * A + B;
        O += T;
    }
    R *sig = reinterpret_cast<R *>(ws + c->off_sig);
    sig[n] = (R)(c->g_inf * sxy);
    sig[np + n] = (R)(c->g_inf * sxx);
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
        out[N + n] = (double)sig[np + n];  // N1 = sigma_xx - sigma_yy, sigma_yy = 0
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

void launch_init(bool f64, char *ws, const ChanDev *chans, int ch,
                 const NodeTile *, int n_tiles, const double *u0_dev,
                 hipStream_t st)
{
    if (f64)
        hipLaunchKernelGGL(k_init<double>, dim3(n_tiles), dim3(kBlock), 0, st, ws,
                           chans, ch, u0_dev);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(n_tiles), dim3(kBlock), 0, st, ws,
                           chans, ch, u0_dev);
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

void launch_lb(bool f64, char *ws, const ChanDev *chans, const NodeTile *tiles,
               int n_tiles, const int64_t *tcount, int trel, hipStream_t st)
{
    if (f64)
        hipLaunchKernelGGL(k_lb<double>, dim3(n_tiles), dim3(kBlock), 0, st, ws,
                           chans, tiles, tcount, trel);
    else
        hipLaunchKernelGGL(k_lb<float>, dim3(n_tiles), dim3(kBlock), 0, st, ws,
                           chans, tiles, tcount, trel);
}

void launch_hist(bool f64, int vec, char *ws, const ChanDev *chans,
                 const HistTile *tiles, int n_tiles, const int64_t *tcount, int trel,
                 hipStream_t st)
{
    if (n_tiles <= 0)
        return;
#define LBMAX_HIST(R, V, U)                                                     \
    hipLaunchKernelGGL((k_hist<R, V, U>), dim3(n_tiles), dim3(kBlock), 0, st, ws, \
                       chans, tiles, tcount, trel)
    if (f64) {
        if (vec == 4)
            LBMAX_HIST(double, 4, 4);
        else if (vec == 2)
            LBMAX_HIST(double, 2, 8);
        else
            LBMAX_HIST(double, 1, 8);
    } else {
        if (vec == 4)
            LBMAX_HIST(float, 4, 4);
        else if (vec == 2)
            LBMAX_HIST(float, 2, 8);
        else
            LBMAX_HIST(float, 1, 8);
    }
#undef LBMAX_HIST
}

void launch_combine(bool f64, char *ws, const ChanDev *chans, const NodeTile *tiles,
                    int n_tiles, hipStream_t st)
{
    if (f64)
        hipLaunchKernelGGL(k_combine<double>, dim3(n_tiles), dim3(kBlock), 0, st,
                           ws, chans, tiles);
    else
        hipLaunchKernelGGL(k_combine<float>, dim3(n_tiles), dim3(kBlock), 0, st,
                           ws, chans, tiles);
}

void launch_tick(int64_t *tcount, int64_t add, hipStream_t st)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, tcount, add);
}

void launch_set_force(ChanDev *chans, int ch, double gx, double gy, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_force, dim3(1), dim3(64), 0, st, chans, ch, gx, gy);
}

void launch_readout(bool f64, int which, char *ws, const ChanDev *chans, int ch,
                    int n_nodes, double *stage, hipStream_t st)
{
    if (f64)
        hipLaunchKernelGGL(k_readout<double>, dim3(blocks_for(n_nodes)), dim3(kBlock),
                           0, st, which, ws, chans, ch, stage);
    else
        hipLaunchKernelGGL(k_readout<float>, dim3(blocks_for(n_nodes)), dim3(kBlock),
                           0, st, which, ws, chans, ch, stage);
}

}  // namespace lbmax
