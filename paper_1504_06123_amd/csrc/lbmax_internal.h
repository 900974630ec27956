// lbmax_internal.h -- device-side data layout shared by the kernels and the
// host runtime of liblbmax.  Not part of the public interface (include/lbmax.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmax {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kWave = 64;          // threads per wavefront
constexpr int kFuseThreads = 1024; // workgroup of the fused in-block steps
constexpr int kFuseMaxNodes = 1024; // channels up to this size take them
// Widest channel for which the default takes the global-memory fused form
// (not the LDS one): FP64 populations, 1 x N channels, N_h 2048, 32-step
// blocks measured 9.0 against 10.2 us per step unfused at 512 nodes, 11.8
// against 10.4 at 1024.
constexpr int kFuseGlobalMaxNodes = 512;
constexpr int kNodeAlign = 64;     // node-plane stride is a multiple of this
constexpr int kMinChunkLen = 128;  // shortest age range of one history chunk
constexpr int kMaxChunks = 64;     // most age ranges per channel
constexpr int64_t kPartialBudget = int64_t(1) << 20;  // chunks * stride cap
constexpr int kMaxBlock = 32;      // most steps served by one history pass
// Planes of the per-chunk partials and of the block sums (doubles, [plane][np]
// per chunk): A_m at m, B_m at kMaxBlock + m, chunk strain total at kPlaneT.
constexpr int kPlaneB = kMaxBlock;
constexpr int kPlaneT = 2 * kMaxBlock;
constexpr int kPartPlanes = 2 * kMaxBlock + 1;
// Block planes of a channel on the quasi-logarithmic grid: A_m, B_m as
// above, then the interior strain of each grid block at kPlaneGrid + bi.
constexpr int kPlaneGrid = 2 * kMaxBlock;
// Most steps served by one pass over a grid channel (longer blocks of the
// other channels are served in sub-blocks of this length).
constexpr int kMaxGridBlock = 16;
constexpr int kTileCounters = 8;   // persistent-pass tile counters (one per tile group)
// Full tensor: S_xx, S_xy, S_yy per step of the block, then the range's
// total deformation (4 planes).
constexpr int kFingerPartPlanes = 3 * kMaxBlock + 4;
constexpr int kMaxFingerBlock = 16;

// Per-channel parameters and workspace offsets, read by every kernel.
// 256 bytes so a table row never straddles two scalar cache lines twice.
struct alignas(256) ChanDev {
    int32_t lx, ly, n, np;          // nodes n = lx*ly, plane stride np
    int32_t n_hist, has_r, nchunks, max_chunks;
    int32_t vec;                    // history kernel: nodes per lane (1, 2, 4)
    int32_t qb, qc;                 // quasi-logarithmic grid: blocks B, entries C (qb = 0: none)
    int32_t finger;                 // 1: full Finger tensor (8-plane ring: kappa, g; sigma_yy)
    int32_t coupling;               // 0: body force div sigma; 1: the paper's forcing term
    int32_t law;                    // 0: Eq. nlmax; 1: accumulated-strain damping; 2: Eq. inlM
    double omega;                   // 1/tau_LB
    double g_inf;
    double inv_tau, inv_gc;         // 1/tau, 1/gamma_c (0 for gamma_c = inf)
    double l2_tau, l2_gc;           // log2(e)/tau, log2(e)/gamma_c
    double gx, gy;                  // body-force acceleration
    int64_t off_pop;                // [2][9][np] populations minus a_i (split storage:
                                    // FP32 remainders n*_i - n^eq_i of the moments below)
    int64_t off_mom;                // [2][3][np] FP64 rho - 1, u_x, u_y by step parity
                                    // (split storage only; 0 otherwise)
    int64_t off_sig;                // [3][np]  sigma_xy, sigma_xx, sigma_yy
    int64_t off_vel;                // [2][np]  u_x, u_y
    int64_t off_rho;                // [np]     rho - 1
    int64_t off_ring_s;             // [n_hist][np] shear rate ([8][n_hist][np] full tensor)
    int64_t off_ring_r;             // [n_hist][np] |gamma_dot| (has_r only)
    int64_t off_part;               // [kPartPlanes or kFingerPartPlanes][max_chunks][np] doubles
    int64_t off_blk;                // [2 or 3 * kMaxBlock (+ qb)][np] doubles: block sums
    int64_t off_grid_s;             // [qb][qc][np] averaged shear rate of each grid entry
    int64_t off_grid_r;             // [qb][qc][np] |gamma_dot| of the averaged gradient (has_r)
    int64_t off_grid_d;             // [3][qb][qc][np] averaged D components (has_r)
    int64_t off_trace;              // [np] tr sigma two steps back (paper coupling)
    // Adjoint replay: while rec != 0 (a device address), the lattice step t
    // also records its input populations n*(t-1) and sigma_xy^{t-1} of each
    // node at rec + (t - rec_t0) * 10 * np elements (the layout of the
    // adjoint's step record).
    int64_t rec;
    int64_t rec_t0;
};
static_assert(sizeof(ChanDev) == 256, "ChanDev layout");

// One workgroup of the lattice / combine / readout kernels: 256 nodes.
struct NodeTile {
    int32_t ch, n0;
};

// One unit of history work: nodes [n0, n0 + span) x ages [k0, k1), span =
// 64*vec for the simple-shear pass (one wavefront per tile, four tiles per
// workgroup), 256 for the full-tensor and accumulated-strain passes (one
// workgroup per tile).
struct HistTile {
    int32_t ch, n0, k0, k1, chunk, pad;
};

// Kernel launchers (lbmax_kernels.hip).  All launches go on `st`.  `prec`:
// 0 = FP64 lattice and history, 1 = split population storage (FP32 remainders
// with FP64 moments) with FP32 history, 2 = FP64 lattice (populations,
// moments, stress planes) with FP32 history (ring and window sums).  Stress,
// velocity and density planes are FP64 in every mode.
// `tcount` is the device step counter; a kernel works on step
// t = *tcount + trel.
void launch_init(int prec, char *ws, const ChanDev *chans, int ch,
                 const NodeTile *tiles, int n_tiles, const double *u0_dev,
                 hipStream_t st);
void launch_fill_zero(void *p, size_t bytes, hipStream_t st);
// The lattice kernel also zeroes the persistent-pass tile counters.
void launch_lb(int prec, char *ws, const ChanDev *chans, const NodeTile *tiles,
               int n_tiles, const int64_t *tcount, int trel, int *tile_counters,
               hipStream_t st);
// History pass (first step of a block of `block` steps) for the tiles of the
// channels whose lane width is `vec`.  persistent_grid > 0 launches that many
// persistent workgroups claiming tiles from *counter.
void launch_hist_pass(int prec, int vec, int block, char *ws, const ChanDev *chans,
                      const HistTile *tiles, int n_tiles, const int64_t *tcount,
                      int trel, int persistent_grid, int *counter, hipStream_t st);
int hist_pass_blocks_per_cu(int prec, int vec, int block);
// Full-tensor pass for the tiles of the full-tensor channels (block <= 16).
void launch_finger_pass(int prec, int block, char *ws, const ChanDev *chans,
                        const HistTile *tiles, int n_tiles, const int64_t *tcount, int trel,
                        int persistent_grid, int *counter, hipStream_t st);
int finger_pass_blocks_per_cu(int prec, int block);
// Accumulated-strain damping: one pass per block, O(1) work per entry.
void launch_wm_pass(int prec, int block, char *ws, const ChanDev *chans, const HistTile *tiles,
                    int n_tiles, const int64_t *tcount, int trel, hipStream_t st);
// Instantaneous law (Eq. inlM), every step, node-local (other channels return).
void launch_inst_step(int prec, char *ws, const ChanDev *chans, const NodeTile *tiles,
                      int n_tiles, const int64_t *tcount, int trel, hipStream_t st);
// FP64 combine of chunk partials into sigma and the block sums.
void launch_combine(int prec, int block, char *ws, const ChanDev *chans,
                    const NodeTile *tiles, int n_tiles, hipStream_t st);
// Step m (1 <= m < block) of a block: gradient, push, sigma from the block sums.
void launch_hist_step(int prec, int m, char *ws, const ChanDev *chans,
                      const NodeTile *tiles, int n_tiles, const int64_t *tcount,
                      int trel, hipStream_t st);
// Quasi-logarithmic grid channels, every step: gradient, push, combination of
// full blocks, history integral -> sigma (other channels' tiles return).
// With blocks of block > 1 steps, step m = 0 of a block also forms the
// interior sums of the block and steps m > 0 visit only the other entries.
void launch_grid_step(int prec, int block, int m, char *ws, const ChanDev *chans,
                      const NodeTile *tiles, int n_tiles, const int64_t *tcount, int trel,
                      hipStream_t st);
// Steps m0 .. m0 + count - 1 of a block, after its pass, for handles whose
// channels all fit one workgroup (window histories, n <= kFuseMaxNodes): one
// workgroup per channel runs the lattice and in-block history phases of
// every step.
// With `lds`, the form that keeps each channel's lattice state in LDS and
// the rows pushed since the pass in registers (FP32 handles whose channels
// take the simple-shear integral law and the body-force coupling); it needs
// fused_lds_bytes(prec) of dynamic LDS, allowed by prepare_fused_lds (0 on
// success, -1 for the other precisions).
void launch_fused_steps(int prec, bool lds, char *ws, const ChanDev *chans, int n_ch,
                        const int64_t *tcount, int trel, int m0, int count, hipStream_t st);
size_t fused_lds_bytes(int prec);
int prepare_fused_lds(int prec);
void launch_tick(int64_t *tcount, int64_t add, hipStream_t st);
void launch_set_force(ChanDev *chans, int ch, double gx, double gy,
                      hipStream_t st);
// Readouts into FP64 staging (nodes of one channel): which = 0 fields
// (rho, ux, uy), 1 stress (sxy, n1), 2 gradient (kxx, kxy, kyx, kyy).
void launch_readout(int prec, int which, char *ws, const ChanDev *chans,
                    int ch, int n_nodes, double *stage, hipStream_t st);

}  // namespace lbmax

namespace lbmax {

// Adjoint workspace of one channel (byte offsets into the adjoint workspace).
// Workgroups over the age window per group of nodes in the adjoint's
// history transpose.
constexpr int kAdjGroups = 8;
// Most reverse steps one blocked launch pair (k_adj_bulk, k_adj_span) takes,
// and the fixed age ranges the bulk pass splits each entry's window into.
constexpr int kAdjMaxBlock = 32;
constexpr int kAdjBulkRanges = 16;
// Widest channel the blocked sweep takes: its span workgroup loops over a
// channel's nodes with 256 threads, and from three nodes a thread on (more
// than 512 nodes) the per-step kernels, which give every node its own
// threads, are faster (measured: 1.02x at 512 nodes, 0.81x at 768, 0.66x at
// 1024).
constexpr int kAdjBlockedMaxNodes = 512;

// The step records, loss gradients and recorded shear rates come in two
// buffers (by segment parity), so the replay of one segment can fill one
// while the reverse sweep of the next-later segment reads the other.
struct alignas(128) AdjChan {
    int64_t off_sbar_ring;  // [n_hist][np] R  adjoint of sigma_xy, row t mod n_hist
    int64_t off_nbar;       // [9][np] R  adjoint of the post-collision populations
    int64_t off_dbar;       // [9][np] R  adjoint of the pulled populations
    int64_t off_fbar;       // [np] R     adjoint of the force f_x
    int64_t off_part;       // [kAdjGroups][2][np] double  history-transpose partial sums
    int64_t off_acc;        // [4][np] double  per-node parameter gradients
    int64_t off_rec[2];     // [seg_len][10][np] R  n*(t-1) (9 planes), sigma_xy^{t-1}
    int64_t off_dldu[2];    // [seg_len][np] double  dL/du_x of each step
    int64_t off_recs[2];    // [seg_len][np] RH  shear rate s_t pushed at each step
    int64_t off_bulk;       // [kAdjMaxBlock][2][np] double  far sums of a reverse block
};

// The adjoint kernels of step t = *t0 + slot (t0 in device memory, so one
// captured sweep serves every segment of the same length) on record buffer
// buf.  They read the forward state only through the records and a snapshot
// of the channel table (chans), never the workspace, so the next replay may
// run beside them.
void launch_adj_a(int prec, const ChanDev *chans, const NodeTile *tiles, int n_tiles,
                  char *aws, const AdjChan *achans, const int64_t *t0, int slot, int buf,
                  hipStream_t st);
void launch_adj_b(int prec, const ChanDev *chans, const NodeTile *tiles, int n_tiles,
                  char *aws, const AdjChan *achans, const int64_t *t0, int slot, int buf,
                  hipStream_t st);
// Blocked reverse sweep (channels of at most kAdjBlockedMaxNodes nodes): the block of
// reverse steps slot_hi, slot_hi - 1, ..., slot_hi - count + 1 (count <=
// kAdjMaxBlock) as one bulk pass over the adjoint ring for the block's
// entries and one launch of one workgroup per channel for the steps (with
// the block's adjoint state on chip when max_ly, the widest channel's ly, is
// at most 128).
void launch_adj_bulk(int prec, const ChanDev *chans, const NodeTile *tiles, int n_tiles,
                     char *aws, const AdjChan *achans, const int64_t *t0, int slot_hi,
                     int count, int buf, hipStream_t st);
void launch_adj_span(int prec, const ChanDev *chans, int n_ch, int max_ly, char *aws,
                     const AdjChan *achans, const int64_t *t0, int slot_hi, int count,
                     int buf, hipStream_t st);
void launch_store_i64(int64_t *p, int64_t v, hipStream_t st);
// Step records on in the device channel table (each channel's record area of
// buffer buf in the adjoint workspace aws, from step t0), or off (aws null).
void launch_set_record(ChanDev *chans, const AdjChan *achans, int n_ch, char *aws, int buf,
                       int64_t t0, hipStream_t st);
void launch_adj_reduce(const ChanDev *chans, int n_ch, char *aws, const AdjChan *achans,
                       double *out, hipStream_t st);
void launch_set_params(ChanDev *chans, int ch, double g_inf, double tau_m, double gamma_c,
                       hipStream_t st);

}  // namespace lbmax
