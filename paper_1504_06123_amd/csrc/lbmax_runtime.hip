// lbmax_runtime.hip -- host side of liblbmax: the C interface declared in
// include/lbmax.h.  Validates descriptions, lays out the caller-owned
// workspace, builds the launch tile lists, enqueues steps (plain launches or
// hipGraph replays), and implements readouts and state snapshots.
#include "lbmax.h"
#include "lbmax_checks.h"
#include "lbmax_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace lbmax;

// ---------------------------------------------------------------------------
// The library's own adjoint workspace, for lb_adjoint_begin_noalloc: a static
// device array, one copy on each GPU the library runs on, held until the
// process ends and shared by every handle on that GPU.  In host code its name
// is only a stand-in: the device address of each GPU's copy is taken once per
// device with hipGetSymbolAddress (lb_init, that device current) and that
// address is what kernels and copies receive.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Device address of the array on GPU dev (the current device), looked up on
// the first call for that device.
hipError_t scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

thread_local std::string g_err;

lb_status fail(lb_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Block-sum planes of a channel, doubles per node: A_m and B_m (and the
// sigma_yy sums of a full-tensor channel), then one interior strain per
// block of a grid channel.
int blk_planes(const ChanDev &c) { return c.finger ? 3 * kMaxBlock : 2 * kMaxBlock + c.qb; }

constexpr uint64_t kStateMagic = 0x4C424D4158535431ull;  // "LBMAXST1"
constexpr uint32_t kStateVersion = 6;
constexpr size_t kStateHeader = 256;
constexpr int64_t kMaxStepsPerBatch = int64_t(1) << 20;

struct StateHeader {
    uint64_t magic;
    uint32_t version;
    uint32_t precision;
    int64_t t;
    int32_t n_ch;
    int32_t reserved;
    uint64_t bytes;
    int32_t block_len;
    int32_t block_pos;
};

bool unidirectional(const lb_channel_desc &d)
{
    if (d.lx != 1 || d.gy != 0.0)
        return false;
    if (d.u0)
        for (int y = 0; y < d.ly; ++y)
            if (d.u0[(size_t)d.ly + y] != 0.0)
                return false;
    return true;
}

std::string check_desc(const lb_channel_desc *ch, int32_t n_ch, lb_precision prec)
{
    if (!ch)
        return "channel array is NULL";
    if (n_ch < 1)
        return "n_ch must be >= 1";
    for (int i = 0; i < n_ch; ++i) {
        const lb_channel_desc &d = ch[i];
        char buf[160];
        auto bad = [&](const char *what) {
            snprintf(buf, sizeof buf, "channel %d: %s", i, what);
            return std::string(buf);
        };
        if (d.lx < 1)
            return bad("lx must be >= 1");
        if (d.ly < 3)
            return bad("ly must be >= 3");
        // the history pass addresses 8 ring rows of a plane with 32-bit offsets
        if ((int64_t)d.lx * d.ly > ((int64_t)1 << 26) - 64)
            return bad("too many nodes (at most 2^26 - 64 per channel)");
        if (d.hist_blocks < 0)
            return bad("hist_blocks must be >= 0");
        if (d.hist_blocks == 0 && d.law != 2 && d.n_hist < 2)
            return bad("n_hist must be >= 2");
        // FP32 histories take the age of an entry as an FP32 number, exact
        // below 2^24
        if (prec != LB_F64 && d.hist_blocks == 0 && d.law != 2 && d.n_hist > (1 << 24))
            return bad("n_hist must be <= 2^24 with FP32 histories");
        if (d.finger != 0 && d.finger != 1)
            return bad("finger must be 0 or 1");
        if (d.paper_coupling != 0 && d.paper_coupling != 1)
            return bad("paper_coupling must be 0 or 1");
        if (d.law < 0 || d.law > 2)
            return bad("law must be 0 (nlM), 1 (accumulated-strain damping) or 2 "
                       "(instantaneous)");
        if (d.law != 0 && (d.finger || d.hist_blocks > 0))
            return bad("the alternative laws use the simple-shear reduction on the uniform "
                       "window (finger = 0, hist_blocks = 0)");
        if (d.finger && d.hist_blocks > 0)
            return bad("the full Finger tensor runs on the uniform window (hist_blocks = 0)");
        if (d.hist_blocks > 0) {
            if (d.hist_blocks > 20)
                return bad("hist_blocks must be <= 20");
            if (d.hist_block_len < 2)
                return bad("hist_block_len must be >= 2");
            if (((int64_t)d.hist_block_len << d.hist_blocks) > ((int64_t)1 << 30))
                return bad("hist_block_len * 2^hist_blocks must be <= 2^30");
        }
        if (!std::isfinite(d.tau_lb) || !(d.tau_lb > 0.5))
            return bad("tau_lb must be finite and > 1/2");
        if (!std::isfinite(d.g_inf) || d.g_inf < 0.0)
            return bad("g_inf must be finite and >= 0");
        if (!std::isfinite(d.tau_m) || !(d.tau_m > 0.0))
            return bad("tau_m must be finite and > 0");
        if (std::isnan(d.gamma_c) || !(d.gamma_c > 0.0))
            return bad("gamma_c must be > 0 (or +inf)");
        if (!std::isfinite(d.gx) || !std::isfinite(d.gy))
            return bad("body force must be finite");
        if (d.u0) {
            const size_t cnt = 2 * (size_t)d.lx * d.ly;
            for (size_t k = 0; k < cnt; ++k)
                if (!std::isfinite(d.u0[k]))
                    return bad("u0 has a non-finite entry");
        }
    }
    return "";
}

// Workspace plan: header | channel table | node tiles | history tiles |
// readout staging | per-channel planes.  Everything 256-byte aligned.
struct Plan {
    size_t total = 0;
    size_t off_tcount = 0, off_chans = 0, off_node_tiles = 0, off_hist_tiles = 0,
           off_stage = 0, stage_bytes = 0;
    int n_node_tiles = 0, n_hist_tiles_max = 0;
    std::vector<ChanDev> chans;
};

int max_chunks_for(int n_hist, int np)
{
    int m = std::min(kMaxChunks, std::max(1, n_hist / kMinChunkLen));
    const int64_t cap = std::max<int64_t>(1, kPartialBudget / np);
    return (int)std::min<int64_t>(m, cap);
}

// Element sizes of the lattice planes (stress, velocity, density), of the
// stored populations and of the history ring.
size_t lattice_bytes(lb_precision) { return 8; }
size_t pop_bytes(lb_precision prec) { return prec == LB_F32 ? 4 : 8; }
size_t history_bytes(lb_precision prec) { return prec == LB_F64 ? 8 : 4; }
int prec_code(lb_precision prec) { return prec == LB_F64 ? 0 : (prec == LB_F32 ? 1 : 2); }

Plan make_plan(const lb_channel_desc *ch, int32_t n_ch, lb_precision prec)
{
    const size_t R = lattice_bytes(prec), RH = history_bytes(prec);
    Plan P;
    size_t off = 0;
    P.off_tcount = off;
    off += 256;
    P.off_chans = off;
    off = align_up(off + (size_t)n_ch * sizeof(ChanDev), 256);
    size_t stage = 0;
    P.chans.resize(n_ch);
    for (int i = 0; i < n_ch; ++i) {
        const lb_channel_desc &d = ch[i];
        ChanDev &c = P.chans[i];
        std::memset(&c, 0, sizeof c);
        c.lx = d.lx;
        c.ly = d.ly;
        c.n = d.lx * d.ly;
        c.np = (int)align_up((size_t)c.n, kNodeAlign);
        c.finger = d.finger;
        c.coupling = d.paper_coupling;
        c.law = d.law;
        c.qb = d.hist_blocks;
        c.qc = d.hist_blocks > 0 ? d.hist_block_len : 0;
        c.n_hist = (d.hist_blocks > 0 || d.law == 2) ? 0 : d.n_hist;
        c.has_r = (unidirectional(d) && !d.finger) ? 0 : 1;
        c.max_chunks = (d.hist_blocks > 0 || d.law != 0) ? 1 : max_chunks_for(d.n_hist, c.np);
        c.nchunks = 1;
        c.vec = 1;
        c.omega = 1.0 / d.tau_lb;
        c.g_inf = d.g_inf;
        c.inv_tau = 1.0 / d.tau_m;
        c.inv_gc = std::isinf(d.gamma_c) ? 0.0 : 1.0 / d.gamma_c;
        c.l2_tau = M_LOG2E * c.inv_tau;
        c.l2_gc = M_LOG2E * c.inv_gc;
        c.gx = d.gx;
        c.gy = d.gy;
        const int blocks = (c.n + kBlock - 1) / kBlock;
        P.n_node_tiles += blocks;
        // history tiles: at most one per wavefront of nodes and age chunk
        if (c.qb == 0 && c.law != 2)
            P.n_hist_tiles_max += ((c.n + kWave - 1) / kWave) * c.max_chunks;
        stage = std::max(stage, (size_t)4 * c.n);
    }
    P.off_node_tiles = off;
    off = align_up(off + (size_t)P.n_node_tiles * sizeof(NodeTile), 256);
    P.off_hist_tiles = off;
    off = align_up(off + (size_t)P.n_hist_tiles_max * sizeof(HistTile), 256);
    P.off_stage = off;
    P.stage_bytes = align_up(stage * sizeof(double), 256);
    off += P.stage_bytes;
    for (int i = 0; i < n_ch; ++i) {
        ChanDev &c = P.chans[i];
        const size_t plane = (size_t)c.np * R;
        c.off_pop = (int64_t)off;
        off = align_up(off + 18 * (size_t)c.np * pop_bytes(prec), 256);
        c.off_mom = 0;
        if (prec == LB_F32) {
            c.off_mom = (int64_t)off;
            off = align_up(off + 6 * (size_t)c.np * sizeof(double), 256);
        }
        c.off_sig = (int64_t)off;
        off = align_up(off + 3 * plane, 256);
        c.off_vel = (int64_t)off;
        off = align_up(off + 2 * plane, 256);
        c.off_rho = (int64_t)off;
        off = align_up(off + plane, 256);
        c.off_trace = (int64_t)off;
        off = align_up(off + plane, 256);
        const size_t hplane = (size_t)c.np * RH;
        c.off_ring_s = (int64_t)off;
        off = align_up(off + (c.finger ? 8 : 1) * (size_t)c.n_hist * hplane, 256);
        c.off_ring_r = (int64_t)off;
        if (c.has_r && !c.finger)
            off = align_up(off + (size_t)c.n_hist * hplane, 256);
        c.off_part = (int64_t)off;
        if (c.max_chunks > 1)
            off = align_up(off + (size_t)(c.finger ? kFingerPartPlanes : kPartPlanes) *
                                     c.max_chunks * c.np * sizeof(double),
                           256);
        c.off_blk = (int64_t)off;
        off = align_up(off + (size_t)blk_planes(c) * c.np * sizeof(double), 256);
        const size_t grows = (size_t)c.qb * c.qc;  // 0 without a grid
        c.off_grid_s = (int64_t)off;
        off = align_up(off + grows * hplane, 256);
        c.off_grid_r = (int64_t)off;
        if (c.has_r)
            off = align_up(off + grows * hplane, 256);
        c.off_grid_d = (int64_t)off;
        if (c.has_r)
            off = align_up(off + 3 * grows * hplane, 256);
    }
    P.total = off;
    return P;
}

}  // namespace

struct lb_handle {
    int n_ch = 0;
    lb_precision prec = LB_F32;
    int pc = 1;  // kernel precision code
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    Plan plan;
    std::vector<int> ly, lx, n_hist;
    int64_t t = 0;          // completed steps
    int block = 1;          // steps served by one history pass
    int block_pos = 0;      // steps done in the current block (0: next is a pass)
    bool has_out = false;   // readout planes belong to step t-1
    bool poisoned = false;
    int checks = LB_CHECK_FINITE | LB_CHECK_MACH;  // lb_set_checks
    int warnings = 0;                              // raised since the last lb_warnings
    // device pointers into the workspace
    int64_t *d_tcount = nullptr;
    int *d_tile_counters = nullptr;  // in the header block after the step counter
    bool persistent = false;
    int num_cus = 0;
    ChanDev *d_chans = nullptr;
    NodeTile *d_node_tiles = nullptr;
    HistTile *d_hist_tiles = nullptr;
    double *d_stage = nullptr;
    int n_node_tiles = 0, n_hist_tiles = 0;
    // history tile groups: lane width 1, 2, 4 (simple-shear pass), full tensor,
    // accumulated-strain damping
    int hist_group_begin[5] = {0, 0, 0, 0, 0}, hist_group_count[5] = {0, 0, 0, 0, 0};
    bool any_finger = false, any_wm = false, any_inst = false;
    bool any_chunked = false;
    bool any_grid = false, any_window = false;  // channels on the grid / the uniform window
    bool fuse_ok = false;      // every channel fits the fused in-block steps
    bool fuse_lds_ok = false;  // ... and takes the LDS-resident form
    bool fuse_global_ok = false;  // ... and is narrow enough for the global-memory form to pay
    bool fuse_lds_ready = false;  // its dynamic LDS size is allowed
    int fuse_mode = 1;         // lb_set_fused
    // host mirrors kept alive for asynchronous uploads
    std::vector<NodeTile> node_tiles;
    std::vector<HistTile> hist_tiles;
    std::vector<char> upload;
    // graph replay
    int graph_steps = 0;
    bool graph_dirty = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // adjoint sweep
    char *aws = nullptr;
    size_t aws_bytes = 0;
    AdjChan *d_achans = nullptr;
    double *d_adj_out = nullptr;
    std::vector<AdjChan> achans;  // n_ch entries from lb_init on
    void *scratch = nullptr;      // the library's device array on this handle's GPU
    int64_t *d_adj_t0 = nullptr;     // [2]: first step of the segment in each record buffer
    ChanDev *d_adj_snap = nullptr;   // [2][n_ch]: channel table of the segment in each buffer
    double *d_adj_stage[2] = {nullptr, nullptr};  // dL/du_x as given, per record buffer
    // the reverse sweeps run on their own stream, beside the next segment's
    // replay on the handle's stream; events order the two
    hipStream_t adj_stream = nullptr;
    // reads of a checkpoint's header and forces in lb_adjoint_segment, which
    // must not wait for the replay in flight on the handle's stream
    hipStream_t io_stream = nullptr;
    hipEvent_t adj_ev_replay = nullptr;
    hipEvent_t adj_ev_input = nullptr;  // the segment's dL/du_x has left the caller's buffer
    hipEvent_t adj_ev_sweep[2] = {nullptr, nullptr};
    bool adj_sweep_pending[2] = {false, false};
    int adj_segments = 0;            // segments swept since lb_adjoint_begin
    // captured reverse sweeps by segment length (for this adjoint workspace)
    std::vector<std::pair<int, hipGraphExec_t>> adj_execs;  // key: 2 * n_steps + buffer
    int adj_seg_len = 0;
    int adj_block = kAdjMaxBlock;  // lb_set_adjoint_block
    int64_t adj_next = -1;  // the next segment must end at this step (-1: no sweep)
    // timing: event pairs recorded around launches, resolved on demand
    bool profile = false;
    std::vector<hipEvent_t> free_events;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[3];
    double kernel_ms[3] = {0.0, 0.0, 0.0};
    int64_t kernel_launches[3] = {0, 0, 0};
};

namespace {

#define HIP_TRY(h, call)                                                        \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            if (h)                                                              \
                (h)->poisoned = true;                                           \
            return fail(LB_EDEVICE, std::string(#call) + ": " +                 \
                                        hipGetErrorString(e_));                 \
        }                                                                       \
    } while (0)

lb_status check_launch(lb_handle *h, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        h->poisoned = true;
        return fail(LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
    return LB_OK;
}

lb_status usable(lb_handle *h)
{
    if (!h)
        return fail(LB_EINVAL, "handle is NULL");
    if (h->poisoned)
        return fail(LB_ESTATE, "handle is poisoned by an earlier device error");
    return LB_OK;
}

// Lane widths with a history-pass instantiation for a block length.
int effective_vec(int vec, int block)
{
    if (block >= 8)
        return 1;
    if (block > 1)
        return std::min(vec, 2);
    return vec;
}

// Split every channel's window into its chunks and list the tiles, longest
// age range first so uneven channels finish together.  A simple-shear tile
// covers 64*vec nodes (one wavefront), a full-tensor or accumulated-strain
// tile 256 (one workgroup).
void build_tiles(lb_handle *h)
{
    h->node_tiles.clear();
    h->hist_tiles.clear();
    h->any_chunked = false;
    h->any_grid = h->any_window = h->any_inst = false;
    for (int ci = 0; ci < h->n_ch; ++ci) {
        const ChanDev &c = h->plan.chans[ci];
        for (int n0 = 0; n0 < c.n; n0 += kBlock)
            h->node_tiles.push_back({ci, n0});
        if (c.qb > 0) {
            h->any_grid = true;  // stepped by k_grid_step, no history tiles
            continue;
        }
        if (c.law == 2) {
            h->any_inst = true;  // stepped by k_inst_step, no history
            continue;
        }
        h->any_window = true;
        if (c.nchunks > 1)
            h->any_chunked = true;
        const int span = (c.finger || c.law) ? kBlock : kWave * effective_vec(c.vec, h->block);
        for (int k = 0; k < c.nchunks; ++k) {
            const int k0 = (int)((int64_t)c.n_hist * k / c.nchunks);
            const int k1 = (int)((int64_t)c.n_hist * (k + 1) / c.nchunks);
            for (int n0 = 0; n0 < c.n; n0 += span)
                h->hist_tiles.push_back({ci, n0, k0, k1, k, 0});
        }
    }
    // Group by lane width (one launch each), longest age range first inside
    // a group.
    auto group = [h](const HistTile &a) {
        if (h->plan.chans[a.ch].law == 1)
            return 4;
        if (h->plan.chans[a.ch].finger)
            return 3;
        const int v = effective_vec(h->plan.chans[a.ch].vec, h->block);
        return v == 4 ? 2 : (v == 2 ? 1 : 0);
    };
    std::stable_sort(h->hist_tiles.begin(), h->hist_tiles.end(),
                     [&](const HistTile &a, const HistTile &b) {
                         if (group(a) != group(b))
                             return group(a) < group(b);
                         return (a.k1 - a.k0) > (b.k1 - b.k0);
                     });
    for (int g = 0; g < 5; ++g)
        h->hist_group_count[g] = 0;
    for (const HistTile &tl : h->hist_tiles)
        h->hist_group_count[group(tl)] += 1;
    h->hist_group_begin[0] = 0;
    h->hist_group_begin[1] = h->hist_group_count[0];
    h->hist_group_begin[2] = h->hist_group_count[0] + h->hist_group_count[1];
    h->hist_group_begin[3] = h->hist_group_begin[2] + h->hist_group_count[2];
    h->hist_group_begin[4] = h->hist_group_begin[3] + h->hist_group_count[3];
    h->any_finger = h->hist_group_count[3] > 0;
    h->any_wm = h->hist_group_count[4] > 0;
    h->n_node_tiles = (int)h->node_tiles.size();
    h->n_hist_tiles = (int)h->hist_tiles.size();
    h->fuse_ok = !h->any_grid && !h->any_inst;
    h->fuse_lds_ok = h->fuse_ok;
    h->fuse_global_ok = h->fuse_ok;
    for (const ChanDev &c : h->plan.chans) {
        if (c.n > kFuseMaxNodes)
            h->fuse_ok = h->fuse_lds_ok = false;
        if (c.n > kFuseGlobalMaxNodes)
            h->fuse_global_ok = false;
        if (c.law != 0 || c.finger || c.coupling || c.has_r)
            h->fuse_lds_ok = false;
    }
    if (h->fuse_lds_ok && !h->fuse_lds_ready)
        h->fuse_lds_ready = prepare_fused_lds(h->pc) == 0;
}

// Default launch shape: wide lanes for large channels, and enough age chunks
// that the history launch has about 2048 workgroups.
void default_tiling(lb_handle *h)
{
    int total = 0;
    for (ChanDev &c : h->plan.chans) {
        const bool plain = c.qb == 0 && c.law == 0 && !c.finger;
        c.vec = !plain ? 1 : (c.n >= (1 << 16) ? 4 : (c.n >= (1 << 12) ? 2 : 1));
        if (c.qb == 0 && c.law != 2)
            total += (c.n + kBlock * c.vec - 1) / (kBlock * c.vec);
    }
    total = std::max(total, 1);
    const int want = std::max(1, (2048 + total - 1) / total);
    for (ChanDev &c : h->plan.chans)
        c.nchunks = std::max(1, std::min(want, c.max_chunks));
}

lb_status upload_tables(lb_handle *h)
{
    if ((int)h->hist_tiles.size() > h->plan.n_hist_tiles_max ||
        (int)h->node_tiles.size() > h->plan.n_node_tiles)
        return fail(LB_EINVAL, "internal: tile lists exceed their workspace area");
    HIP_TRY(h, hipMemcpyAsync(h->d_chans, h->plan.chans.data(),
                              h->plan.chans.size() * sizeof(ChanDev),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->d_node_tiles, h->node_tiles.data(),
                              h->node_tiles.size() * sizeof(NodeTile),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->d_hist_tiles, h->hist_tiles.data(),
                              h->hist_tiles.size() * sizeof(HistTile),
                              hipMemcpyHostToDevice, h->stream));
    // The host vectors are reused only after this synchronisation.
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->graph_dirty = true;
    return LB_OK;
}

lb_status take_event(lb_handle *h, hipEvent_t *ev)
{
    if (!h->free_events.empty()) {
        *ev = h->free_events.back();
        h->free_events.pop_back();
        return LB_OK;
    }
    HIP_TRY(h, hipEventCreate(ev));
    return LB_OK;
}

// Add up the elapsed time of every recorded pair (the stream must be idle).
lb_status resolve_timing(lb_handle *h)
{
    for (int w = 0; w < 3; ++w) {
        for (auto &pr : h->pending[w]) {
            float ms = 0.f;
            HIP_TRY(h, hipEventElapsedTime(&ms, pr.first, pr.second));
            h->kernel_ms[w] += ms;
            h->kernel_launches[w] += 1;
            h->free_events.push_back(pr.first);
            h->free_events.push_back(pr.second);
        }
        h->pending[w].clear();
    }
    return LB_OK;
}

// One step's launches, step t = *tcount + trel, position m in its block (0:
// the history pass).  With `timed`, HIP event pairs bracket the lattice launch
// (slot 1) and the history work (slot 0 for a pass, slot 2 for a block step).
lb_status enqueue_step(lb_handle *h, hipStream_t st, int trel, int m, bool timed)
{
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    if (timed) {
        for (int i = 0; i < 4; ++i) {
            lb_status s = take_event(h, &e[i]);
            if (s != LB_OK)
                return s;
        }
        HIP_TRY(h, hipEventRecord(e[0], st));
    }
    launch_lb(h->pc, h->ws, h->d_chans, h->d_node_tiles, h->n_node_tiles,
              h->d_tcount, trel, h->d_tile_counters, st);
    if (timed) {
        HIP_TRY(h, hipEventRecord(e[1], st));
        HIP_TRY(h, hipEventRecord(e[2], st));
    }
    if (h->any_grid)
        launch_grid_step(h->pc, h->block, m, h->ws, h->d_chans, h->d_node_tiles,
                         h->n_node_tiles, h->d_tcount, trel, st);
    if (h->any_inst)
        launch_inst_step(h->pc, h->ws, h->d_chans, h->d_node_tiles, h->n_node_tiles,
                         h->d_tcount, trel, st);
    if (m == 0) {
        static const int kVec[3] = {1, 2, 4};
        for (int g = 0; g < 3; ++g) {
            const int pgrid =
                h->persistent ? h->num_cus * hist_pass_blocks_per_cu(h->pc, kVec[g], h->block)
                              : 0;
            launch_hist_pass(h->pc, kVec[g], h->block, h->ws, h->d_chans,
                             h->d_hist_tiles + h->hist_group_begin[g], h->hist_group_count[g],
                             h->d_tcount, trel, pgrid, h->d_tile_counters + g, st);
        }
        if (h->any_wm)
            launch_wm_pass(h->pc, h->block, h->ws, h->d_chans,
                           h->d_hist_tiles + h->hist_group_begin[4], h->hist_group_count[4],
                           h->d_tcount, trel, st);
        if (h->any_finger) {
            const int pgrid =
                h->persistent ? h->num_cus * finger_pass_blocks_per_cu(h->pc, h->block) : 0;
            launch_finger_pass(h->pc, h->block, h->ws, h->d_chans,
                               h->d_hist_tiles + h->hist_group_begin[3], h->hist_group_count[3],
                               h->d_tcount, trel, pgrid, h->d_tile_counters + 3, st);
        }
        if (h->any_chunked)
            launch_combine(h->pc, h->block, h->ws, h->d_chans, h->d_node_tiles,
                           h->n_node_tiles, st);
    } else if (h->any_window) {
        launch_hist_step(h->pc, m, h->ws, h->d_chans, h->d_node_tiles, h->n_node_tiles,
                         h->d_tcount, trel, st);
    }
    if (timed) {
        HIP_TRY(h, hipEventRecord(e[3], st));
        h->pending[1].push_back({e[0], e[1]});
        h->pending[m == 0 ? 0 : 2].push_back({e[2], e[3]});
    }
    return check_launch(h, "step launch");
}

// The in-block steps run fused: mode 2 whenever the channels fit a
// workgroup; mode 1 (the default) in the LDS form where it applies, else in
// the global-memory form only up to kFuseGlobalMaxNodes nodes per channel.
bool fused_in_effect(const lb_handle *h)
{
    if (!h->fuse_ok || h->fuse_mode == 0 || h->block <= 1)
        return false;
    if (h->fuse_mode == 2)
        return true;
    return (h->fuse_lds_ok && h->fuse_lds_ready) || h->fuse_global_ok;
}

// Enqueue up to `left` steps starting at block position m: a fused launch
// for the rest of the block when the handle allows it and m > 0, else one
// step.  Sets *done to the steps enqueued.
lb_status enqueue_span(lb_handle *h, hipStream_t st, int trel, int m, int64_t left, bool timed,
                       int *done)
{
    if (fused_in_effect(h) && m > 0) {
        const int k = (int)std::min<int64_t>(left, h->block - m);
        hipEvent_t e[2] = {nullptr, nullptr};
        if (timed) {
            for (int i = 0; i < 2; ++i) {
                lb_status s = take_event(h, &e[i]);
                if (s != LB_OK)
                    return s;
            }
            HIP_TRY(h, hipEventRecord(e[0], st));
        }
        const bool lds = h->fuse_mode == 1 && h->fuse_lds_ok && h->fuse_lds_ready;
        launch_fused_steps(h->pc, lds, h->ws, h->d_chans, h->n_ch, h->d_tcount, trel, m, k, st);
        if (timed) {
            HIP_TRY(h, hipEventRecord(e[1], st));
            h->pending[2].push_back({e[0], e[1]});
        }
        *done = k;
        return check_launch(h, "fused steps launch");
    }
    *done = 1;
    return enqueue_step(h, st, trel, m, timed);
}

lb_status capture_graph(lb_handle *h)
{
    if (h->graph_exec) {
        (void)hipGraphExecDestroy(h->graph_exec);
        h->graph_exec = nullptr;
    }
    if (h->graph) {
        (void)hipGraphDestroy(h->graph);
        h->graph = nullptr;
    }
    if (!h->cap_stream)
        HIP_TRY(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0, k = 0; i < h->graph_steps; i += k) {
        lb_status s = enqueue_span(h, h->cap_stream, i, i % h->block, h->graph_steps - i, false,
                                   &k);
        if (s != LB_OK) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(h->cap_stream, &g);
            if (g)
                (void)hipGraphDestroy(g);
            return s;
        }
    }
    launch_tick(h->d_tcount, h->graph_steps, h->cap_stream);
    HIP_TRY(h, hipStreamEndCapture(h->cap_stream, &h->graph));
    HIP_TRY(h, hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
    h->graph_dirty = false;
    return LB_OK;
}

lb_status readout(lb_handle *h, int32_t ch, int which, int comps,
                  double **outs)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (ch < 0 || ch >= h->n_ch)
        return fail(LB_EINVAL, "channel index out of range");
    if (!h->has_out)
        return fail(LB_ESTATE, "no completed step to read");
    const int N = h->plan.chans[ch].n;
    launch_readout(h->pc, which, h->ws, h->d_chans, ch, N, h->d_stage, h->stream);
    s = check_launch(h, "readout");
    if (s != LB_OK)
        return s;
    std::vector<double> host((size_t)comps * N);
    HIP_TRY(h, hipMemcpyAsync(host.data(), h->d_stage, host.size() * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < comps; ++k)
        if (outs[k])
            std::memcpy(outs[k], host.data() + (size_t)k * N, N * sizeof(double));
    // velocity readout: the lattice Mach guard (both components, requested or not)
    if (which == 0 && (h->checks & LB_CHECK_MACH) &&
        mach_guard_trips(max_speed(host.data() + N, host.data() + 2 * (size_t)N, N)))
        h->warnings |= LB_WARN_MACH;
    if (h->checks & LB_CHECK_FINITE) {
        const ValueScan v = scan_values(host.data(), host.size());
        if (v.nonfinite)
            return fail(LB_ENONFINITE, "readout of channel " + std::to_string(ch) + ": " +
                                           std::to_string(v.nonfinite) +
                                           " non-finite values (the run has diverged)");
    }
    return LB_OK;
}

// Per-channel state sections: (workspace offset, rows, bytes per row) in
// the order of the state layout.
struct Section {
    int64_t ws_off;
    size_t rows, row_bytes, ws_pitch;
};

std::vector<Section> state_sections(const lb_handle *h, int ci, int64_t t)
{
    const ChanDev &c = h->plan.chans[ci];
    const size_t R = lattice_bytes(h->prec), RH = history_bytes(h->prec);
    const size_t rowb = (size_t)c.n * R, pitch = (size_t)c.np * R;
    const size_t hrowb = (size_t)c.n * RH, hpitch = (size_t)c.np * RH;
    const size_t PB = pop_bytes(h->prec);
    const int64_t cur = c.off_pop + (int64_t)(((t + 1) & 1) * 9 * (size_t)c.np * PB);
    std::vector<Section> v;
    v.push_back({cur, 9, (size_t)c.n * PB, (size_t)c.np * PB});
    v.push_back({c.off_sig, 3, rowb, pitch});
    v.push_back({c.off_vel, 2, rowb, pitch});
    v.push_back({c.off_rho, 1, rowb, pitch});
    v.push_back({c.off_trace, 1, rowb, pitch});
    if (c.qb > 0) {
        const size_t grows = (size_t)c.qb * c.qc;
        v.push_back({c.off_grid_s, grows, hrowb, hpitch});
        if (c.has_r) {
            v.push_back({c.off_grid_r, grows, hrowb, hpitch});
            v.push_back({c.off_grid_d, 3 * grows, hrowb, hpitch});
        }
    } else if (c.finger) {
        v.push_back({c.off_ring_s, 8 * (size_t)c.n_hist, hrowb, hpitch});
    } else {
        v.push_back({c.off_ring_s, (size_t)c.n_hist, hrowb, hpitch});
        if (c.has_r)
            v.push_back({c.off_ring_r, (size_t)c.n_hist, hrowb, hpitch});
    }
    v.push_back({c.off_blk, (size_t)blk_planes(c), (size_t)c.n * sizeof(double),
                 (size_t)c.np * sizeof(double)});
    return v;
}

size_t state_size(const lb_handle *h)
{
    size_t off = kStateHeader;
    for (int ci = 0; ci < h->n_ch; ++ci) {
        for (const Section &s : state_sections(h, ci, 0))
            off = align_up(off + s.rows * s.row_bytes, 256);
        off = align_up(off + 2 * sizeof(double), 256);
    }
    return off;
}


// ---------------------------------------------------------------------------
// Adjoint sweep
// ---------------------------------------------------------------------------
// Layout of an adjoint workspace: the channel table, the reduced gradients,
// the first step of the segment being swept (per record buffer), a snapshot
// of the forward channel table (per record buffer), then per channel its
// planes.  Writes each channel's offsets into chans[0 .. n_ch) when chans is
// not null (no allocation: the lb_adjoint_begin_noalloc path uses it too).
struct AdjLayout {
    size_t total = 0, off_table = 0, off_out = 0, off_t0 = 0, off_snap = 0;
    size_t off_stage[2] = {0, 0};  // [seg_len][sum of nodes] double: dL/du_x as the caller gives it
};

AdjLayout adj_layout(const lb_handle *h, int seg_len, AdjChan *chans)
{
    const size_t R = lattice_bytes(h->prec), RH = history_bytes(h->prec);
    AdjLayout P;
    size_t off = 0;
    P.off_table = off;
    off = align_up(off + (size_t)h->n_ch * sizeof(AdjChan), 256);
    P.off_out = off;
    off = align_up(off + (size_t)h->n_ch * 4 * sizeof(double), 256);
    P.off_t0 = off;
    off = align_up(off + 2 * sizeof(int64_t), 256);
    P.off_snap = off;
    off = align_up(off + 2 * (size_t)h->n_ch * sizeof(ChanDev), 256);
    size_t total_nodes = 0;
    for (const ChanDev &c : h->plan.chans)
        total_nodes += (size_t)c.n;
    for (int b = 0; b < 2; ++b) {
        P.off_stage[b] = off;
        off = align_up(off + (size_t)seg_len * total_nodes * sizeof(double), 256);
    }
    for (int ci = 0; ci < h->n_ch; ++ci) {
        const ChanDev &c = h->plan.chans[ci];
        const size_t plane = (size_t)c.np * R;
        AdjChan a{};
        a.off_sbar_ring = (int64_t)off;
        off = align_up(off + (size_t)c.n_hist * plane, 256);
        a.off_nbar = (int64_t)off;
        off = align_up(off + 9 * plane, 256);
        a.off_dbar = (int64_t)off;
        off = align_up(off + 9 * plane, 256);
        a.off_fbar = (int64_t)off;
        off = align_up(off + plane, 256);
        a.off_part = (int64_t)off;
        off = align_up(off + (size_t)kAdjGroups * 2 * c.np * sizeof(double), 256);
        a.off_acc = (int64_t)off;
        off = align_up(off + 4 * (size_t)c.np * sizeof(double), 256);
        a.off_bulk = (int64_t)off;
        off = align_up(off + (size_t)kAdjMaxBlock * 2 * c.np * sizeof(double), 256);
        for (int b = 0; b < 2; ++b) {
            a.off_rec[b] = (int64_t)off;
            off = align_up(off + (size_t)seg_len * 10 * plane, 256);
            a.off_dldu[b] = (int64_t)off;
            off = align_up(off + (size_t)seg_len * c.np * sizeof(double), 256);
            a.off_recs[b] = (int64_t)off;
            off = align_up(off + (size_t)seg_len * c.np * RH, 256);
        }
        if (chans)
            chans[ci] = a;
    }
    P.total = off;
    return P;
}

std::string adjoint_unsupported(const lb_handle *h, int seg_len)
{
    for (int ci = 0; ci < h->n_ch; ++ci) {
        const ChanDev &c = h->plan.chans[ci];
        if (c.qb > 0)
            return "the adjoint covers the uniform history window; channel " +
                   std::to_string(ci) + " uses the quasi-logarithmic grid";
        if (c.finger)
            return "the adjoint covers the simple-shear reduction; channel " +
                   std::to_string(ci) + " uses the full Finger tensor";
        if (c.coupling)
            return "the adjoint covers the body-force coupling; channel " + std::to_string(ci) +
                   " uses the paper's forcing term";
        if (c.law)
            return "the adjoint covers the integral nlM law; channel " + std::to_string(ci) +
                   " uses another constitutive law";
        if (c.lx != 1 || c.has_r)
            return "the adjoint covers unidirectional channels (lx = 1, gy = 0, u0_y = 0); "
                   "channel " + std::to_string(ci) + " is not";
        if (seg_len > c.n_hist)
            return "seg_len must not exceed the history window of every channel";
    }
    if (seg_len < 1)
        return "seg_len must be >= 1";
    return "";
}

// Segments up to this length replay a captured reverse sweep.
constexpr int kAdjGraphMaxSteps = 1024;

// Reverse steps per blocked launch pair in effect: the setting where every
// channel has at most kAdjBlockedMaxNodes nodes, else 1 (the per-step
// kernels).
int adj_block_in_effect(const lb_handle *h)
{
    if (h->adj_block <= 1)
        return 1;
    for (const ChanDev &c : h->plan.chans)
        if (c.ly > kAdjBlockedMaxNodes)
            return 1;
    return h->adj_block;
}

// Enqueue the reverse sweep of slots n_steps - 1 .. 0 on record buffer buf:
// k_adj_a and k_adj_b per step, or per block of reverse steps one bulk pass
// and one span launch.
lb_status enqueue_adj_sweep(lb_handle *h, int n_steps, int buf, hipStream_t st, bool check)
{
    const ChanDev *snap = h->d_adj_snap + (size_t)buf * h->n_ch;
    const int64_t *t0 = h->d_adj_t0 + buf;
    const int blk = adj_block_in_effect(h);
    if (blk > 1) {
        int max_ly = 0;
        for (const ChanDev &c : h->plan.chans)
            max_ly = std::max(max_ly, c.ly);
        for (int hi = n_steps - 1; hi >= 0; hi -= blk) {
            const int count = std::min(blk, hi + 1);
            launch_adj_bulk(h->pc, snap, h->d_node_tiles, h->n_node_tiles, h->aws, h->d_achans,
                            t0, hi, count, buf, st);
            launch_adj_span(h->pc, snap, h->n_ch, max_ly, h->aws, h->d_achans, t0, hi, count, buf,
                            st);
            if (check) {
                lb_status s = check_launch(h, "adjoint block");
                if (s != LB_OK)
                    return s;
            }
        }
        return LB_OK;
    }
    for (int k = n_steps - 1; k >= 0; --k) {
        launch_adj_a(h->pc, snap, h->d_node_tiles, h->n_node_tiles, h->aws, h->d_achans, t0, k,
                     buf, st);
        launch_adj_b(h->pc, snap, h->d_node_tiles, h->n_node_tiles, h->aws, h->d_achans, t0, k,
                     buf, st);
        if (check) {
            lb_status s = check_launch(h, "adjoint step");
            if (s != LB_OK)
                return s;
        }
    }
    return LB_OK;
}

void drop_adj_graphs(lb_handle *h)
{
    for (auto &e : h->adj_execs)
        (void)hipGraphExecDestroy(e.second);
    h->adj_execs.clear();
}

// The reverse sweep of n_steps steps on record buffer buf (k_adj_a then
// k_adj_b for slots n_steps-1 .. 0), captured once per length and buffer and
// replayed for every segment.  The graph holds the adjoint workspace's
// addresses and the node-tile pointer and count (fixed for the handle's life:
// node tiles depend on the channels only); lb_adjoint_begin drops the graphs
// when the adjoint workspace or segment length changes.
lb_status adj_sweep_graph(lb_handle *h, int n_steps, int buf, hipGraphExec_t *out)
{
    const int key = 2 * n_steps + buf;
    for (auto &e : h->adj_execs)
        if (e.first == key) {
            *out = e.second;
            return LB_OK;
        }
    if (!h->cap_stream)
        HIP_TRY(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    (void)enqueue_adj_sweep(h, n_steps, buf, h->cap_stream, false);
    const hipError_t cap = hipGetLastError();
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(h->cap_stream, &g);
    if (cap != hipSuccess || end != hipSuccess || !g) {
        if (g)
            (void)hipGraphDestroy(g);
        h->poisoned = true;
        return fail(LB_EDEVICE, std::string("adjoint sweep capture: ") +
                                    hipGetErrorString(cap != hipSuccess ? cap : end));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t inst = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (inst != hipSuccess) {
        h->poisoned = true;
        return fail(LB_EDEVICE, std::string("adjoint sweep graph: ") + hipGetErrorString(inst));
    }
    h->adj_execs.push_back({key, exec});
    *out = exec;
    return LB_OK;
}

// Wait for every reverse sweep enqueued on the adjoint stream.
lb_status adj_drain(lb_handle *h)
{
    if (h->adj_stream)
        HIP_TRY(h, hipStreamSynchronize(h->adj_stream));
    h->adj_sweep_pending[0] = h->adj_sweep_pending[1] = false;
    return LB_OK;
}

}  // namespace

extern "C" {

const char *lb_last_error(void) { return g_err.c_str(); }

size_t lb_workspace_bytes(const lb_channel_desc *ch, int32_t n_ch, lb_precision prec)
{
    if (prec != LB_F64 && prec != LB_F32 && prec != LB_F32_P64) {
        g_err = "unknown precision";
        return 0;
    }
    std::string why = check_desc(ch, n_ch, prec);
    if (!why.empty()) {
        g_err = why;
        return 0;
    }
    return make_plan(ch, n_ch, prec).total;
}

lb_status lb_init(const lb_channel_desc *ch, int32_t n_ch, lb_precision prec, void *d_ws,
                  size_t ws_bytes, void *stream, lb_handle **out)
{
    if (!out)
        return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (prec != LB_F64 && prec != LB_F32 && prec != LB_F32_P64)
        return fail(LB_EINVAL, "unknown precision");
    std::string why = check_desc(ch, n_ch, prec);
    if (!why.empty())
        return fail(LB_EINVAL, why);
    if (!d_ws)
        return fail(LB_EINVAL, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0)
        return fail(LB_ENOMEM, "workspace must be 256-byte aligned");
    Plan plan = make_plan(ch, n_ch, prec);
    if (ws_bytes < plan.total)
        return fail(LB_ENOMEM, "workspace too small: need " + std::to_string(plan.total) +
                                   " bytes, got " + std::to_string(ws_bytes));

    lb_handle *h = new lb_handle();
    h->n_ch = n_ch;
    h->prec = prec;
    h->pc = prec_code(prec);
    h->ws = static_cast<char *>(d_ws);
    h->ws_bytes = ws_bytes;
    h->stream = static_cast<hipStream_t>(stream);
    h->plan = std::move(plan);
    h->d_tcount = reinterpret_cast<int64_t *>(h->ws + h->plan.off_tcount);
    h->d_tile_counters = reinterpret_cast<int *>(h->ws + h->plan.off_tcount + 64);
    h->d_chans = reinterpret_cast<ChanDev *>(h->ws + h->plan.off_chans);
    h->d_node_tiles = reinterpret_cast<NodeTile *>(h->ws + h->plan.off_node_tiles);
    h->d_hist_tiles = reinterpret_cast<HistTile *>(h->ws + h->plan.off_hist_tiles);
    h->d_stage = reinterpret_cast<double *>(h->ws + h->plan.off_stage);
    for (int i = 0; i < n_ch; ++i) {
        h->lx.push_back(ch[i].lx);
        h->ly.push_back(ch[i].ly);
        h->n_hist.push_back(ch[i].n_hist);
    }

    h->achans.resize(n_ch);
    default_tiling(h);
    build_tiles(h);
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess || h->num_cus <= 0) {
            delete h;
            return fail(LB_EDEVICE, "cannot query the compute-unit count");
        }
        const hipError_t e = scratch_address(dev, &h->scratch);
        if (e != hipSuccess) {
            delete h;
            return fail(LB_EDEVICE, std::string("device address of the library's array: ") +
                                        hipGetErrorString(e));
        }
    }

    auto bail = [&](lb_status s) {
        delete h;
        return s;
    };

    // Zero the whole workspace (step counter, rings, partials), then upload
    // the tables and initialise each channel.
    launch_fill_zero(h->ws, h->plan.total, h->stream);
    lb_status s = check_launch(h, "zero fill");
    if (s != LB_OK)
        return bail(s);
    s = upload_tables(h);
    if (s != LB_OK)
        return bail(s);
    for (int i = 0; i < n_ch; ++i) {
        const ChanDev &c = h->plan.chans[i];
        const double *u0_dev = nullptr;
        if (ch[i].u0) {
            const size_t bytes = 2 * (size_t)c.n * sizeof(double);
            if (bytes > h->plan.stage_bytes)
                return bail(fail(LB_ENOMEM, "staging too small for u0"));
            if (hipMemcpyAsync(h->d_stage, ch[i].u0, bytes, hipMemcpyHostToDevice,
                               h->stream) != hipSuccess)
                return bail(fail(LB_EDEVICE, "u0 upload failed"));
            u0_dev = h->d_stage;
        }
        launch_init(h->pc, h->ws, h->d_chans, i, nullptr, (c.n + kBlock - 1) / kBlock,
                    u0_dev, h->stream);
        s = check_launch(h, "init");
        if (s != LB_OK)
            return bail(s);
        // The staging area is reused by the next channel: wait for this one.
        if (ch[i].u0 && hipStreamSynchronize(h->stream) != hipSuccess)
            return bail(fail(LB_EDEVICE, "init synchronisation failed"));
    }
    *out = h;
    return LB_OK;
}

lb_status lb_set_force(lb_handle *h, int32_t ch, double gx, double gy)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (ch < 0 || ch >= h->n_ch)
        return fail(LB_EINVAL, "channel index out of range");
    if (!std::isfinite(gx) || !std::isfinite(gy))
        return fail(LB_EINVAL, "body force must be finite");
    if (!h->plan.chans[ch].has_r && gy != 0.0)
        return fail(LB_EINVAL, "unidirectional channel: gy must stay 0");
    h->plan.chans[ch].gx = gx;
    h->plan.chans[ch].gy = gy;
    launch_set_force(h->d_chans, ch, gx, gy, h->stream);
    return check_launch(h, "set_force");
}

lb_status lb_step(lb_handle *h, int64_t n_steps)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (n_steps < 0)
        return fail(LB_EINVAL, "n_steps must be >= 0");
    int64_t left = n_steps;
    // Plain launches of a batch of steps starting at the current block
    // position; the device counter advances once per batch.
    auto eager = [&](int64_t count) -> lb_status {
        while (count > 0) {
            const int batch = (int)std::min(count, kMaxStepsPerBatch);
            for (int i = 0, k = 0; i < batch; i += k) {
                lb_status e = enqueue_span(h, h->stream, i, h->block_pos, batch - i, h->profile,
                                           &k);
                if (e != LB_OK)
                    return e;
                h->block_pos = (h->block_pos + k) % h->block;
            }
            launch_tick(h->d_tcount, batch, h->stream);
            lb_status e = check_launch(h, "tick");
            if (e != LB_OK)
                return e;
            count -= batch;
        }
        return LB_OK;
    };
    if (h->graph_steps > 0 && !h->profile) {
        // finish the current block, then replay whole graphs
        const int64_t head = h->block_pos == 0 ? 0 : std::min<int64_t>(left, h->block - h->block_pos);
        s = eager(head);
        if (s != LB_OK)
            return s;
        left -= head;
        if (left >= h->graph_steps) {
            if (h->graph_dirty) {
                s = capture_graph(h);
                if (s != LB_OK)
                    return s;
            }
            while (left >= h->graph_steps) {
                HIP_TRY(h, hipGraphLaunch(h->graph_exec, h->stream));
                left -= h->graph_steps;
            }
        }
    }
    s = eager(left);
    if (s != LB_OK)
        return s;
    h->t += n_steps;
    if (n_steps > 0)
        h->has_out = true;
    return LB_OK;
}

int64_t lb_time(const lb_handle *h) { return h ? h->t : -1; }

lb_status lb_set_checks(lb_handle *h, int32_t flags)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (flags & ~(LB_CHECK_FINITE | LB_CHECK_MACH))
        return fail(LB_EINVAL, "unknown check flags");
    h->checks = flags;
    return LB_OK;
}

int32_t lb_warnings(lb_handle *h)
{
    if (!h)
        return 0;
    const int w = h->warnings;
    h->warnings = 0;
    return w;
}

lb_status lb_fields(lb_handle *h, int32_t ch, double *rho, double *ux, double *uy)
{
    double *o[3] = {rho, ux, uy};
    return readout(h, ch, 0, 3, o);
}

lb_status lb_stress(lb_handle *h, int32_t ch, double *sxy, double *n1)
{
    double *o[2] = {sxy, n1};
    return readout(h, ch, 1, 2, o);
}

lb_status lb_grad(lb_handle *h, int32_t ch, double *kappa)
{
    if (h && ch >= 0 && ch < h->n_ch && !kappa)
        return fail(LB_EINVAL, "kappa is NULL");
    const int N = (h && ch >= 0 && ch < h->n_ch) ? h->plan.chans[ch].n : 0;
    double *o[4] = {kappa, kappa ? kappa + N : nullptr, kappa ? kappa + 2 * (size_t)N : nullptr,
                    kappa ? kappa + 3 * (size_t)N : nullptr};
    return readout(h, ch, 2, 4, o);
}

size_t lb_state_bytes(const lb_handle *h) { return h ? state_size(h) : 0; }

lb_status lb_save_state(lb_handle *h, void *d_dst)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (!d_dst || reinterpret_cast<uintptr_t>(d_dst) % 256 != 0)
        return fail(LB_EINVAL, "state buffer must be non-NULL and 256-byte aligned");
    char *dst = static_cast<char *>(d_dst);
    size_t off = kStateHeader;
    h->upload.assign(state_size(h) > 0 ? kStateHeader + 16 * (size_t)h->n_ch : 0, 0);
    StateHeader hd{kStateMagic, kStateVersion, (uint32_t)h->prec, h->t, h->n_ch, 0,
                   state_size(h), h->block, h->block_pos};
    std::memcpy(h->upload.data(), &hd, sizeof hd);
    for (int ci = 0; ci < h->n_ch; ++ci) {
        for (const Section &sec : state_sections(h, ci, h->t)) {
            HIP_TRY(h, hipMemcpy2DAsync(dst + off, sec.row_bytes, h->ws + sec.ws_off,
                                        sec.ws_pitch, sec.row_bytes, sec.rows,
                                        hipMemcpyDeviceToDevice, h->stream));
            off = align_up(off + sec.rows * sec.row_bytes, 256);
        }
        double g[2] = {h->plan.chans[ci].gx, h->plan.chans[ci].gy};
        std::memcpy(h->upload.data() + kStateHeader + 16 * (size_t)ci, g, 16);
        HIP_TRY(h, hipMemcpyAsync(dst + off, h->upload.data() + kStateHeader + 16 * (size_t)ci,
                                  16, hipMemcpyHostToDevice, h->stream));
        off = align_up(off + 2 * sizeof(double), 256);
    }
    HIP_TRY(h, hipMemcpyAsync(dst, h->upload.data(), sizeof hd, hipMemcpyHostToDevice,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}

namespace {

// Restore a state: header and forces are read to the host on `meta` (and
// that stream synchronised), the sections are copied on the handle's stream.
// With meta = the handle's stream the call returns once the copies are done
// (lb_load_state); with another stream they stay queued behind the handle's
// stream work, and the source must stay unchanged until that work has run
// (lb_adjoint_segment: a checkpoint the forward run finished, read while a
// replay may still be running).
lb_status load_state_impl(lb_handle *h, const void *d_src, hipStream_t meta)
{
    if (!d_src || reinterpret_cast<uintptr_t>(d_src) % 256 != 0)
        return fail(LB_EINVAL, "state buffer must be non-NULL and 256-byte aligned");
    const char *src = static_cast<const char *>(d_src);
    StateHeader hd{};
    HIP_TRY(h, hipMemcpyAsync(&hd, src, sizeof hd, hipMemcpyDeviceToHost, meta));
    HIP_TRY(h, hipStreamSynchronize(meta));
    if (hd.magic != kStateMagic || hd.version != kStateVersion)
        return fail(LB_EINVAL, "not a state buffer of this library version");
    if (hd.precision != (uint32_t)h->prec || hd.n_ch != h->n_ch || hd.bytes != state_size(h))
        return fail(LB_EINVAL, "state buffer belongs to a different configuration");
    if (hd.t < 0)
        return fail(LB_EINVAL, "negative step count in state");
    if (hd.block_pos < 0 || hd.block_pos >= std::max(1, hd.block_len) ||
        (hd.block_pos != 0 && hd.block_len != h->block))
        return fail(LB_EINVAL, "state is inside a block of a different length");
    std::vector<double> forces(2 * (size_t)h->n_ch);
    size_t off = kStateHeader;
    for (int ci = 0; ci < h->n_ch; ++ci) {
        for (const Section &sec : state_sections(h, ci, hd.t)) {
            HIP_TRY(h, hipMemcpy2DAsync(h->ws + sec.ws_off, sec.ws_pitch, src + off,
                                        sec.row_bytes, sec.row_bytes, sec.rows,
                                        hipMemcpyDeviceToDevice, h->stream));
            off = align_up(off + sec.rows * sec.row_bytes, 256);
        }
        HIP_TRY(h, hipMemcpyAsync(&forces[2 * ci], src + off, 16, hipMemcpyDeviceToHost, meta));
        off = align_up(off + 2 * sizeof(double), 256);
    }
    // Split storage: the moments of step t-1 (the base of the stored
    // remainders) are the loaded density and velocity planes.
    for (int ci = 0; ci < h->n_ch; ++ci) {
        const ChanDev &c = h->plan.chans[ci];
        if (!c.off_mom)
            continue;
        const size_t pb = (size_t)c.np * sizeof(double);
        char *m = h->ws + c.off_mom + (size_t)((hd.t + 1) & 1) * 3 * pb;
        HIP_TRY(h, hipMemcpyAsync(m, h->ws + c.off_rho, pb, hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(h, hipMemcpyAsync(m + pb, h->ws + c.off_vel, 2 * pb, hipMemcpyDeviceToDevice,
                                  h->stream));
    }
    HIP_TRY(h, hipStreamSynchronize(meta));
    for (int ci = 0; ci < h->n_ch; ++ci) {
        if (!std::isfinite(forces[2 * ci]) || !std::isfinite(forces[2 * ci + 1]) ||
            (!h->plan.chans[ci].has_r && forces[2 * ci + 1] != 0.0)) {
            h->poisoned = true;
            return fail(LB_ESTATE, "state buffer carries an invalid force; handle poisoned");
        }
        h->plan.chans[ci].gx = forces[2 * ci];
        h->plan.chans[ci].gy = forces[2 * ci + 1];
        launch_set_force(h->d_chans, ci, forces[2 * ci], forces[2 * ci + 1], h->stream);
    }
    launch_tick(h->d_tcount, hd.t - h->t, h->stream);
    lb_status s = check_launch(h, "load_state");
    if (s != LB_OK)
        return s;
    h->t = hd.t;
    h->has_out = hd.t > 0;
    h->block_pos = hd.block_pos;
    return LB_OK;
}

}  // namespace

lb_status lb_load_state(lb_handle *h, const void *d_src)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    return load_state_impl(h, d_src, h->stream);
}

int32_t lb_max_chunks(const lb_handle *h, int32_t ch)
{
    if (!h || ch < 0 || ch >= h->n_ch)
        return 0;
    return h->plan.chans[ch].max_chunks;
}

lb_status lb_set_tiling(lb_handle *h, int32_t ch, int32_t n_chunks, int32_t nodes_per_lane)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (ch < 0 || ch >= h->n_ch)
        return fail(LB_EINVAL, "channel index out of range");
    ChanDev &c = h->plan.chans[ch];
    if (n_chunks < 1 || n_chunks > c.max_chunks)
        return fail(LB_EINVAL, "n_chunks must be in [1, lb_max_chunks]");
    if (nodes_per_lane != 1 && nodes_per_lane != 2 && nodes_per_lane != 4)
        return fail(LB_EINVAL, "nodes_per_lane must be 1, 2 or 4");
    c.nchunks = n_chunks;
    c.vec = nodes_per_lane;
    build_tiles(h);
    return upload_tables(h);
}

lb_status lb_get_tiling(const lb_handle *h, int32_t ch, int32_t *n_chunks,
                        int32_t *nodes_per_lane)
{
    if (!h || ch < 0 || ch >= h->n_ch)
        return fail(LB_EINVAL, "bad handle or channel index");
    if (n_chunks)
        *n_chunks = h->plan.chans[ch].nchunks;
    if (nodes_per_lane)
        *nodes_per_lane = effective_vec(h->plan.chans[ch].vec, h->block);
    return LB_OK;
}

lb_status lb_set_graph(lb_handle *h, int32_t steps_per_graph)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (steps_per_graph < 0 || steps_per_graph > 4096)
        return fail(LB_EINVAL, "steps_per_graph must be in [0, 4096]");
    if (steps_per_graph % h->block != 0)
        return fail(LB_EINVAL, "steps_per_graph must be a multiple of the block length");
    h->graph_steps = steps_per_graph;
    h->graph_dirty = true;
    return LB_OK;
}

lb_status lb_set_block(lb_handle *h, int32_t steps_per_pass)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (steps_per_pass != 1 && steps_per_pass != 2 && steps_per_pass != 4 &&
        steps_per_pass != 8 && steps_per_pass != 16 && steps_per_pass != 32)
        return fail(LB_EINVAL, "steps_per_pass must be 1, 2, 4, 8, 16 or 32");
    if (h->graph_steps % steps_per_pass != 0)
        return fail(LB_EINVAL, "the graph length must stay a multiple of the block length");
    for (const ChanDev &c : h->plan.chans)
        if (c.finger && steps_per_pass > kMaxFingerBlock)
            return fail(LB_EINVAL, "full-tensor channels take at most 16 steps per pass");
    h->block = steps_per_pass;
    h->block_pos = 0;  // the next step starts a block with a fresh pass
    h->graph_dirty = true;
    build_tiles(h);  // lane widths depend on the block length
    return upload_tables(h);
}

int32_t lb_get_block(const lb_handle *h) { return h ? h->block : 0; }

lb_status lb_set_fused(lb_handle *h, int32_t mode)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (mode < 0 || mode > 2)
        return fail(LB_EINVAL, "fused mode must be 0, 1 or 2");
    h->fuse_mode = mode;
    h->graph_dirty = true;
    return LB_OK;
}

lb_status lb_set_adjoint_block(lb_handle *h, int32_t steps)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (steps < 1 || steps > kAdjMaxBlock)
        return fail(LB_EINVAL, "adjoint block must be in [1, " + std::to_string(kAdjMaxBlock) +
                                   "]");
    if (steps != h->adj_block) {
        // the captured sweeps hold the old launch sequence; none may be in
        // flight when they are destroyed
        s = adj_drain(h);
        if (s != LB_OK)
            return s;
        drop_adj_graphs(h);
        h->adj_block = steps;
    }
    return LB_OK;
}

int32_t lb_get_adjoint_block(const lb_handle *h)
{
    return h ? adj_block_in_effect(h) : 0;
}

int32_t lb_get_fused(const lb_handle *h)
{
    if (!h || !fused_in_effect(h))
        return 0;
    return (h->fuse_mode == 1 && h->fuse_lds_ok && h->fuse_lds_ready) ? 2 : 1;
}

lb_status lb_set_persistent(lb_handle *h, int32_t enable)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    h->persistent = enable != 0;
    h->graph_dirty = true;
    return LB_OK;
}

lb_status lb_profile(lb_handle *h, int32_t enable)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    h->profile = enable != 0;
    // Enabling starts a fresh measurement.
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    s = resolve_timing(h);
    if (s != LB_OK)
        return s;
    for (int w = 0; w < 3; ++w) {
        h->kernel_ms[w] = 0.0;
        h->kernel_launches[w] = 0;
    }
    return LB_OK;
}

lb_status lb_kernel_time(lb_handle *h, int32_t which, double *total_ms, int64_t *launches)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (which < 0 || which > 2)
        return fail(LB_EINVAL, "which must be 0 (history pass), 1 (lattice) or 2 (block step)");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    s = resolve_timing(h);
    if (s != LB_OK)
        return s;
    if (total_ms)
        *total_ms = h->kernel_ms[which];
    if (launches)
        *launches = h->kernel_launches[which];
    return LB_OK;
}


lb_status lb_set_params(lb_handle *h, int32_t ch, double g_inf, double tau_m, double gamma_c)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (ch < 0 || ch >= h->n_ch)
        return fail(LB_EINVAL, "channel index out of range");
    if (!std::isfinite(g_inf) || g_inf < 0.0 || !std::isfinite(tau_m) || !(tau_m > 0.0) ||
        std::isnan(gamma_c) || !(gamma_c > 0.0))
        return fail(LB_EINVAL, "need g_inf >= 0, tau_m > 0 finite, gamma_c > 0 (or +inf)");
    ChanDev &c = h->plan.chans[ch];
    c.g_inf = g_inf;
    c.inv_tau = 1.0 / tau_m;
    c.inv_gc = std::isinf(gamma_c) ? 0.0 : 1.0 / gamma_c;
    c.l2_tau = M_LOG2E * c.inv_tau;
    c.l2_gc = M_LOG2E * c.inv_gc;
    // block sums already formed hold the old decay rates: start a new block
    h->block_pos = 0;
    launch_set_params(h->d_chans, ch, g_inf, tau_m, gamma_c, h->stream);
    return check_launch(h, "set_params");
}

size_t lb_adjoint_workspace_bytes(const lb_handle *h, int32_t seg_len)
{
    if (!h)
        return 0;
    std::string why = adjoint_unsupported(h, seg_len);
    if (!why.empty()) {
        g_err = why;
        return 0;
    }
    return adj_layout(h, seg_len, nullptr).total;
}

}  // extern "C"

namespace {

// Start a sweep on the adjoint workspace at aws (validated by the caller):
// lay it out, zero it with a fill kernel, upload the channel table.
lb_status adjoint_begin_at(lb_handle *h, char *aws, size_t bytes, int seg_len)
{
    const size_t need = adj_layout(h, seg_len, nullptr).total;
    if (bytes < need)
        return fail(LB_ENOMEM, "adjoint workspace too small: need " + std::to_string(need));
    lb_status s = adj_drain(h);  // an earlier sweep still reading the workspace
    if (s != LB_OK)
        return s;
    if (!h->adj_stream) {
        HIP_TRY(h, hipStreamCreateWithFlags(&h->adj_stream, hipStreamNonBlocking));
        HIP_TRY(h, hipStreamCreateWithFlags(&h->io_stream, hipStreamNonBlocking));
        HIP_TRY(h, hipEventCreateWithFlags(&h->adj_ev_replay, hipEventDisableTiming));
        HIP_TRY(h, hipEventCreateWithFlags(&h->adj_ev_input, hipEventDisableTiming));
        for (int b = 0; b < 2; ++b)
            HIP_TRY(h, hipEventCreateWithFlags(&h->adj_ev_sweep[b], hipEventDisableTiming));
    }
    const AdjLayout P = adj_layout(h, seg_len, h->achans.data());
    if (h->aws != aws || h->adj_seg_len != seg_len)
        drop_adj_graphs(h);  // they address the previous workspace
    h->aws = aws;
    h->aws_bytes = bytes;
    h->d_achans = reinterpret_cast<AdjChan *>(h->aws + P.off_table);
    h->d_adj_out = reinterpret_cast<double *>(h->aws + P.off_out);
    h->d_adj_t0 = reinterpret_cast<int64_t *>(h->aws + P.off_t0);
    h->d_adj_snap = reinterpret_cast<ChanDev *>(h->aws + P.off_snap);
    for (int b = 0; b < 2; ++b)
        h->d_adj_stage[b] = reinterpret_cast<double *>(h->aws + P.off_stage[b]);
    h->adj_seg_len = seg_len;
    h->adj_segments = 0;
    launch_fill_zero(h->aws, P.total, h->stream);
    s = check_launch(h, "adjoint zero fill");
    if (s != LB_OK)
        return s;
    HIP_TRY(h, hipMemcpyAsync(h->d_achans, h->achans.data(), h->achans.size() * sizeof(AdjChan),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->adj_next = h->t;
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_adjoint_begin(lb_handle *h, void *d_aws, size_t bytes, int32_t seg_len)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    std::string why = adjoint_unsupported(h, seg_len);
    if (!why.empty())
        return fail(LB_EINVAL, why);
    if (!d_aws || reinterpret_cast<uintptr_t>(d_aws) % 256 != 0)
        return fail(LB_ENOMEM, "adjoint workspace must be non-NULL and 256-byte aligned");
    return adjoint_begin_at(h, static_cast<char *>(d_aws), bytes, seg_len);
}

lb_status lb_adjoint_begin_noalloc(lb_handle *h, int32_t seg_len)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    std::string why = adjoint_unsupported(h, seg_len);
    if (!why.empty())
        return fail(LB_EINVAL, why);
    const size_t need = adj_layout(h, seg_len, nullptr).total;
    if (need > kScratchBytes)
        return fail(LB_ENOMEM, "adjoint workspace of " + std::to_string(need) +
                                   " bytes exceeds the library's " +
                                   std::to_string(kScratchBytes) + "-byte device array");
    if (!h->scratch)
        return fail(LB_EDEVICE, "the library's device array has no address on this GPU");
    return adjoint_begin_at(h, static_cast<char *>(h->scratch), kScratchBytes, seg_len);
}

namespace {

// lb_adjoint_segment after its dL/du_x upload is queued: the replay with
// step records on, the copies the sweep reads, and the sweep on the adjoint
// stream.  Returns without waiting for the upload (the caller does).
lb_status adjoint_segment_rest(lb_handle *h, int buf, int64_t t0, int n_steps,
                               size_t total_nodes)
{
    // Replay the segment on the handle's stream (beside the sweep of the
    // later segment on the adjoint stream); its lattice steps record their
    // input populations and stress into the step records.  The record
    // fields of the device channel table are set and cleared on the stream;
    // the host table keeps them at zero.
    launch_set_record(h->d_chans, h->d_achans, h->n_ch, h->aws, buf, t0, h->stream);
    lb_status s = check_launch(h, "adjoint record on");
    if (s != LB_OK)
        return s;
    s = lb_step(h, n_steps);
    launch_set_record(h->d_chans, h->d_achans, h->n_ch, nullptr, buf, 0, h->stream);
    lb_status s2 = check_launch(h, "adjoint record off");
    if (s != LB_OK)
        return s;
    if (s2 != LB_OK)
        return s2;
    // The segment's shear rates (ring rows t0 .. t0 + n_steps - 1, wrapping),
    // dL/du_x spread over the channels' planes, and the channel table into
    // the buffer, so the sweep reads nothing the next replay overwrites.
    const size_t RH = history_bytes(h->prec);
    size_t col = 0;
    for (int ci = 0; ci < h->n_ch; ++ci) {
        const ChanDev &c = h->plan.chans[ci];
        const AdjChan &a = h->achans[ci];
        const size_t rowb = (size_t)c.np * RH;
        const int H = c.n_hist;
        const int first = (int)(t0 % H);
        const int run1 = std::min(n_steps, H - first);
        HIP_TRY(h, hipMemcpyAsync(h->aws + a.off_recs[buf], h->ws + c.off_ring_s + first * rowb,
                                  (size_t)run1 * rowb, hipMemcpyDeviceToDevice, h->stream));
        if (run1 < n_steps)
            HIP_TRY(h, hipMemcpyAsync(h->aws + a.off_recs[buf] + (size_t)run1 * rowb,
                                      h->ws + c.off_ring_s, (size_t)(n_steps - run1) * rowb,
                                      hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(h, hipMemcpy2DAsync(h->aws + a.off_dldu[buf], (size_t)c.np * sizeof(double),
                                    h->d_adj_stage[buf] + col, total_nodes * sizeof(double),
                                    (size_t)c.n * sizeof(double), (size_t)n_steps,
                                    hipMemcpyDeviceToDevice, h->stream));
        col += (size_t)c.n;
    }
    ChanDev *snap = h->d_adj_snap + (size_t)buf * h->n_ch;
    HIP_TRY(h, hipMemcpyAsync(snap, h->d_chans, (size_t)h->n_ch * sizeof(ChanDev),
                              hipMemcpyDeviceToDevice, h->stream));
    launch_store_i64(h->d_adj_t0 + buf, t0, h->stream);
    s = check_launch(h, "adjoint segment start");
    if (s != LB_OK)
        return s;
    HIP_TRY(h, hipEventRecord(h->adj_ev_replay, h->stream));
    // Reverse sweep of the segment on the adjoint stream, after the replay:
    // one captured graph per segment length and buffer, the segment's first
    // step in device memory.
    HIP_TRY(h, hipStreamWaitEvent(h->adj_stream, h->adj_ev_replay, 0));
    if (n_steps <= kAdjGraphMaxSteps) {
        hipGraphExec_t exec = nullptr;
        s = adj_sweep_graph(h, n_steps, buf, &exec);
        if (s != LB_OK)
            return s;
        HIP_TRY(h, hipGraphLaunch(exec, h->adj_stream));
    } else {
        // longer segments launch directly (a graph of 2 n_steps nodes would
        // cost more to build than it saves)
        s = enqueue_adj_sweep(h, n_steps, buf, h->adj_stream, true);
        if (s != LB_OK)
            return s;
    }
    HIP_TRY(h, hipEventRecord(h->adj_ev_sweep[buf], h->adj_stream));
    h->adj_sweep_pending[buf] = true;
    return LB_OK;
}

}  // namespace

lb_status lb_adjoint_segment(lb_handle *h, const void *d_ckpt, const double *dL_dux,
                             int32_t n_steps)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (h->adj_next < 0)
        return fail(LB_ESTATE, "no adjoint sweep in progress (call lb_adjoint_begin)");
    if (n_steps < 1 || n_steps > h->adj_seg_len)
        return fail(LB_EINVAL, "n_steps must be in [1, seg_len]");
    if (!dL_dux)
        return fail(LB_EINVAL, "dL_dux is NULL");
    const int64_t want_end = h->adj_next;
    // the checkpoint's header and forces come over the io stream, so the
    // state copies queue behind the replay still running
    s = load_state_impl(h, d_ckpt, h->io_stream);
    if (s != LB_OK)
        return s;
    const int64_t t0 = h->t;
    if (t0 + n_steps != want_end) {
        h->poisoned = true;
        return fail(LB_ESTATE, "segment does not end where the previous one began; handle "
                               "poisoned");
    }
    // Record buffer of this segment; the sweep two segments back read it last.
    const int buf = h->adj_segments & 1;
    if (h->adj_sweep_pending[buf])
        HIP_TRY(h, hipStreamWaitEvent(h->stream, h->adj_ev_sweep[buf], 0));
    // dL/du_x (host [n_steps][sum of nodes]) crosses to the device first, in
    // one contiguous copy (a strided copy from pageable host memory goes row
    // by row); the call waits for this copy only, so the caller queues the
    // next segment while this one replays.
    size_t total_nodes = 0;
    for (const ChanDev &c : h->plan.chans)
        total_nodes += (size_t)c.n;
    HIP_TRY(h, hipMemcpyAsync(h->d_adj_stage[buf], dL_dux,
                              (size_t)n_steps * total_nodes * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
    const hipError_t rec = hipEventRecord(h->adj_ev_input, h->stream);
    if (rec != hipSuccess) {
        (void)hipStreamSynchronize(h->stream);  // the copy may still read dL_dux
        h->poisoned = true;
        return fail(LB_EDEVICE, std::string("adjoint segment input event: ") +
                                    hipGetErrorString(rec));
    }
    // The rest of the segment; on every way out of it, the caller's buffer
    // is released only once its copy has finished.
    const lb_status st = adjoint_segment_rest(h, buf, t0, n_steps, total_nodes);
    const hipError_t w = hipEventSynchronize(h->adj_ev_input);
    if (st != LB_OK)
        return st;
    if (w != hipSuccess) {
        h->poisoned = true;
        return fail(LB_EDEVICE, std::string("adjoint segment input copy: ") +
                                    hipGetErrorString(w));
    }
    h->adj_next = t0;
    h->adj_segments += 1;
    return LB_OK;
}

lb_status lb_adjoint_end(lb_handle *h, double *dL_dtheta)
{
    lb_status s = usable(h);
    if (s != LB_OK)
        return s;
    if (h->adj_next < 0)
        return fail(LB_ESTATE, "no adjoint sweep in progress");
    if (!dL_dtheta)
        return fail(LB_EINVAL, "dL_dtheta is NULL");
    // after every sweep, on the adjoint stream
    hipStream_t st = h->adj_stream ? h->adj_stream : h->stream;
    launch_adj_reduce(h->d_chans, h->n_ch, h->aws, h->d_achans, h->d_adj_out, st);
    s = check_launch(h, "adjoint reduce");
    if (s != LB_OK)
        return s;
    HIP_TRY(h, hipMemcpyAsync(dL_dtheta, h->d_adj_out, (size_t)h->n_ch * 4 * sizeof(double),
                              hipMemcpyDeviceToHost, st));
    s = adj_drain(h);
    if (s != LB_OK)
        return s;
    h->adj_next = -1;
    return LB_OK;
}

lb_status lb_destroy(lb_handle *h)
{
    if (!h)
        return fail(LB_EINVAL, "handle is NULL");
    if (h->graph_exec)
        (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph)
        (void)hipGraphDestroy(h->graph);
    drop_adj_graphs(h);
    if (h->adj_stream) {
        (void)hipStreamSynchronize(h->adj_stream);
        (void)hipStreamDestroy(h->adj_stream);
    }
    if (h->io_stream)
        (void)hipStreamDestroy(h->io_stream);
    if (h->adj_ev_replay)
        (void)hipEventDestroy(h->adj_ev_replay);
    if (h->adj_ev_input)
        (void)hipEventDestroy(h->adj_ev_input);
    for (int b = 0; b < 2; ++b)
        if (h->adj_ev_sweep[b])
            (void)hipEventDestroy(h->adj_ev_sweep[b]);
    if (h->cap_stream)
        (void)hipStreamDestroy(h->cap_stream);
    for (int w = 0; w < 3; ++w)
        for (auto &pr : h->pending[w]) {
            h->free_events.push_back(pr.first);
            h->free_events.push_back(pr.second);
        }
    for (hipEvent_t e : h->free_events)
        (void)hipEventDestroy(e);
    delete h;
    return LB_OK;
}

}  // extern "C"
