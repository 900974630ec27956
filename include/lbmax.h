/*
 * lbmax.h -- C interface of the MI355X hybrid lattice-Boltzmann engine with
 * the integral nonlinear Maxwell (nlM) constitutive equation
 * (Papenkort & Voigtmann, arXiv:1504.06123).
 *
 * Problem statement the calls follow (Sec. I Eq. ns, Sec. II Eqs. gitt,
 * nlmax, nlM, Sec. III): an incompressible fluid in a planar channel --
 * x periodic, no-slip walls at y = -1/2 and y = ly - 1/2 -- driven by a body
 * force rho*g that is switched on (startup) or off (cessation), starting
 * from a stress-free rest state.  The Newtonian background viscosity
 * eta_inf is the BGK viscosity rho c_s^2 (tau_LB - 1/2); the structural
 * stress is the history integral of Eq. (gitt) with the modulus of
 * Eq. (nlmax), G_inf exp(-(t-t')/tau) exp(-(t-t')|gamma_dot(t')|/gamma_c),
 * evaluated in the simple-shear reduction (sigma_xy, N1 = sigma_xx -
 * sigma_yy, sigma_yy = 0) over a window of the last n_hist steps.  The
 * stress enters the lattice-Boltzmann update as the body force div(sigma),
 * lagged by one step.  Results returned: density, velocity, velocity
 * gradient kappa, sigma_xy and N1.
 *
 * Conventions shared by every call:
 *  - Lattice units: dt = dx = 1, rho_0 = 1.  Node index = y*lx + x; every
 *    host output array is FP64, [ly][lx] (x fastest), caller-owned.
 *  - Device memory is borrowed, never allocated: the caller allocates the
 *    workspace (lb_workspace_bytes) and state buffers (lb_state_bytes) and
 *    keeps them alive until lb_destroy.  The library never calls hipMalloc.
 *  - Work is ordered on the HIP stream given to lb_init.  lb_step only
 *    enqueues; readout calls (lb_fields, lb_stress, lb_grad) synchronise
 *    that stream before returning.  A handle is not thread-safe.
 *  - Readouts refer to the last completed step.  Before the first step they
 *    return LB_ESTATE.
 *  - Every call returns lb_status; no C++ exception crosses this boundary.
 *    lb_last_error() gives a thread-local message for the last failure.
 *    Invalid arguments are reported before any device work is enqueued and
 *    leave the handle unchanged.  After LB_EDEVICE the handle is poisoned:
 *    every later call except lb_destroy returns LB_ESTATE.
 */
#ifndef LBMAX_H
#define LBMAX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,     /* invalid argument; nothing was enqueued            */
    LB_ENOMEM = -2,     /* workspace or buffer too small / misaligned        */
    LB_EDEVICE = -3,    /* a HIP call failed; the handle is now poisoned     */
    LB_ESTATE = -4,     /* call not valid in the handle's current state      */
    LB_ENONFINITE = -5  /* a readout returned non-finite values (lb_set_checks) */
} lb_status;

/*
 * Arithmetic of the whole path.  In every mode the stress, velocity and
 * density planes are FP64, and so are the accumulated strain (prefix sum of
 * the shear rate, Sec. III Eq. eeval) and the combination of partial sums.
 *  LB_F64: populations, history ring and history sums in FP64.
 *  LB_F32: FP32 populations in split storage, FP32 history.  A stored
 *          post-collision population is the FP32 remainder
 *          n*_i - n^eq_i(rho, u) against the second-order equilibrium
 *          (Sec. III) of the moments its collision used, which are kept in
 *          FP64 (rho - 1, u_x, u_y per node and step parity); a pulled
 *          population is rebuilt in FP64 from its source node's moments and
 *          remainder.  The remainder is the forcing term plus
 *          (1 - 1/tau_LB) times the non-equilibrium part, so FP32 rounding
 *          acts on that small part only and the conserved moments carry no
 *          FP32 rounding from step to step (FP32 deviations n_i - a_i drift:
 *          a velocity that grows by a small amount per step loses part of
 *          each increment to FP32 rounding, coherently).  History ring in
 *          FP32; each window sum is formed as FP32 partial sums over groups
 *          of up to 128 rows, each added into a Kahan-compensated FP32 total
 *          (sum and compensation, read out as their FP64 difference).
 *  LB_F32_P64: populations as FP64 deviations n_i - a_i, history as in
 *          LB_F32.
 */
typedef enum { LB_F64 = 0, LB_F32 = 1, LB_F32_P64 = 2 } lb_precision;

/*
 * One channel.  Requirements (checked, LB_EINVAL otherwise):
 *   lx >= 1, ly >= 3, lx * ly <= 2^26 - 64, tau_lb > 1/2, n_hist >= 2 (unless the grid or law 2
 *   is used; with LB_F32 and LB_F32_P64 also n_hist <= 2^24, where entry
 *   ages are exact in FP32), g_inf >= 0, tau_m > 0,
 *   gamma_c > 0 (may be +INFINITY: the linear / UCM limit of Sec. II),
 *   all numbers finite except gamma_c = +INF.
 * g_inf = 0 gives a Newtonian fluid.  (gx, gy) is the body-force
 * acceleration; the force density is rho*g (Eq. ns).  u0, when not NULL,
 * is a host array [2][ly][lx] of initial velocities; the initial
 * populations are the equilibrium n^eq(rho = 1, u0) (NULL: rest).
 * A channel with lx == 1, gy == 0 and u0_y == 0 everywhere is
 * unidirectional: u_y stays zero, |gamma_dot| = |kappa_xy|, and its history
 * ring stores the shear rate only; lb_set_force rejects gy != 0 for it.
 *
 * History grid.  hist_blocks == 0: the history integral runs over a uniform
 * window of the last n_hist steps.  hist_blocks = B >= 1: it runs over the
 * quasi-logarithmic grid of Sec. III instead, B blocks of
 * C = hist_block_len entries (2 <= C, B <= 20, C * 2^B <= 2^30; n_hist is
 * then ignored).  Block b = 1..B has the time step 2^(B-b) (block B, the
 * newest, the LB step).  Each step a new entry enters block B; when a block
 * then holds C + 1 entries, its two oldest are combined (strains added,
 * velocity gradient averaged, |gamma_dot| taken from the averaged gradient)
 * into the newest entry of block b - 1, and block 1's combined entries are
 * dropped.  Before t = 0 every block is full of zero entries (rest).  The
 * integral uses the trapezoid rule on the entries' start times.  Such a
 * channel takes temporal blocking (lb_set_block) when C >= steps_per_pass + 2
 * (shorter blocks visit every entry every step), no window split, and no
 * adjoint.
 *
 * Stress tensor.  finger == 0: the simple-shear reduction of the Finger
 * tensor (sigma_xy = int s G, sigma_xx = int 2 s gamma G, sigma_yy = 0;
 * exact for unidirectional flow).  finger == 1: the full tensor of Eq. gitt,
 * -d_t'B(t, t') = E kappa(t') E^T + transpose with E(t, t') the ordered
 * product of exp(kappa dt) over the steps from t' to t - 1 (Eq. eeval);
 * sigma_yy enters the force and N1 = sigma_xx - sigma_yy.  Needs
 * hist_blocks == 0; blocks of at most 16 steps (lb_set_block); no adjoint.
 *
 * Stress coupling.  paper_coupling == 0: the stress of the previous step
 * enters as the body force div sigma (forcing term with the external force
 * rho*g + div sigma; mass conserved exactly).  paper_coupling == 1: the
 * paper's own forcing term, Eq. bodyforce in full -- the traceless part of
 * sigma^{t-1} in the second moment, the trace through the density rate
 * d_t delta rho = -(tr sigma^{t-1} - tr sigma^{t-2}) / (2 cs2),
 * rho = sum n + d_t delta rho / 2 and the external force rho*g only
 * (Eq. hydrofields).  No adjoint.
 *
 * Constitutive law.  law == 0: the integral nonlinear Maxwell model
 * (Eqs. gitt, nlmax).  law == 1: its variant of Sec. II with the
 * accumulated strain in the damping, G exp(-(t - t')/tau) exp(-R(t, t') /
 * gamma_c) with R the |gamma_dot| summed over the steps t', ..., t - 1.
 * law == 2: the instantaneous law, Eq. inlM read at time t: sigma_xy =
 * G tau_M s, N1 = 2 G tau_M^2 s^2, tau_M = 1/(1/tau + |gamma_dot|/gamma_c)
 * (no history; n_hist ignored).  Laws 1 and 2 need finger == 0 and
 * hist_blocks == 0, take no window split and no adjoint.
 */
typedef struct {
    int32_t lx, ly;
    double tau_lb;
    double g_inf, tau_m, gamma_c;
    int32_t n_hist;
    double gx, gy;
    const double *u0;
    int32_t hist_blocks, hist_block_len;
    int32_t finger;
    int32_t paper_coupling;
    int32_t law;
} lb_channel_desc;

typedef struct lb_handle lb_handle;

/* Bytes of device workspace needed for these channels (0 if the
 * description is invalid; lb_last_error says why).  Pure host call. */
size_t lb_workspace_bytes(const lb_channel_desc *ch, int32_t n_ch,
                          lb_precision prec);

/*
 * Create a handle for n_ch >= 1 channels advanced together (one launch per
 * phase covers every channel).  d_ws: device pointer, 256-byte aligned, at
 * least lb_workspace_bytes(...) bytes, owned by the caller.  stream: a
 * hipStream_t (NULL = default stream).  Enqueues the initialisation: the
 * initial populations, a zero history (rest before t = 0, Eq. maxwell),
 * zero stress.  On success *out receives the handle.
 */
lb_status lb_init(const lb_channel_desc *ch, int32_t n_ch, lb_precision prec,
                  void *d_ws, size_t ws_bytes, void *stream, lb_handle **out);

/* Change the body force of channel ch from the next step on (startup /
 * cessation, Sec. IV.B).  Stream-ordered. */
lb_status lb_set_force(lb_handle *h, int32_t ch, double gx, double gy);

/* Enqueue n_steps >= 0 time steps of every channel.  One step is: stream
 * and collide (BGK + forcing with rho*g + div sigma of the previous step,
 * Sec. III Eqs. bodyforce, hydrofields), velocity gradient, history push,
 * history integral (Eqs. gitt, nlmax) -> sigma. */
lb_status lb_step(lb_handle *h, int64_t n_steps);

/* Number of completed steps (host-side counter). */
int64_t lb_time(const lb_handle *h);

/*
 * Failure detection at readouts.  flags (default: both):
 *   LB_CHECK_FINITE: lb_fields, lb_stress and lb_grad return LB_ENONFINITE
 *     when a value they return is NaN or infinite (the run has diverged);
 *     the output arrays are still filled, and the handle stays usable.
 *   LB_CHECK_MACH: lb_fields raises LB_WARN_MACH when the channel's largest
 *     speed |u| exceeds 0.1 (lattice Mach number |u| / c_s above 0.17, with
 *     c_s = 1/sqrt(3) the D2Q9 speed of sound of Sec. III; the BGK scheme
 *     follows the incompressible equations of Sec. I only at small Mach
 *     number).  It is a warning: the call still returns LB_OK.
 * lb_warnings returns the warnings raised since its last call (bitmask) and
 * clears them; 0 for a NULL handle.
 */
enum { LB_CHECK_FINITE = 1, LB_CHECK_MACH = 2 };
enum { LB_WARN_MACH = 1 };
lb_status lb_set_checks(lb_handle *h, int32_t flags);
int32_t lb_warnings(lb_handle *h);

/* Density rho = sum n_i and velocity u = (j + f/2)/rho of the last
 * completed step (Sec. III Eq. hydrofields; with paper_coupling == 1, rho
 * includes d_t delta rho / 2).  Any pointer may be NULL.  Synchronises the
 * stream. */
lb_status lb_fields(lb_handle *h, int32_t ch, double *rho, double *ux,
                    double *uy);

/* sigma_xy and N1 = sigma_xx - sigma_yy of the last completed step: the
 * structural stress, the history integral of Eq. gitt with the modulus of
 * Eq. nlmax (or the law the channel takes), without the Newtonian background
 * eta_inf D of Eq. nlM; N1 is the first normal-stress difference of Sec. IV. */
lb_status lb_stress(lb_handle *h, int32_t ch, double *sxy, double *n1);

/* Velocity gradient kappa_ab = d_b u_a (kappa = (grad v)^T, Sec. I) of the
 * last completed step by second-order differences (Sec. III); out is
 * [4][ly][lx] ordered kxx, kxy, kyx, kyy. */
lb_status lb_grad(lb_handle *h, int32_t ch, double *kappa);

/*
 * State snapshot (checkpoint / resume).  lb_state_bytes gives the size of a
 * device buffer holding the full state; lb_save_state copies the state into
 * it (stream-ordered), lb_load_state restores it.  Layout (all sections
 * 256-byte aligned, R = double; RP = the population storage type: float for
 * LB_F32, double otherwise; RH = the history type: double for LB_F64, float
 * otherwise):
 *   header, 256 bytes: uint64 magic 0x4C424D4158535431, uint32 version = 6,
 *     uint32 precision, int64 t (completed steps), int32 n_ch,
 *     int32 reserved, uint64 total bytes, int32 block length,
 *     int32 block position (steps of the current block already done);
 *   then per channel, in order, N = lx*ly:
 *     pop  [9][N] RP post-collision populations of step t-1 minus the
 *                    weights a_i (LB_F32: minus the equilibrium n^eq_i of the
 *                    vel and drho sections instead); before the first step
 *                    the initial state shifted back by one streaming step.
 *                    Direction order q = 0..8: (0,0), (1,0), (-1,0), (0,1),
 *                    (0,-1), (1,1), (-1,-1), (1,-1), (-1,1).
 *     sig  [3][N] R  sigma_xy, sigma_xx, sigma_yy of step t-1
 *     vel  [2][N] R  u_x, u_y of step t-1 (before the first step: u0)
 *     drho [N]    R  rho - 1 of step t-1
 *     trp  [N]    R  tr sigma^{t-2} (used by the paper coupling; zero else)
 *     ring_s [n_hist][N] RH shear rate s(t') = kappa_xy, row t' mod n_hist
 *     ring_r [n_hist][N] RH |gamma_dot(t')| (absent for unidirectional
 *                           channels)
 *   (a full-tensor channel has instead ring [8][n_hist][N] RH: kappa_xx,
 *     kappa_xy, kappa_yx, kappa_yy of t', then exp(kappa(t') dt) - I
 *     row-major, each plane with row t' mod n_hist;
 *   a channel on the quasi-logarithmic grid has, instead of the two rings:
 *     grid_s [B][C][N] RH   averaged shear rate of each entry; block b-1
 *                           first, row (b-1)*C + (i mod C) for the i-th
 *                           entry the block ever held, counting its C
 *                           initial zero entries
 *     grid_r [B][C][N] RH   |gamma_dot| of the averaged gradient, and
 *     grid_d [3][B][C][N] RH  averaged 2 kappa_xx, kappa_xy + kappa_yx,
 *                           2 kappa_yy (both absent for unidirectional
 *                           channels))
 *     blk  [64][N] double   window sums of the block in progress (see
 *                           lb_set_block); read only when the block
 *                           position is not 0 ([96][N] for a full-tensor
 *                           channel; [64 + B][N] on the grid, the last B
 *                           planes the strain of each grid block's entries
 *                           held through the block, oldest grid block first)
 *     force  2 doubles: gx, gy.
 * Ring rows of times before t = 0 are zero.
 */
size_t lb_state_bytes(const lb_handle *h);
lb_status lb_save_state(lb_handle *h, void *d_dst);
lb_status lb_load_state(lb_handle *h, const void *d_src);

/*
 * Launch shaping (used by the autotuner).  lb_set_tiling sets, for channel
 * ch, the number of age ranges its history window is split into
 * (n_chunks in [1, lb_max_chunks(h, ch)]; the ranges are reduced by separate
 * workgroups and combined in FP64 in a fixed order) and the nodes each lane
 * of the history kernel owns (nodes_per_lane in {1, 2, 4}; one ring row is
 * then read as a 1-, 2- or 4-wide vector; with temporal blocking of 2 or 4
 * steps at most 2 are used, with 8 or more steps 1).  lb_get_tiling reads the
 * lane width in use and the chunk count.  lb_set_graph(h, s) replays s steps per hipGraph launch inside
 * lb_step (0 = plain launches).  All take effect at the next lb_step; only
 * the chunk split changes results, and only through rounding order.
 */
int32_t lb_max_chunks(const lb_handle *h, int32_t ch);
lb_status lb_set_tiling(lb_handle *h, int32_t ch, int32_t n_chunks,
                        int32_t nodes_per_lane);
lb_status lb_get_tiling(const lb_handle *h, int32_t ch, int32_t *n_chunks,
                        int32_t *nodes_per_lane);
lb_status lb_set_graph(lb_handle *h, int32_t steps_per_graph);

/*
 * Temporal blocking of the history integral.  Every history entry except
 * the newest is known one step ahead, so one pass over the history ring can
 * form the window sums of steps_per_pass (1, 2, 4, 8, 16 or 32) consecutive steps;
 * the following steps of the block add only the entries pushed since the
 * pass and shift the accumulated strain by the strain since the pass, which
 * enters the normal-stress sum affinely (Sec. III Eq. eeval: gamma(t,t') is a
 * sum of the shear rate over [t', t)).  On the quasi-logarithmic grid the
 * pass covers the entries each grid block holds through the whole block with
 * unchanged neighbours; the steps of the block visit the rest (the entries
 * received, combined away, or at a grid block's ends).  Results differ from unblocked
 * stepping only by rounding order.  A change takes effect at the next step
 * (which starts a new block); the graph length (lb_set_graph) must be a
 * multiple of it.  Default 1.
 */
lb_status lb_set_block(lb_handle *h, int32_t steps_per_pass);
int32_t lb_get_block(const lb_handle *h);

/*
 * Fused in-block steps.  When every channel of the handle has a uniform
 * window (hist_blocks == 0, law != 2) and at most 1024 nodes, the steps of a
 * block after its history pass run as one launch: one workgroup per channel
 * advances the lattice and the history of all those steps, with workgroup
 * barriers in place of kernel boundaries.  If moreover the handle is LB_F32
 * and every channel is unidirectional and takes the simple-shear integral law
 * (law == 0, finger == 0) with the body-force coupling (paper_coupling == 0),
 * the workgroup keeps the channel's populations (rebuilt in FP64 from the
 * split storage once per node and step), velocity and stress in LDS and the
 * history rows pushed since the pass in registers (the stencils then read no
 * global memory).  mode: 0
 * separate launches, 1 fused (the default: the LDS form where it applies,
 * else the global-memory form when every channel has at most 512 nodes;
 * wider, that form is slower than separate launches and the steps run
 * separately), 2 fused without the LDS form whenever the channels fit.
 * Results are identical in every mode.
 * lb_get_fused returns 0 when the steps are not fused (mode 0, a channel
 * that does not qualify, or blocks of one step), 1 for the fused launch, 2
 * for its LDS form.  Takes effect at the next lb_step.  For lb_kernel_time a
 * fused launch counts as one in-block launch.
 */
lb_status lb_set_fused(lb_handle *h, int32_t mode);
int32_t lb_get_fused(const lb_handle *h);

/*
 * Persistent history pass (enable != 0): instead of one workgroup per tile,
 * as many workgroups as are resident on the chip at once claim tiles from a
 * device counter, longest age range first, until all channels' tiles are
 * done -- one launch balances many uneven channels.  Results are identical
 * to the plain launch.  Default off.
 */
lb_status lb_set_persistent(lb_handle *h, int32_t enable);

/*
 * Per-kernel timing with HIP events recorded on the handle's stream around
 * every history pass (which = 0, including the chunk combine), every lattice
 * launch (which = 1) and every in-block history step (which = 2).  Enabled by lb_profile(h, 1) for plain launches;
 * lb_kernel_time returns the accumulated milliseconds and launch count and
 * synchronises the stream.
 */
lb_status lb_profile(lb_handle *h, int32_t enable);
lb_status lb_kernel_time(lb_handle *h, int32_t which, double *total_ms,
                         int64_t *launches);

/*
 * Material parameters of channel ch from the next step on (G_inf, tau,
 * gamma_c of Eq. nlmax; same validity rules as lb_channel_desc).  The next
 * step starts a new block (see lb_set_block) with a fresh history pass.
 */
lb_status lb_set_params(lb_handle *h, int32_t ch, double g_inf, double tau_m,
                        double gamma_c);

/*
 * Discrete adjoint of the stepping, for gradients of a loss of the sampled
 * velocities with respect to (G_inf, tau, gamma_c, g_x) of every channel.
 * Supported for unidirectional channels (lx = 1, gy = 0, u0_y = 0): there
 * d/dx vanishes, sigma_xx never reaches the force and |gamma_dot| = |s|, so
 * the transpose involves sigma_xy only (Sec. IV.C: normal stresses do not
 * feed back in translation-invariant flow).  The transpose of every step of
 * lb_step is applied in reverse time: collision, forcing and moments, the
 * stress divergence, the velocity gradient, and the history integral, whose
 * transpose gathers, for each history entry, the adjoint stresses of the
 * n_hist steps that saw it.
 *
 * Protocol (checkpointing): during the forward run save a state with
 * lb_save_state every seg_len steps (at most n_hist; the force must stay
 * constant inside a segment).  After the last step, call
 *   lb_adjoint_begin(h, aws, bytes, seg_len)   -- aws: caller-owned device
 *       buffer of lb_adjoint_workspace_bytes(h, seg_len) bytes, 256-aligned;
 *       the sweep will cover the steps before the current step count;
 * then, for the segments from last to first,
 *   lb_adjoint_segment(h, ckpt, dL_dux, n_steps)  -- ckpt: the state saved
 *       at the segment's first step; the segment must end where the previous
 *       call began; dL_dux: host array [n_steps][sum of lx*ly over channels]
 *       of dL/du_x for each step of the segment (zero where the loss does
 *       not sample), channels concatenated in order.  The segment is
 *       replayed from ckpt (overwriting the forward state) and swept back;
 * and finally
 *   lb_adjoint_end(h, dL_dtheta)  -- host [n_ch][4]: dL/dG_inf, dL/dtau,
 *       dL/dgamma_c, dL/dg_x, summed over the covered steps.
 * Accumulation is per node in FP64 and reduced in node order (bitwise
 * reproducible).  Arithmetic of the transposes: the handle's precision, with
 * the history gather in FP64.  The reverse sweep of a segment of up to 1024
 * steps is captured once per segment length as a HIP graph and replayed for
 * later segments and sweeps with the same adjoint workspace and seg_len
 * (lb_adjoint_begin with another buffer or seg_len drops the graphs;
 * lb_destroy frees them); longer segments launch their kernels directly.
 *
 * Streams: lb_adjoint_segment returns once dL_dux has been copied to the
 * device, so dL_dux may be reused at once; the segment's replay runs on in
 * the handle's stream, so ckpt must stay unchanged until lb_adjoint_end
 * returns.  The checkpoint's header and forces are read over a third stream,
 * so the next segment's state copies queue behind the replay in flight.
 * The segment's reverse sweep runs on a second stream; both streams are
 * created at the first lb_adjoint_begin (default priority; destroyed by
 * lb_destroy).  The sweep is ordered against the replays by events and
 * reads records that are double-buffered in the adjoint workspace, so it
 * overlaps the replay of the next segment.  lb_adjoint_end waits for the
 * last sweep.  The workspace must stay allocated until lb_adjoint_end.
 *
 * Against a single call per segment that takes (t0, t1, sample_every) and
 * returns the accumulated gradient: the segment's range follows from the
 * call order and the checkpoint's step count, dL_dux holds every step of the
 * segment (zeros where the loss does not sample, so any sampling pattern is
 * expressed), and the gradient is reduced once, at lb_adjoint_end.
 */
size_t lb_adjoint_workspace_bytes(const lb_handle *h, int32_t seg_len);
lb_status lb_adjoint_begin(lb_handle *h, void *d_aws, size_t bytes, int32_t seg_len);

/*
 * lb_adjoint_begin for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the adjoint workspace is the library's own static device array of 64 MiB,
 * one per GPU (the GPU current at lb_init), held until the process ends.
 * Allocates nothing, on the device or through any library.  Returns
 * LB_ENOMEM, with nothing enqueued, when lb_adjoint_workspace_bytes(h,
 * seg_len) exceeds 64 MiB.  The array is shared by every handle on that GPU
 * and keeps the last sweep's contents (each begin clears what must start at
 * zero); sweeps that overlap on one GPU -- two handles between their
 * lb_adjoint_begin_noalloc and lb_adjoint_end at once -- race and give wrong
 * gradients, so callers run them one at a time.  The rest of the protocol
 * (lb_adjoint_segment, lb_adjoint_end) is unchanged.
 */
lb_status lb_adjoint_begin_noalloc(lb_handle *h, int32_t seg_len);
lb_status lb_adjoint_segment(lb_handle *h, const void *d_ckpt, const double *dL_dux,
                             int32_t n_steps);
lb_status lb_adjoint_end(lb_handle *h, double *dL_dtheta);

/*
 * Form of the reverse sweep.  steps = 1: two launches per reverse step, the
 * history transpose (for the entry of that step, a gather over all n_hist
 * ages of the adjoint stresses) and the lattice part.  steps = M > 1
 * (default 32, at most 32): the sweep goes in blocks of M reverse steps, the
 * temporal blocking of the forward pass applied to the transpose.  Each
 * entry's window is summed in fixed parts: ages 0 .. 31, then 16 ranges that
 * split the rest.  One pass sums the far ranges for the M entries of a block
 * (they reach adjoint stresses of later steps, all in the adjoint ring when
 * the block starts); one launch of one workgroup per channel then runs the
 * block's steps -- the near ages and the lattice part -- with workgroup
 * barriers where the per-step form has launch boundaries.  Applies when
 * every channel has at most 512 nodes (wider, the per-step kernels are
 * faster); otherwise the sweep runs per step.
 * The gradients of the blocked form do not depend on M or on the segment
 * lengths, bit for bit; they agree with the per-step form up to the order of
 * the FP64 history sums.  Takes effect at the next lb_adjoint_segment; a
 * change waits for the sweeps in flight and drops the captured sweeps.
 * Returns LB_EINVAL for steps outside [1, 32].  lb_get_adjoint_block returns
 * the form in effect (1 where the blocked form does not apply, 0 for a NULL
 * handle).
 */
lb_status lb_set_adjoint_block(lb_handle *h, int32_t steps);
int32_t lb_get_adjoint_block(const lb_handle *h);

/* Release host-side handle memory.  Device memory stays the caller's. */
lb_status lb_destroy(lb_handle *h);

/* Thread-local message of the last failed call ("" if none). */
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMAX_H */
