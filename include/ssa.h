/*
 * ssa.h — C ABI of libssa: the massively batched exact Gillespie step and its
 * Gumbel-Softmax straight-through backward on AMD Instinct MI355X (gfx950).
 *
 * What the library computes (paper: "Exact Discrete Stochastic Simulation
 * with Deep-Learning-Scale Gradient Optimization", Vilar & Saiz):
 *   Forward (Sec. 2, Sec. 3.2, Eq. 6): for every trajectory, repeat
 *     a_j = k_j h_j(X) (mass action, Sec. 2), a0 = sum_j a_j,
 *     tau = -ln(u_0)/a0, j* = argmax_j [ln a_j + G_j] with G_j = -ln(-ln u_{1+j}),
 *     X += v_{j*}, t += tau,
 *   and record an observation of the path (exact bin time averages, Sec. 4.4,
 *   or the final counts).
 *   Backward (Sec. 3.1, Sec. 3.3-3.4, Eqs. 3-7, Fig. 1): gradient of a loss
 *   L(obs) with respect to theta = ln k (Sec. 4.1) through the
 *   straight-through surrogate: the forward's noise is regenerated from the
 *   counter-based random stream, soft samples y~ = softmax((ln a + G)/T) carry
 *   the selection gradient and the reparameterised waiting time carries the
 *   clock gradient.
 *
 * Random stream: Philox4x32-10 (Salmon et al., SC'11).  Word w of step k of
 * trajectory id i is lane w%4 of the block with counter
 * (w/4, k, i, purpose<<24 | epoch) and key (lo32(seed), hi32(seed)); it maps
 * to u = (2*(x>>9)+1)*2^-24.  Word 0 drives tau, word 1+j channel j.
 *
 * Memory: unless stated otherwise, array arguments of ssa_forward,
 * ssa_backward and ssa_step_batch are DEVICE pointers owned by the caller.
 * Those calls never allocate, free or synchronise: all work is enqueued on
 * `stream`, so they can be captured into a HIP graph.  Host-side argument
 * errors return before anything is enqueued.  The C ABI uses no C++ types and
 * throws nothing.
 *
 * Batches of networks: a network handle may hold several networks with
 * different species, channel and trajectory counts.  Network n owns
 * N_n species, M_n channels, P_n parameters, B_n trajectories and n_obs_n
 * observed species.  Arrays are packed network after network:
 *   theta / d_params   float  [sum P_n]            (slice at param_offset[n])
 *   x0 / x_final       int32  [sum N_n*B_n]        (block [N_n][B_n], species-major)
 *   t_final            double [sum B_n]
 *   steps_done         int32  [sum B_n]
 *   obs / d_obs        double [sum W_n*B_n]        (block [W_n][B_n], or [B_n][W_n] with
 *                       SSA_OBS_TRAJ_MAJOR; W_n = n_bins*n_obs_n as [point][obs] for bins
 *                       and grids, n_obs_n for final counts, n_obs_n + 1 for tail means;
 *                       [sum W_n] with SSA_OBS_ENSEMBLE_MEAN)
 *   ensemble means     double [sum W_n]            (ssa_obs_mean; a shared d_obs)
 *   d_params_per_traj  float  [sum P_n*B_n]        (block [P_n][B_n])
 * ssa_net_layout() returns every offset.
 */
#ifndef SSA_H
#define SSA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ssa_status {
    SSA_OK = 0,
    SSA_EINVAL = -1,       /* bad argument (NULL, out of range, inconsistent sizes) */
    SSA_ESHAPE = -2,       /* network or batch shape the library cannot run */
    SSA_EWORKSPACE = -3,   /* a buffer is smaller than the size the library asked for */
    SSA_EOVERFLOW = -4,    /* device: a copy number left the int32 range */
    SSA_ENONFINITE = -5,   /* device: a non-finite or negative propensity or clock */
    SSA_EHIP = -6,         /* a HIP runtime call failed */
    SSA_ENOTSUP = -7       /* valid request this build does not implement */
} ssa_status;

/* Observation kinds, per observed species o of a network with B trajectories:
 *   SSA_OBS_FINAL  obs[o][B]: the final counts.
 *   SSA_OBS_BINS   obs[b][o][B], b < n_bins: the exact time average of the
 *                  piecewise-constant path over bin b of n_bins uniform bins
 *                  of [0, t_obs] (the bin-averaged loss of Sec. 4.4).
 *   SSA_OBS_GRID   obs[g][o][B], g < n_bins: the path linearly interpolated
 *                  between its event points (t_k, X_k) at the grid time
 *                  t_obs g / (n_bins - 1), held at the last state after the
 *                  last event (the interpolated ensemble trajectories of
 *                  Sec. 4.1).  Runs in the topology-specialised lane mode
 *                  only: any other plan returns SSA_ENOTSUP. */
enum { SSA_OBS_FINAL = 0, SSA_OBS_BINS = 1, SSA_OBS_GRID = 2, SSA_OBS_TAIL = 3 };
/*   SSA_OBS_TAIL   obs[o][B] for o < n_obs: the mean of observed count o over
 *                  the last m = n_bins of the n_steps + 1 states X_0 .. X_n of
 *                  the run, and obs[n_obs][B]: the mean of their times t_k
 *                  (the per-segment rate of change of the start-point map,
 *                  Sec. 4.2, is (mean count - start count) / mean time).  A
 *                  trajectory that stops early (absorbing state, t_end) holds
 *                  its last state and clock over the remaining states.  Needs
 *                  a bounded n_steps, 1 <= n_bins <= n_steps, the point-major
 *                  layout with a per-trajectory d_obs, the Gumbel-max selection
 *                  and the topology-specialised lane mode (else SSA_ENOTSUP);
 *                  W_n = n_obs_n + 1, and ssa_net_layout returns its offsets. */

/* Channel selection of the forward:
 *   SSA_SELECT_GUMBEL_MAX   argmax_j ln a_j + G_j (Sec. 3.2), run as the exponential
 *                           race argmin_j E_j / a_j over words 1..M of the step;
 *   SSA_SELECT_INVERSE_CDF  the standard direct method (Sec. 2): the first j whose
 *                           cumulative propensity exceeds u_1 a0, with u_1 from word 1.
 *                           Forward only (ssa_backward returns SSA_ENOTSUP), final or bin
 *                           observations, topology-specialised lane mode only.  It is the
 *                           baseline of the selection-variant throughput comparison. */
enum { SSA_SELECT_GUMBEL_MAX = 0, SSA_SELECT_INVERSE_CDF = 1 };

/* Memory order of a network's observation block (obs of ssa_forward, d_obs of
 * ssa_backward):
 *   SSA_OBS_POINT_MAJOR  [W_n][B_n]: value w of every trajectory is contiguous;
 *   SSA_OBS_TRAJ_MAJOR   [B_n][W_n]: the W_n values of one trajectory are
 *                        contiguous.  Every trajectory then writes (and the
 *                        backward reads) whole cache lines of its own as it
 *                        crosses bins or grid points at its own pace.
 *                        Topology-specialised lane mode only (else SSA_ENOTSUP).
 * A loss of ensemble means (Sec. 4.1, Sec. 4.4) gives every trajectory of a
 * network the same dL/dobs; with dobs_shared set, ssa_backward reads d_obs as
 * that one block of W_n values per network (the ssa_obs_mean layout), whatever
 * obs_layout is.  Topology-specialised lane mode only. */
enum { SSA_OBS_POINT_MAJOR = 0, SSA_OBS_TRAJ_MAJOR = 1, SSA_OBS_ENSEMBLE_MEAN = 2 };
/* SSA_OBS_ENSEMBLE_MEAN: ssa_forward writes the ensemble means themselves
 * (the ssa_obs_mean layout, double [sum W_n]) and never stores the values of
 * single trajectories.  Each wave sums its trajectories' values in LDS with
 * integer additions: runs of whole bins as counts in difference arrays (exact),
 * the bins an interval or the tail only partly covers in fixed point with
 * 2^-32 resolution (the means carry at most 2^-33 absolute error from it).
 * Each 64-trajectory tile leaves one row of sums and the rows of a network are
 * reduced in a fixed order, so the result is the same on every call.  Bin and
 * grid observations (grid values are summed in the same fixed point, the held
 * tail as counts), topology-specialised lane mode, n_bins * n_obs <= 1000 and
 * 16 * n_bins * n_obs + 8 * n_obs <= 16384 (the LDS of one wave);
 * ssa_backward then needs dobs_shared.  Anything else returns SSA_ENOTSUP.
 * The sums are exact for observed counts below 2^25 (64 trajectories add into
 * one slot); a larger count is left out and raises the overflow flag that
 * ssa_device_status reports as SSA_EOVERFLOW. */

/* How ssa_backward obtains the fired channel of each step.
 *   SSA_BWD_TAPE:      ssa_forward stores the fired channel index of every
 *                      step in a compact tape (1, 2, 4 or 8 bits a step);
 *                      the backward sweeps each checkpoint segment in reverse
 *                      and regenerates noise, propensities and waiting times
 *                      from the Philox counters.
 *   SSA_BWD_RECOMPUTE: nothing per step is stored; the backward re-runs each
 *                      segment forward from its checkpoint to recover the
 *                      choices, then sweeps it in reverse.
 *   SSA_BWD_TANGENT:   forward-mode accumulation of the same straight-through
 *                      derivative (Eqs. 3-7): ssa_forward carries dX/d ln k_q
 *                      and dt/d ln k_q for every channel q along the path and
 *                      writes d obs / d ln k_q into the "checkpoint" buffer
 *                      ([point][obs][channel][B] per network, FP64, at
 *                      n_obs * M * B values per point and network; no
 *                      checkpoints or tape); ssa_backward contracts them with
 *                      d_obs, with no reverse sweep.  For batches in the
 *                      topology-specialised lane mode whose networks have at
 *                      most 4 channels and N * M <= 32, the final or bin
 *                      observation in the point-major layout with a
 *                      per-trajectory d_obs, step-limited runs (t_end =
 *                      INFINITY) and the Gumbel-max selection; otherwise
 *                      SSA_ENOTSUP.  The temperature is read by the forward.
 *   SSA_BWD_AUTO:      the library picks (tape). */
enum { SSA_BWD_AUTO = 0, SSA_BWD_TAPE = 1, SSA_BWD_RECOMPUTE = 2, SSA_BWD_TANGENT = 3 };

/* Host description of one or more networks (all pointers are HOST memory and
 * are copied by ssa_net_create).  Channel tables are packed network after
 * network; species indices are local to their network.
 *   reactant[2j], reactant[2j+1]: reactant species of channel j, -1 for none.
 *     (-1,-1): order 0, a = k;  (s,-1): a = k X_s;  (s,s'), s != s': a = k X_s X_s';
 *     (s,s): homodimerisation, a = k X_s (X_s - 1)/2   (Sec. 2).
 *   rate_index[j]: local parameter slot of channel j (tied rates allowed).
 *   stoich: dense change vectors, network n contributes M_n*N_n entries in
 *     [channel][species] order; every entry must be in [-8, 7].
 *   obs_species: local species observed, n_obs_n entries per network.
 *   t_obs: window of the bin or grid observation of each network (may be NULL if no
 *     run uses bins). */
typedef struct ssa_network_desc {
    int32_t n_networks;
    const int32_t *n_species;      /* [n_networks] */
    const int32_t *n_reactions;    /* [n_networks] */
    const int32_t *n_params;       /* [n_networks] */
    const int32_t *n_traj;         /* [n_networks] */
    const int32_t *n_obs;          /* [n_networks] */
    const int32_t *reactant;       /* [sum M_n * 2] */
    const int32_t *rate_index;     /* [sum M_n] */
    const int8_t *stoich;          /* [sum M_n * N_n] */
    const int32_t *obs_species;    /* [sum n_obs_n] */
    const double *t_obs;           /* [n_networks] bin or grid observations span [0, t_obs[n]] */
    int32_t exec_mode;             /* SSA_EXEC_*: how trajectories map onto lanes */
    int32_t wave_split;            /* wave mode: -1 library's choice, 0 one persistent launch
                                      for the whole batch, 1 one launch per lane-group width */
    int32_t wave_lanes;            /* wave mode: width cap, 8, 16, 32 or 64 lanes per trajectory
                                      (0: 64, the library's choice).  A network goes to the
                                      narrowest group of at most wave_lanes lanes in which each
                                      lane draws one Philox block (four channel words); one that
                                      needs more blocks runs on wave_lanes lanes drawing two
                                      blocks each; one that needs more than 2 wave_lanes blocks
                                      keeps the library's width.  Other values: SSA_EINVAL.  The
                                      fired channels do not depend on the width; clocks and
                                      gradients differ by the rounding order of group sums. */
} ssa_network_desc;

/* Execution modes.
 *   SSA_EXEC_SPEC: one trajectory per lane, kernels compiled at plan time for
 *                  each network topology (channel tables become constants);
 *                  networks up to 64 species and 64 channels, at most 16
 *                  distinct topologies per handle.
 *   SSA_EXEC_LANE: one trajectory per lane, generic kernels reading the tables
 *                  (up to 16 species and 32 channels).
 *   SSA_EXEC_WAVE: one trajectory per group of 8-64 lanes sharing its channels
 *                  (up to 64 species and 511 channels; the group width is
 *                  set by wave_lanes); persistent launches pulling
 *                  trajectories from a work counter in cost order.
 *   SSA_EXEC_AUTO: the library picks: SPEC when every network has at most 32
 *                  channels (larger ones compile for minutes and spill in
 *                  the specialised backward), else LANE for small batches,
 *                  else WAVE. */
enum { SSA_EXEC_AUTO = 0, SSA_EXEC_SPEC = 1, SSA_EXEC_LANE = 2, SSA_EXEC_WAVE = 3 };

typedef struct ssa_net ssa_net;    /* opaque handle: device-resident tables */

/* Offsets of network n inside the packed arrays (see the header comment). */
typedef struct ssa_net_layout_t {
    int64_t traj_offset;
    int64_t state_offset;
    int64_t param_offset;
    int64_t obs_offset;            /* for the observation kind and n_bins of the query */
    int64_t ppt_offset;            /* d_params_per_traj */
    int64_t mean_offset;           /* ensemble means / shared d_obs, same kind and n_bins */
} ssa_net_layout_t;

/* Run settings shared by forward, backward and step calls.
 * Set every field; ssa_config_default() fills sensible values. */
typedef struct ssa_config {
    uint64_t seed;
    uint32_t purpose;              /* stream domain: 0 simulate, 1 target, 2 pilot, ... */
    uint32_t epoch;                /* low 24 bits enter the counter */
    const uint32_t *d_epoch;       /* optional DEVICE scalar overriding epoch (graph replays) */
    const uint32_t *traj_ids;      /* optional DEVICE [sum B_n] global trajectory ids; NULL: 0..B-1 */
    int32_t n_steps;               /* fire at most this many channels per trajectory */
    double t_end;                  /* fire only while t + tau <= t_end; +INFINITY: no limit */
    int32_t obs_kind;              /* SSA_OBS_FINAL, SSA_OBS_BINS, SSA_OBS_GRID or SSA_OBS_TAIL */
    int32_t n_bins;                /* bins (>= 1) or grid points (>= 2) per observed species, or
                                      the tail length m of SSA_OBS_TAIL */
    float temperature;             /* Gumbel-Softmax temperature T of Eq. (3), > 0 */
    int32_t ckpt_every;            /* K: steps between state checkpoints (>= 1) */
    int32_t bwd_mode;              /* SSA_BWD_* */
    int32_t tie_capacity;          /* entries the near-tie log can hold */
    const float *d_temperature;    /* optional DEVICE scalar overriding temperature, read by the
                                      backward when it runs (annealing T under graph replay);
                                      it must then hold a finite value > 0.  NULL: temperature */
    int32_t selection;             /* SSA_SELECT_*: how the forward picks the channel */
    int32_t obs_layout;            /* SSA_OBS_POINT_MAJOR, SSA_OBS_TRAJ_MAJOR or SSA_OBS_ENSEMBLE_MEAN */
    int32_t dobs_shared;           /* nonzero: d_obs holds one dL/dobs block [W_n] per network */
    int32_t relaxed;               /* 1: the relaxed forward of Eq. 4 (Sec. 3.3) and the exact
                                      backward of that map, the first phase of the two-phase
                                      training (Sec. 3.5); gene-network runs only (SSA_ENOTSUP
                                      elsewhere).  0: the exact forward (default) */
} ssa_config;

/* One logged step where the selection (kind 0) or the t_end stop decision
 * (kind 1) was within the library's FP32 error of the alternative, or (kind 2)
 * where the event time fell close to a bin edge:
 * kind 0: relative gap of the two smallest E_j/a_j <= 2e-6;
 * kind 1: |t + tau - t_end| <= 1e-5 t_end, chosen = 1 if the step fired;
 * kind 2: bin observation, topology-specialised lane mode:
 *         |t + tau - e| <= 4e-7 e for the edge e = t_obs i / n_bins, i >= 1;
 *         chosen = 1 if t + tau >= e (the derivative of the bin averages with
 *         respect to this event time is taken on that side of the edge),
 *         second = i, margin = (t + tau - e) / e. */
typedef struct ssa_tie {
    uint32_t traj;                 /* packed trajectory index (not the global id) */
    uint32_t step;
    int32_t chosen;
    int32_t second;
    float margin;
    int32_t kind;
} ssa_tie;

void ssa_config_default(ssa_config *cfg);

/* Copies the description to the device and plans execution (allocates device
 * memory; call outside graph capture).  Returns SSA_ESHAPE for networks this
 * build cannot run. */
ssa_status ssa_net_create(const ssa_network_desc *desc, ssa_net **out);
void ssa_net_destroy(ssa_net *net);

/* Totals of a handle. */
ssa_status ssa_net_sizes(const ssa_net *net, int64_t *n_traj_total, int64_t *state_total,
                         int64_t *param_total, int64_t *n_networks);
ssa_status ssa_net_layout(const ssa_net *net, int32_t obs_kind, int32_t n_bins, int32_t network,
                          ssa_net_layout_t *out);

/* Device bytes the caller must provide:
 *   ckpt_bytes:  checkpoints and choice tape written by ssa_forward, read by
 *                ssa_backward (0 when cfg->n_steps is unbounded);
 *   work_bytes:  scratch for ssa_forward and ssa_backward. */
ssa_status ssa_buffer_sizes(const ssa_net *net, const ssa_config *cfg, size_t *ckpt_bytes,
                            size_t *work_bytes);

/* Forward simulation of every trajectory: the direct method of Sec. 2 with the
 * channel chosen by Gumbel-max (Sec. 3.2) or by the inverse CDF
 * (cfg->selection), the hard update of Eq. 6, and the path observed as
 * Sec. 4.1-4.4 describe.
 *   theta [sum P_n] (ln k, float), x0 (int32 state layout);
 *   out: x_final, t_final, steps_done, obs (may be NULL if n_obs = 0);
 *   ckpt: may be NULL (then no backward is possible);
 *   ties/n_ties: near-tie log (may be NULL); *n_ties counts every near-tie,
 *   entries beyond tie_capacity are dropped;
 *   work: work_bytes of scratch (the library clears what it needs).
 * Device-side faults (overflow, non-finite propensities) set sticky flags
 * that ssa_device_status() reports. */
ssa_status ssa_forward(const ssa_net *net, const ssa_config *cfg, const float *theta,
                       const int32_t *x0, int32_t *x_final, double *t_final,
                       int32_t *steps_done, double *obs, void *ckpt, size_t ckpt_bytes,
                       ssa_tie *ties, uint32_t *n_ties, void *work, size_t work_bytes,
                       hipStream_t stream);

/* Straight-through backward (Sec. 3.1, Sec. 3.3-3.4, Eqs. 3-7, Fig. 1): the
 * hard path of the forward with the gradient of the Gumbel-Softmax sample of
 * Eq. 3 at temperature cfg->temperature.  Inputs are the forward's inputs and outputs
 * (same cfg, theta, x0) and d_obs = dL/dobs (double, obs layout; with
 * cfg->dobs_shared, one block of W_n values per network at its mean_offset,
 * used for every trajectory of the network).
 *   d_params [sum P_n] float: overwritten with dL/dtheta (deterministic:
 *     per-trajectory FP64 partials reduced in a fixed order);
 *   d_params_per_traj: optional [sum P_n*B_n] per-trajectory gradients. */
ssa_status ssa_backward(const ssa_net *net, const ssa_config *cfg, const float *theta,
                        const int32_t *x0, const int32_t *x_final, const double *t_final,
                        const int32_t *steps_done, const void *ckpt, size_t ckpt_bytes,
                        const double *d_obs, float *d_params, float *d_params_per_traj,
                        void *work, size_t work_bytes, hipStream_t stream);

/* ssa_backward without a work buffer, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and kernels as ssa_backward,
 * minus work / work_bytes: the scratch lives in a file-scope device array of
 * the library, 32 MiB, one copy per GPU (resolved by ssa_net_create on the
 * handle's device and held until the process ends).  A configuration whose
 * work_bytes (ssa_buffer_sizes) exceed 32 MiB returns SSA_EWORKSPACE before
 * anything is enqueued.  Nothing is allocated or freed.  All calls on one GPU
 * share the array, and each call overwrites it: calls that overlap on one GPU
 * (concurrent streams, or host threads without ordering) race and must be
 * serialised by the caller.  The backward writes every value it reads back
 * from the scratch, so no clearing between calls is needed. */
ssa_status ssa_backward_static(const ssa_net *net, const ssa_config *cfg, const float *theta,
                               const int32_t *x0, const int32_t *x_final, const double *t_final,
                               const int32_t *steps_done, const void *ckpt, size_t ckpt_bytes,
                               const double *d_obs, float *d_params, float *d_params_per_traj,
                               hipStream_t stream);

/* One direct-method step (Sec. 2; the selection of Sec. 3.2 and the update of
 * Eq. 6, as in ssa_forward) with step index `step` for every trajectory, for step-wise
 * inspection.  x (state layout) and t [sum B_n] are updated in
 * place for trajectories that fire.  chosen [sum B_n]: fired channel, -1 if
 * a0 = 0, -2 if the step would pass t_end.  tau [sum B_n] float.
 * a: optional [sum M_n*B_n] propensities (block [M_n][B_n]). */
ssa_status ssa_step_batch(const ssa_net *net, const ssa_config *cfg, const float *theta,
                          int32_t *x, double *t, uint32_t step, int32_t *chosen, float *tau,
                          float *a, hipStream_t stream);

/* Ensemble mean of an observation buffer (the statistic the losses of
 * Sec. 4.1 and Sec. 4.4 compare): mean[mean_offset_n + w] = the average over
 * the B_n trajectories of network n of value w < W_n, for the obs_kind,
 * n_bins and obs_layout of cfg.  Each network is summed in FP64 in a fixed
 * order (chunks of trajectories, then the chunks in index order), so the
 * result is the same on every call; a network without trajectories gets 0.
 *   obs: DEVICE, the forward's layout; mean: DEVICE double [sum W_n];
 *   work: the work buffer of ssa_buffer_sizes for the same cfg (its contents
 *   are overwritten; do not share it with a concurrent forward or backward).
 * Enqueues on `stream` only (graph-capturable), any execution mode. */
/* (SSA_OBS_ENSEMBLE_MEAN observations are means already: SSA_EINVAL.) */
ssa_status ssa_obs_mean(const ssa_net *net, const ssa_config *cfg, const double *obs, double *mean,
                        void *work, size_t work_bytes, hipStream_t stream);

/* Sticky device flags raised since the handle was created (bit 0: overflow,
 * bit 1: non-finite propensity or clock).  Synchronises `stream`. */
ssa_status ssa_device_status(const ssa_net *net, hipStream_t stream, uint32_t *flags);

const char *ssa_status_string(ssa_status s);
/* Detail of the last failing call on this thread ("" if none). */
const char *ssa_last_error(void);

/* ------------------------------------------------------------------------
 * Gene-regulatory network classifier (Sec. 4.3, Fig. 4A).
 *
 * The pixels x of an image are fixed input factors.  Each of n_hid = 256
 * hidden genes H_h and n_out output genes O_o is ON with probability
 * sigmoid(bias + sum of weighted regulator levels) and produced at beta times
 * that probability; every gene decays at delta = delta_min + exp(psi), which
 * keeps the decay rate above delta_min.  Channels (word 1+j drives channel j):
 *   j = h                 0 -> H_h   a = beta sigmoid(u_h),  u_h = b_h + sum_i W_hi x_i
 *   j = n_hid + h         H_h -> 0   a = delta_h H_h
 *   j = 2 n_hid + o       0 -> O_o   a = beta sigmoid(v_o),  v_o = c_o + sum_h U_oh H_h
 *   j = 2 n_hid + n_out + o  O_o -> 0  a = delta_{n_hid+o} O_o
 * The contraction W x runs on bf16 matrix cores: W and x are rounded to
 * bfloat16 (nearest even), products are summed in FP32.  v_o is kept in FP64
 * and updated by +-U_oh whenever H_h changes.
 *
 * Layouts (device memory, caller-owned):
 *   theta, d_params  float  [P]: W [n_hid][n_in] | b [n_hid] | U [n_out][n_hid] |
 *                    c [n_out] | psi [n_hid + n_out],
 *                    P = n_hid*n_in + n_hid + n_out*n_hid + n_out + n_hid + n_out
 *   x_img            float  [n_images][n_in]
 *   u_hid            float  [n_images][n_hid]   (written by the forward)
 *   x0, x_final      int32  [n_hid + n_out][B]  (species-major; B = n_images*n_rep,
 *                    trajectory q runs image q / n_rep)
 *   t_final          double [B];  steps_done int32 [B]
 *   obs, d_obs       double [n_out][B]          (final output counts)
 *   d_compact        double [B][C], C = n_hid + n_out*n_hid + n_out + n_hid + n_out:
 *                    per trajectory [dL/du (n_hid) | dL/dU | dL/dc | dL/dpsi]
 *                    (dL/db = dL/du; dL/dW = sum_q dL/du_q bf16(x_{image q})^T)
 * Runs use cfg->seed, purpose, epoch, d_epoch, traj_ids, n_steps, temperature,
 * d_temperature, tie_capacity and relaxed; the observation is always the final
 * output counts, and cfg->t_end must be +INFINITY (SSA_ENOTSUP otherwise).
 *
 * Relaxed runs (cfg->relaxed = 1; Eq. 4, Sec. 3.3): the state is real and
 * every step moves it by sum_j y~_j v_j, the soft sample of Eq. 3 at the
 * forward's noise (temperature cfg->temperature, or *d_temperature), with a
 * decay channel of a gene at or below zero out of the sample.  obs receives
 * the final output levels (real), x_final their roundings to the nearest
 * integer; no near-ties are logged.  The tape buffer then holds the starting
 * point of every step, (n_steps + 1) rows of n_hid + 32 floats per trajectory
 * (ssa_grn_buffer_sizes reports it), and ssa_grn_backward returns the
 * gradient of the relaxed map itself (no stop-gradient).
 * ------------------------------------------------------------------------ */
typedef struct ssa_grn_desc {
    int32_t n_in;                  /* input factors per image (>= 1) */
    int32_t n_hid;                 /* hidden genes: 256 */
    int32_t n_out;                 /* output genes: 1..16 */
    int32_t n_images;              /* images per run */
    int32_t n_rep;                 /* trajectories per image */
    float beta;                    /* production rate of a gene that is ON (> 0) */
    float delta_min;               /* floor of every decay rate (>= 0) */
} ssa_grn_desc;

typedef struct ssa_grn ssa_grn;    /* opaque handle */

/* Validates the shape and allocates the handle's device status word. */
ssa_status ssa_grn_create(const ssa_grn_desc *desc, ssa_grn **out);
void ssa_grn_destroy(ssa_grn *grn);

/* Device bytes the caller provides: tape_bytes (fired channels, written by the
 * forward and read by the backward) and work_bytes (backward scratch). */
ssa_status ssa_grn_buffer_sizes(const ssa_grn *grn, const ssa_config *cfg, size_t *tape_bytes,
                                size_t *work_bytes);

/* Hidden pre-activations u_hid and the forward simulation of every
 * trajectory.  tape may be NULL (then no backward is possible); ties/n_ties
 * as for ssa_forward. */
ssa_status ssa_grn_forward(const ssa_grn *grn, const ssa_config *cfg, const float *theta,
                           const float *x_img, const int32_t *x0, float *u_hid,
                           int32_t *x_final, double *t_final, int32_t *steps_done, double *obs,
                           void *tape, size_t tape_bytes, ssa_tie *ties, uint32_t *n_ties,
                           hipStream_t stream);

/* Straight-through backward: overwrites d_params with dL/dtheta (per-trajectory
 * FP64 partials, summed per image and then over images in a fixed order; dW on
 * FP64 matrix cores).  d_compact (optional) receives the per-trajectory
 * partials.  Inputs are the forward's inputs and outputs with the same cfg. */
ssa_status ssa_grn_backward(const ssa_grn *grn, const ssa_config *cfg, const float *theta,
                            const float *x_img, const int32_t *x0, const float *u_hid,
                            const int32_t *x_final,
                            const int32_t *steps_done, const void *tape, size_t tape_bytes,
                            const double *d_obs, float *d_params, double *d_compact,
                            void *work, size_t work_bytes, hipStream_t stream);

/* Sticky device flags of the handle, as ssa_device_status.  Synchronises `stream`. */
ssa_status ssa_grn_device_status(const ssa_grn *grn, hipStream_t stream, uint32_t *flags);

/* Device primitives exposed for verification.
 * ssa_selftest_philox: n blocks; ctr_key [n][6] = (c0,c1,c2,c3,k0,k1), out [n][4].
 * ssa_selftest_neglog: out[i] = the library's FP32 -ln(u) for lattice point
 *   m = first + i, u = (2m+1) 2^-24, for count points (m < 2^23). */
ssa_status ssa_selftest_philox(const uint32_t *ctr_key, uint32_t *out, int64_t n,
                               hipStream_t stream);
ssa_status ssa_selftest_neglog(uint32_t first, int64_t count, float *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SSA_H */
