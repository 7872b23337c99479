/*
 * FP64 CPU oracle of the batched exact Gillespie step and its Gumbel-Softmax
 * straight-through adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  It is a plain, slow reference: one trajectory per
 * OpenMP thread, loops over steps and reactions, FP64 everywhere.  Only the
 * test suite, the package's smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or table with the HIP library.
 */
#ifndef SSA_ORACLE_H
#define SSA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One reaction network (Sec. 2 of the paper): N species, M channels.
 * reactant[2j], reactant[2j+1]: reactant species of channel j (-1 = none;
 * equal pair = homodimerisation).  Parameters theta = ln k (Sec. 4.1);
 * rate_index[j] picks the parameter of channel j.  stoich is the dense [M][N]
 * table of change vectors v_j.
 */
typedef struct orc_net {
    int32_t n_species;
    int32_t n_reactions;
    int32_t n_params;
    const int32_t *reactant;    /* [M*2] */
    const int32_t *rate_index;  /* [M] */
    const int32_t *stoich;      /* [M*N] */
} orc_net;

/* FINAL: final counts.  BINS: exact time averages over n_bins uniform bins of
 * [0, t_obs].  GRID: the path linearly interpolated between its event points
 * (t_k, X_k) at n_bins uniform grid times t_obs g / (n_bins - 1), held at its
 * last state after the last event (Sec. 4.1).  TAIL: the mean of each
 * observed count over the last m = n_bins states X_{n-m+1} .. X_n of an
 * n = n_steps step run, and as value n_obs the mean of their times t_k (the
 * quantities the oscillator's rate-of-change loss compares, Sec. 4.2); a run
 * that stops early holds its last state and clock over the remaining steps. */
enum { ORC_OBS_FINAL = 0, ORC_OBS_BINS = 1, ORC_OBS_GRID = 2, ORC_OBS_TAIL = 3 };

/* Channel selection of the forward: the Gumbel-max (exponential race) of
 * Sec. 3.2, or the standard direct method's inverse CDF (Sec. 2: the first j
 * whose cumulative propensity exceeds u a0), which has no straight-through
 * backward. */
enum { ORC_SELECT_GUMBEL_MAX = 0, ORC_SELECT_INVERSE_CDF = 1 };

typedef struct orc_cfg {
    uint64_t seed;
    uint32_t purpose;
    uint32_t epoch;
    int64_t n_steps;        /* fire at most this many reactions */
    double t_end;           /* fire only while t + tau <= t_end (INFINITY: no limit) */
    int32_t obs_kind;       /* ORC_OBS_FINAL, ORC_OBS_BINS or ORC_OBS_GRID */
    int32_t n_bins;         /* bins, or grid points */
    double t_obs;           /* bins split [0, t_obs] uniformly; the grid spans it */
    int32_t n_obs;
    const int32_t *obs_species;  /* [n_obs] */
    double temperature;     /* Gumbel-Softmax temperature T of Eq. (3) */
    double tie_threshold;   /* relative margin that counts as a near-tie (1e-6) */
    double clock_tol;       /* relative window |t + tau - t_end| <= clock_tol * t_end */
    int32_t selection;      /* ORC_SELECT_* */
    double edge_window;     /* bins: relative window around a bin edge inside which the adjoint
                               takes the GPU's side of the edge for an event time (0: off) */
} orc_cfg;

/* Per-trajectory overrides taken from the GPU's near-tie log.  For trajectory
 * q the entries ov_off[q] .. ov_off[q+1]-1 are sorted by step.
 * kind 0: reaction near-tie, val = reaction the GPU fired.
 * kind 1: clock near-tie at t_end, val = 1 if the GPU fired, 0 if it stopped.
 * kind 2: the event time of the step lies within the GPU's edge window of a bin
 *         edge; val = 1 if the GPU's clock put it at or after the edge.  With
 *         cfg->edge_window > 0 the adjoint assigns the event's clock-derivative
 *         term to the bin on that side (the derivative of a bin average with
 *         respect to an event time jumps at an edge).  An event of the oracle
 *         within half the window of an edge without such an entry, or an entry
 *         for an event farther than twice the window, counts in n_bad. */
typedef struct orc_overrides {
    const int64_t *off;     /* [n_traj+1] */
    const int64_t *step;
    const int32_t *kind;
    const int32_t *val;
} orc_overrides;

/* Per-trajectory diagnostics. */
typedef struct orc_stats {
    double *min_margin;     /* [n_traj] smallest relative margin seen (INFINITY if none) */
    int32_t *n_near;        /* [n_traj] steps with margin <= tie_threshold */
    int32_t *n_resync;      /* [n_traj] override steps where the GPU's choice was adopted */
    int32_t *n_bad;         /* [n_traj] override disagreements that are not near-ties */
    double *bin_edge_dist;  /* [n_traj] min |t_k - edge| over steps k>=1 and inner bin edges (bins only) */
} orc_stats;

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Lattice uniform of a 32-bit word: (2*(x>>9)+1) * 2^-24, in (0, 1). */
double orc_uniform(uint32_t x);

/* The first n_words uniforms of step `step` of trajectory `traj`.
 * Word w comes from block w/4 (lane w%4); block b uses counter
 * (b, step, traj, purpose<<24 | epoch) and key (lo32(seed), hi32(seed)). */
void orc_step_uniforms(uint64_t seed, uint32_t purpose, uint32_t epoch, uint32_t traj,
                       uint32_t step, int32_t n_words, double *u);

/* Forward simulation of n_traj trajectories (x0 and x_final are [n_traj][N]).
 * obs: [n_traj][n_bins][n_obs] bin averages or grid values, [n_traj][n_obs]
 * final counts, or [n_traj][n_obs + 1] tail means (counts, then the clock).
 * theta: [P] (FP32 values promoted).  ov and stats may be NULL.
 * Returns 0, or -1 on invalid arguments. */
int orc_forward(const orc_net *net, const orc_cfg *cfg, const double *theta,
                int64_t n_traj, const uint32_t *traj_ids, const int32_t *x0,
                const orc_overrides *ov,
                int32_t *x_final, double *t_final, int32_t *steps_done, double *obs,
                const orc_stats *stats, int n_threads);

/* Forward plus straight-through adjoint.  d_obs has the layout of obs;
 * grad receives the per-trajectory gradient dL/dtheta, [n_traj][P]. */
int orc_adjoint(const orc_net *net, const orc_cfg *cfg, const double *theta,
                int64_t n_traj, const uint32_t *traj_ids, const int32_t *x0,
                const orc_overrides *ov, const double *d_obs,
                int32_t *x_final, double *t_final, int32_t *steps_done, double *obs,
                double *grad, const orc_stats *stats, int n_threads);

/* orc_adjoint plus kappa [n_traj][P] (may be NULL): per trajectory and
 * parameter, the sum over steps of the magnitudes of the terms that make up
 * each step's gradient contribution (propagated through a magnitude adjoint),
 * the conditioning that bounds the rounding error of an evaluation of the
 * same recursion at lower precision. */
int orc_adjoint_kappa(const orc_net *net, const orc_cfg *cfg, const double *theta,
                      int64_t n_traj, const uint32_t *traj_ids, const int32_t *x0,
                      const orc_overrides *ov, const double *d_obs,
                      int32_t *x_final, double *t_final, int32_t *steps_done, double *obs,
                      double *grad, double *kappa, const orc_stats *stats, int n_threads);

/* Step-by-step record of one trajectory (at most cap steps):
 * X [(cap+1)][N], t [cap+1], tau [cap], j [cap], a [cap][M], u [cap][M+1],
 * margin [cap].  Returns the number of fired steps. */
int64_t orc_trace(const orc_net *net, const orc_cfg *cfg, const double *theta,
                  uint32_t traj_id, const int32_t *x0, int64_t cap,
                  int32_t *X, double *t, double *tau, int32_t *j, double *a,
                  double *u, double *margin);

#ifdef __cplusplus
}
#endif
#endif

#ifndef SSA_ORACLE_GRN_H
#define SSA_ORACLE_GRN_H
#ifdef __cplusplus
extern "C" {
#endif

/* Gene-regulatory network classifier (Sec. 4.3, Fig. 4A): fixed input factors
 * x (the n_in pixel intensities of an image), n_hid hidden genes H and n_out
 * output genes O, each gene switched ON with probability sigmoid(b + sum w x)
 * of its regulators.  Species order: H_0..H_{n_hid-1}, O_0..O_{n_out-1}.
 * Channels, in this order (channel j uses Philox word 1+j):
 *   hidden production  0 -> H_h  a = beta sigmoid(u_h),   u_h = b_h + sum_i W_hi x_i
 *   hidden decay       H_h -> 0  a = delta_h H_h,         delta_h = delta_min + exp(psi_h)
 *   output production  0 -> O_o  a = beta sigmoid(v_o),   v_o = c_o + sum_h U_oh H_h
 *   output decay       O_o -> 0  a = delta_o O_o,         delta_o = delta_min + exp(psi_{n_hid+o})
 * Parameters theta = [W (n_hid x n_in, row-major) | b (n_hid) | U (n_out x n_hid,
 * row-major) | c (n_out) | psi (n_hid + n_out)].
 * Observation: final counts of the output genes. */
typedef struct orc_grn {
    int32_t n_in, n_hid, n_out;
    double beta, delta_min;
} orc_grn;

/* Number of parameters, and the width of the compact per-trajectory gradient
 * [du (n_hid) | dU (n_out x n_hid) | dc (n_out) | dpsi (n_hid + n_out)],
 * where du_h = dL/du_h (= dL/db_h).  dL/dW_hi = sum over trajectories of
 * du_h x_i of the trajectory's image. */
int64_t orc_grn_n_params(const orc_grn *net);
int64_t orc_grn_n_compact(const orc_grn *net);

/* bfloat16 rounding (nearest even, NaN kept quiet) of an FP32 value. */
float orc_bf16(float x);

/* u[m][h] = b_h + sum_i bf16(W_hi) bf16(x_mi), the products and the sum exact
 * in FP64 (theta holds FP32 values; x_img [n_images][n_in] FP32 values). */
void orc_grn_hidden_input(const orc_grn *net, const double *theta, const double *x_img,
                          int64_t n_images, double *u);

/* Forward (and, if d_obs != NULL, the straight-through adjoint) of n_traj
 * trajectories; trajectory q runs on the hidden pre-activations
 * u_hid[image_of[q]] ([n_images][n_hid]).  cfg: seed, purpose, epoch, n_steps,
 * t_end, temperature, tie_threshold, clock_tol are used (obs is always the
 * final output counts).  x0, x_final [n_traj][n_hid+n_out];
 * obs, d_obs [n_traj][n_out]; grad_c [n_traj][orc_grn_n_compact]. */
int orc_grn_run(const orc_grn *net, const orc_cfg *cfg, const double *theta,
                const double *u_hid, int64_t n_traj, const uint32_t *traj_ids,
                const int32_t *image_of, const int32_t *x0, const orc_overrides *ov,
                const double *d_obs, int32_t *x_final, double *t_final, int32_t *steps_done,
                double *obs, double *grad_c, const orc_stats *stats, int n_threads);

/* Fired channels j [cap] and clock t [cap+1] of one trajectory (u_row: its
 * n_hid pre-activations).  Returns the number of fired steps. */
int64_t orc_grn_trace(const orc_grn *net, const orc_cfg *cfg, const double *theta,
                      const double *u_row, uint32_t traj_id, const int32_t *x0, int64_t cap,
                      int32_t *j, double *t);

/* Relaxed (soft) forward of Eq. 4 and its exact adjoint.  The state is real:
 * every step takes the soft sample y_j = softmax_j((ln a_j + G_j)/T) of Eq. 3
 * over the channels with a_j > 0 (same noise words as the hard forward,
 * G_j = -ln(-ln u_{1+j})) and moves X by sum_j y_j v_j; propensities are
 * evaluated at the real state, a decay channel of a gene at or below zero
 * having a_j = 0.  The clock advances by -ln(u_0)/a0.  Runs exactly n_steps
 * steps (production never stops); cfg->t_end must be infinite.
 * With d_obs, grad_c [n_traj][orc_grn_n_compact] receives the gradient of
 * sum_o d_obs[o] O_o(final) through the whole relaxed map (no stop-gradient).
 * x0, x_final [n_traj][N] real; obs [n_traj][n_out] the final output levels. */
int orc_grn_soft_run(const orc_grn *net, const orc_cfg *cfg, const double *theta, const double *u_hid,
                     int64_t n_traj, const uint32_t *traj_ids, const int32_t *image_of, const double *x0,
                     const double *d_obs, double *x_final, double *t_final, double *obs, double *grad_c,
                     int n_threads);

/* The relaxed path of one trajectory: X [(cap+1)][N] states, t [cap+1].
 * Returns the number of steps taken. */
int64_t orc_grn_soft_trace(const orc_grn *net, const orc_cfg *cfg, const double *theta, const double *u_row,
                           uint32_t traj_id, const double *x0, int64_t cap, double *X, double *t);

#ifdef __cplusplus
}
#endif
#endif
