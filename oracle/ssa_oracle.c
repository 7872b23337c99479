/*
 * FP64 CPU oracle of the batched exact Gillespie direct method and its
 * Gumbel-Softmax straight-through adjoint.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg are its only users.  The product path never
 * loads it.  It shares no code with the HIP library; the two meet only in the
 * seeded input descriptions and in the published Philox4x32-10 definition,
 * which each side implements on its own.
 *
 * What is computed, and where the paper defines it:
 *   - Direct method (Sec. 2): propensities a_j(X), a0 = sum_j a_j,
 *     tau = -ln(u_0)/a0, fire one channel, X += v_j, t += tau.
 *   - Mass-action propensities (Sec. 2): k, k X_i, k X_i X_j, k X_i (X_i - 1)/2.
 *   - Channel selection by Gumbel-max (Sec. 3.2): argmax_j [ln a_j + G_j] with
 *     G_j = -ln(-ln u_j).  With E_j = -ln u_j this is argmin_j E_j / a_j, the
 *     same choice in exact arithmetic; the oracle takes that form in FP64.
 *   - Soft sample y~ = softmax((ln a + G)/T) (Eq. 3) and the straight-through
 *     construction (Eqs. 5-7): the forward fires the hard channel, the
 *     backward differentiates sum_j y~_j v_j with the forward's noise held
 *     fixed (Fig. 1 caption), plus the reparameterised waiting time
 *     d tau / d theta = -(tau/a0) d a0/d theta (Sec. 3.1).
 *   - Reverse recursion for dL/dX_k (Fig. 1 caption), extended with the clock
 *     adjoint dL/dt_k because the observation depends on event times.
 *   - Observation by exact time averages of the piecewise-constant path over
 *     uniform bins (Sec. 4.4), by the path linearly interpolated between its
 *     event points onto a uniform time grid (Sec. 4.1), or the final counts.
 * Readings where the paper is silent (random stream layout, uniform lattice,
 * tie handling, stop rules) are listed in the design notes of the repository.
 */
#include "ssa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: round multipliers and Weyl key increments as published.    */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)PHILOX_MUL_A * x0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * x2;
        uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)pb;
        uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)pa;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_WEYL_A;
        k1 += PHILOX_WEYL_B;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double orc_uniform(uint32_t x)
{
    return ((double)(2u * (x >> 9) + 1u)) * 0x1p-24;
}

void orc_step_uniforms(uint64_t seed, uint32_t purpose, uint32_t epoch, uint32_t traj,
                       uint32_t step, int32_t n_words, double *u)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int32_t b = 0; 4 * b < n_words; ++b) {
        uint32_t ctr[4] = {(uint32_t)b, step, traj, (purpose << 24) | (epoch & 0xFFFFFFu)};
        uint32_t r[4];
        orc_philox4x32_10(ctr, key, r);
        for (int l = 0; l < 4 && 4 * b + l < n_words; ++l)
            u[4 * b + l] = orc_uniform(r[l]);
    }
}

/* ------------------------------------------------------------------------ */
/* Propensities (Sec. 2, mass action).                                        */
/* ------------------------------------------------------------------------ */

/* Combinatorial factor h_j(X): a_j = k_j h_j(X). */
static double mass_action_h(const int32_t *rs, const int32_t *X)
{
    int s1 = rs[0], s2 = rs[1];
    if (s1 < 0) return 1.0;
    if (s2 < 0) return (double)X[s1];
    if (s1 == s2) return 0.5 * (double)X[s1] * ((double)X[s1] - 1.0);
    return (double)X[s1] * (double)X[s2];
}

/* dh_j/dX added into g with weight c. */
static void add_grad_h(const int32_t *rs, const int32_t *X, double c, double *g)
{
    int s1 = rs[0], s2 = rs[1];
    if (s1 < 0) return;
    if (s2 < 0) { g[s1] += c; return; }
    if (s1 == s2) { g[s1] += c * ((double)X[s1] - 0.5); return; }
    g[s1] += c * (double)X[s2];
    g[s2] += c * (double)X[s1];
}

/* d ln h_j/dX added into g with weight c (only called where h_j > 0). */
static void add_grad_log_h(const int32_t *rs, const int32_t *X, double c, double *g)
{
    int s1 = rs[0], s2 = rs[1];
    if (s1 < 0) return;
    if (s2 < 0) { g[s1] += c / (double)X[s1]; return; }
    if (s1 == s2) {
        double x = (double)X[s1];
        g[s1] += c * (2.0 * x - 1.0) / (x * (x - 1.0));
        return;
    }
    g[s1] += c / (double)X[s1];
    g[s2] += c / (double)X[s2];
}

/* |dh_j/dX| added into g with weight c >= 0 (magnitudes for the conditioning
 * sums of the adjoint; X >= 0). */
static void add_abs_grad_h(const int32_t *rs, const int32_t *X, double c, double *g)
{
    int s1 = rs[0], s2 = rs[1];
    if (s1 < 0) return;
    if (s2 < 0) { g[s1] += c; return; }
    if (s1 == s2) { g[s1] += c * fabs((double)X[s1] - 0.5); return; }
    g[s1] += c * (double)X[s2];
    g[s2] += c * (double)X[s1];
}

/* |d ln h_j/dX| added into g with weight c >= 0 (only where h_j > 0). */
static void add_abs_grad_log_h(const int32_t *rs, const int32_t *X, double c, double *g)
{
    int s1 = rs[0], s2 = rs[1];
    if (s1 < 0) return;
    if (s2 < 0) { g[s1] += c / (double)X[s1]; return; }
    if (s1 == s2) {
        double x = (double)X[s1];
        g[s1] += c * fabs(2.0 * x - 1.0) / (x * (x - 1.0));
        return;
    }
    g[s1] += c / (double)X[s1];
    g[s2] += c / (double)X[s2];
}

/* ------------------------------------------------------------------------ */
/* Observation helpers: exact bin averages of a piecewise-constant path.     */
/* ------------------------------------------------------------------------ */
static double bin_edge(const orc_cfg *cfg, int b)
{
    return cfg->t_obs * (double)b / (double)cfg->n_bins;
}

/* Bin holding time t (left-closed bins), or -1 if t is outside [0, t_obs). */
static int bin_of(const orc_cfg *cfg, double t)
{
    if (!(t >= 0.0) || t >= cfg->t_obs) return -1;
    int b = (int)floor(t * (double)cfg->n_bins / cfg->t_obs);
    if (b >= cfg->n_bins) b = cfg->n_bins - 1;
    while (b > 0 && t < bin_edge(cfg, b)) --b;
    while (b + 1 < cfg->n_bins && t >= bin_edge(cfg, b + 1)) ++b;
    return b;
}

/* For each bin b overlapping [t0, t1) call acc[b*n_obs + o] += weight(o) * overlap. */
static void add_interval(const orc_cfg *cfg, double t0, double t1, const double *val_per_obs,
                         double *acc)
{
    if (t1 > cfg->t_obs) t1 = cfg->t_obs;
    if (!(t0 < t1)) return;
    int b = bin_of(cfg, t0);
    if (b < 0) return;
    for (; b < cfg->n_bins; ++b) {
        double lo = bin_edge(cfg, b), hi = bin_edge(cfg, b + 1);
        if (lo >= t1) break;
        double ov = fmin(t1, hi) - fmax(t0, lo);
        if (ov > 0.0)
            for (int o = 0; o < cfg->n_obs; ++o)
                acc[(size_t)b * cfg->n_obs + o] += val_per_obs[o] * ov;
    }
}

/* ------------------------------------------------------------------------ */
/* Observation helpers: the path linearly interpolated on a uniform grid.    */
/* ------------------------------------------------------------------------ */
static double grid_time(const orc_cfg *cfg, int g)
{
    return cfg->t_obs * (double)g / (double)(cfg->n_bins - 1);
}

/* First grid index whose time is >= t (n_bins if none). */
static int grid_first_at_or_after(const orc_cfg *cfg, double t)
{
    int g = 0;
    while (g < cfg->n_bins && grid_time(cfg, g) < t) ++g;
    return g;
}

/* ------------------------------------------------------------------------ */
/* One trajectory.                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;          /* fired steps */
    int64_t cap;
    int32_t *X;         /* [(cap+1)*N] */
    double *t;          /* [cap+1] */
    double *tau;        /* [cap] */
    int32_t *j;         /* [cap] */
    double *E;          /* [cap*(M+1)]: E_0 for the clock, E_{1+j} for channel j */
} path_t;

static int path_reserve(path_t *p, int64_t need, int N, int M)
{
    if (need <= p->cap) return 0;
    int64_t c = p->cap ? p->cap : 1024;
    while (c < need) c *= 2;
    int32_t *X = realloc(p->X, sizeof(int32_t) * (size_t)(c + 1) * N);
    if (!X) return -1;
    p->X = X;
    double *t = realloc(p->t, sizeof(double) * (size_t)(c + 1));
    if (!t) return -1;
    p->t = t;
    double *tau = realloc(p->tau, sizeof(double) * (size_t)c);
    if (!tau) return -1;
    p->tau = tau;
    int32_t *j = realloc(p->j, sizeof(int32_t) * (size_t)c);
    if (!j) return -1;
    p->j = j;
    double *E = realloc(p->E, sizeof(double) * (size_t)c * (M + 1));
    if (!E) return -1;
    p->E = E;
    p->cap = c;
    return 0;
}

static void path_free(path_t *p)
{
    free(p->X); free(p->t); free(p->tau); free(p->j); free(p->E);
    memset(p, 0, sizeof(*p));
}

typedef struct {
    double min_margin;
    int32_t n_near, n_resync, n_bad;
    double edge_dist;
} traj_stats_t;

/* Optional per-step outputs of orc_trace. */
typedef struct {
    int64_t cap;
    int32_t *X; double *t; double *tau; int32_t *j; double *a; double *u; double *margin;
} trace_t;

/*
 * Simulates one trajectory.  Final state in X, final clock in *t_out.
 * obs_acc: [n_bins][n_obs] raw integrals (bins) or unused (final).
 * If path != NULL the whole path is kept for the adjoint.
 */
static int64_t simulate_one(const orc_net *net, const orc_cfg *cfg, const double *k,
                            uint32_t traj_id, int32_t *X, double *t_out,
                            const orc_overrides *ov, int64_t q,
                            double *obs_acc, path_t *path, trace_t *tr,
                            traj_stats_t *st, double *scratch)
{
    const int N = net->n_species, M = net->n_reactions;
    double *u = scratch;              /* [M+1] */
    double *a = scratch + (M + 1);    /* [M]   */
    double *xo = a + M;               /* [n_obs] */
    double t = 0.0;
    int64_t p_ov = ov ? ov->off[q] : 0, p_end = ov ? ov->off[q + 1] : 0;
    st->min_margin = INFINITY;
    st->n_near = st->n_resync = st->n_bad = 0;
    st->edge_dist = INFINITY;

    if (path) {
        if (path_reserve(path, 1, N, M)) return -1;
        memcpy(path->X, X, sizeof(int32_t) * N);
        path->t[0] = 0.0;
        path->n = 0;
    }
    if (tr && tr->cap >= 0) {
        memcpy(tr->X, X, sizeof(int32_t) * N);
        tr->t[0] = 0.0;
    }

    int64_t k_step = 0;
    for (; k_step < cfg->n_steps; ++k_step) {
        /* propensities and a0 (Sec. 2) */
        double a0 = 0.0;
        for (int j = 0; j < M; ++j) {
            a[j] = k[j] * mass_action_h(net->reactant + 2 * j, X);
            a0 += a[j];
        }
        if (!(a0 > 0.0)) break;                   /* absorbing state: frozen */

        orc_step_uniforms(cfg->seed, cfg->purpose, cfg->epoch, traj_id, (uint32_t)k_step,
                          M + 1, u);
        double E0 = -log(u[0]);
        double tau = E0 / a0;                     /* tau = -ln(u)/a0 (Sec. 2) */

        /* overrides recorded by the GPU for this step */
        int ov_clock = -1, ov_react = -1;
        while (p_ov < p_end && ov->step[p_ov] < k_step) ++p_ov;
        for (int64_t p = p_ov; p < p_end && ov->step[p] == k_step; ++p) {
            if (ov->kind[p] == 1) ov_clock = ov->val[p];
            else if (ov->kind[p] == 0) ov_react = ov->val[p];
        }

        /* stop rule: fire only while t + tau <= t_end */
        if (isfinite(cfg->t_end)) {
            int fire = (t + tau <= cfg->t_end);
            if (ov_clock >= 0 && ov_clock != fire) {
                if (fabs(t + tau - cfg->t_end) <= cfg->clock_tol * cfg->t_end) st->n_resync++;
                else st->n_bad++;
                fire = ov_clock;
            }
            if (!fire) break;
        }

        int jbest = -1;
        double margin = INFINITY;
        if (cfg->selection == ORC_SELECT_INVERSE_CDF) {
            /* direct method (Sec. 2): the first j with a_1 + ... + a_j > u_1 a0;
             * the margin is the relative distance of u_1 a0 from the nearest
             * interior cumulative boundary */
            const double target = u[1] * a0;
            int last = -1;
            for (int j = 0; j < M; ++j)
                if (a[j] > 0.0) last = j;
            double c = 0.0;
            for (int j = 0; j < M; ++j) {
                if (!(a[j] > 0.0)) continue;
                c += a[j];
                if (j != last) {
                    const double d = fabs(c - target) / a0;
                    if (d < margin) margin = d;
                }
                if (jbest < 0 && c > target) jbest = j;
            }
            if (jbest < 0) jbest = last;
        } else {
            /* exponential race: argmin_j E_j / a_j == argmax_j ln a_j + G_j (Sec. 3.2) */
            double r1 = INFINITY, r2 = INFINITY;
            for (int j = 0; j < M; ++j) {
                if (!(a[j] > 0.0)) continue;
                double r = -log(u[1 + j]) / a[j];
                if (r < r1) { r2 = r1; r1 = r; jbest = j; }
                else if (r < r2) { r2 = r; }
            }
            margin = isfinite(r2) ? (r2 - r1) / r1 : INFINITY;
        }
        if (margin < st->min_margin) st->min_margin = margin;
        if (margin <= cfg->tie_threshold) st->n_near++;
        if (ov_react >= 0 && ov_react != jbest) {
            if (ov_react < M && a[ov_react] > 0.0 && margin <= cfg->tie_threshold) {
                st->n_resync++;
                jbest = ov_react;
            } else {
                st->n_bad++;
                if (ov_react < M && a[ov_react] > 0.0) jbest = ov_react;
            }
        }

        /* observation of the interval [t, t + tau) at state X */
        if (cfg->obs_kind == ORC_OBS_BINS) {
            for (int o = 0; o < cfg->n_obs; ++o) xo[o] = (double)X[cfg->obs_species[o]];
            add_interval(cfg, t, t + tau, xo, obs_acc);
        }

        if (tr && k_step < tr->cap) {
            tr->tau[k_step] = tau;
            tr->j[k_step] = jbest;
            memcpy(tr->a + (size_t)k_step * M, a, sizeof(double) * M);
            memcpy(tr->u + (size_t)k_step * (M + 1), u, sizeof(double) * (M + 1));
            tr->margin[k_step] = margin;
        }
        if (path) {
            if (path_reserve(path, k_step + 1, N, M)) return -1;
            path->tau[k_step] = tau;
            path->j[k_step] = jbest;
            for (int w = 0; w <= M; ++w) path->E[(size_t)k_step * (M + 1) + w] = -log(u[w]);
        }

        /* grid times in [t, t + tau): linear interpolation between (t, X) and
         * (t + tau, X + v_j) */
        if (cfg->obs_kind == ORC_OBS_GRID) {
            const int32_t *vj = net->stoich + (size_t)jbest * N;
            for (int g = grid_first_at_or_after(cfg, t); g < cfg->n_bins; ++g) {
                const double tg = grid_time(cfg, g);
                if (!(tg < t + tau)) break;
                const double f = (tg - t) / tau;
                for (int o = 0; o < cfg->n_obs; ++o) {
                    const int s = cfg->obs_species[o];
                    obs_acc[(size_t)g * cfg->n_obs + o] = (double)X[s] + f * (double)vj[s];
                }
            }
        }

        /* fire: X += v_j (Eq. 6), t += tau */
        const int32_t *v = net->stoich + (size_t)jbest * N;
        for (int s = 0; s < N; ++s) X[s] += v[s];
        t += tau;

        /* state k_step + 1 of the run: one of the last n_bins states? */
        if (cfg->obs_kind == ORC_OBS_TAIL && k_step >= cfg->n_steps - cfg->n_bins) {
            for (int o = 0; o < cfg->n_obs; ++o) obs_acc[o] += (double)X[cfg->obs_species[o]];
            obs_acc[cfg->n_obs] += t;
        }
        if (cfg->obs_kind == ORC_OBS_BINS)
            for (int b = 1; b <= cfg->n_bins; ++b) {
                double d = fabs(t - bin_edge(cfg, b));
                if (d < st->edge_dist) st->edge_dist = d;
            }
        if (cfg->obs_kind == ORC_OBS_GRID)
            for (int g = 0; g < cfg->n_bins; ++g) {
                double d = fabs(t - grid_time(cfg, g));
                if (d < st->edge_dist) st->edge_dist = d;
            }
        if (path) {
            memcpy(path->X + (size_t)(k_step + 1) * N, X, sizeof(int32_t) * N);
            path->t[k_step + 1] = t;
            path->n = k_step + 1;
        }
        if (tr && k_step < tr->cap) {
            memcpy(tr->X + (size_t)(k_step + 1) * N, X, sizeof(int32_t) * N);
            tr->t[k_step + 1] = t;
        }
    }
    /* tail means: the states the run did not reach hold the last one */
    if (cfg->obs_kind == ORC_OBS_TAIL) {
        const int64_t k0 = cfg->n_steps - cfg->n_bins;
        const int64_t rem = cfg->n_steps - (k_step > k0 ? k_step : k0);
        if (rem > 0) {
            for (int o = 0; o < cfg->n_obs; ++o) obs_acc[o] += (double)rem * (double)X[cfg->obs_species[o]];
            obs_acc[cfg->n_obs] += (double)rem * t;
        }
    }
    /* the path is held at its last state up to t_obs */
    if (cfg->obs_kind == ORC_OBS_BINS) {
        for (int o = 0; o < cfg->n_obs; ++o) xo[o] = (double)X[cfg->obs_species[o]];
        add_interval(cfg, t, cfg->t_obs, xo, obs_acc);
    }
    if (cfg->obs_kind == ORC_OBS_GRID)
        for (int g = grid_first_at_or_after(cfg, t); g < cfg->n_bins; ++g)
            for (int o = 0; o < cfg->n_obs; ++o)
                obs_acc[(size_t)g * cfg->n_obs + o] = (double)X[cfg->obs_species[o]];
    *t_out = t;
    return k_step;
}

static int obs_width(const orc_cfg *cfg)
{
    if (cfg->obs_kind == ORC_OBS_TAIL) return cfg->n_obs + 1;
    return cfg->obs_kind == ORC_OBS_FINAL ? cfg->n_obs : cfg->n_bins * cfg->n_obs;
}

static void finish_obs(const orc_cfg *cfg, const int32_t *X, double *obs)
{
    if (cfg->obs_kind == ORC_OBS_GRID) return;
    if (cfg->obs_kind == ORC_OBS_TAIL) {
        for (int i = 0; i <= cfg->n_obs; ++i) obs[i] /= (double)cfg->n_bins;
        return;
    }
    if (cfg->obs_kind == ORC_OBS_BINS) {
        double inv = (double)cfg->n_bins / cfg->t_obs;
        for (int i = 0; i < cfg->n_bins * cfg->n_obs; ++i) obs[i] *= inv;
    } else {
        for (int o = 0; o < cfg->n_obs; ++o) obs[o] = (double)X[cfg->obs_species[o]];
    }
}

static int check_args(const orc_net *net, const orc_cfg *cfg)
{
    if (!net || !cfg || net->n_species <= 0 || net->n_reactions <= 0 || net->n_params <= 0)
        return -1;
    if (cfg->obs_kind == ORC_OBS_BINS && (cfg->n_bins <= 0 || !(cfg->t_obs > 0.0)))
        return -1;
    if (cfg->obs_kind == ORC_OBS_GRID && (cfg->n_bins < 2 || !(cfg->t_obs > 0.0)))
        return -1;
    if (cfg->obs_kind == ORC_OBS_TAIL &&
        (cfg->n_bins < 1 || cfg->n_steps < cfg->n_bins || cfg->n_steps > ((int64_t)1 << 40)))
        return -1;
    if (cfg->obs_kind < ORC_OBS_FINAL || cfg->obs_kind > ORC_OBS_TAIL) return -1;
    if (cfg->selection != ORC_SELECT_GUMBEL_MAX && cfg->selection != ORC_SELECT_INVERSE_CDF) return -1;
    if (cfg->n_obs < 0 || (cfg->n_obs > 0 && !cfg->obs_species)) return -1;
    if (!(cfg->temperature > 0.0)) return -1;
    for (int j = 0; j < net->n_reactions; ++j)
        if (net->rate_index[j] < 0 || net->rate_index[j] >= net->n_params) return -1;
    return 0;
}

static void rates_from_theta(const orc_net *net, const double *theta, double *k)
{
    for (int j = 0; j < net->n_reactions; ++j) k[j] = exp(theta[net->rate_index[j]]);
}

static void store_stats(const orc_stats *stats, int64_t q, const traj_stats_t *st)
{
    if (!stats) return;
    if (stats->min_margin) stats->min_margin[q] = st->min_margin;
    if (stats->n_near) stats->n_near[q] = st->n_near;
    if (stats->n_resync) stats->n_resync[q] = st->n_resync;
    if (stats->n_bad) stats->n_bad[q] = st->n_bad;
    if (stats->bin_edge_dist) stats->bin_edge_dist[q] = st->edge_dist;
}

int orc_forward(const orc_net *net, const orc_cfg *cfg, const double *theta,
                int64_t n_traj, const uint32_t *traj_ids, const int32_t *x0,
                const orc_overrides *ov,
                int32_t *x_final, double *t_final, int32_t *steps_done, double *obs,
                const orc_stats *stats, int n_threads)
{
    if (check_args(net, cfg) || n_traj < 0) return -1;
    const int N = net->n_species, M = net->n_reactions, W = obs_width(cfg);
    double *k = malloc(sizeof(double) * M);
    if (!k) return -1;
    rates_from_theta(net, theta, k);
    int err = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(|:err)
#endif
    for (int64_t q = 0; q < n_traj; ++q) {
        double *scratch = malloc(sizeof(double) * (2 * M + 1 + cfg->n_obs + 1));
        if (!scratch) { err |= 1; continue; }
        int32_t *X = x_final + (size_t)q * N;
        memcpy(X, x0 + (size_t)q * N, sizeof(int32_t) * N);
        double *o = obs + (size_t)q * W;
        memset(o, 0, sizeof(double) * W);
        traj_stats_t st;
        double t;
        int64_t n = simulate_one(net, cfg, k, traj_ids ? traj_ids[q] : (uint32_t)q, X, &t,
                                 ov, q, o, NULL, NULL, &st, scratch);
        if (n < 0) err |= 1;
        t_final[q] = t;
        steps_done[q] = (int32_t)n;
        finish_obs(cfg, X, o);
        store_stats(stats, q, &st);
        free(scratch);
    }
    free(k);
    return err ? -1 : 0;
}

/* Bin of an event time t_{k+1} = t for the clock-derivative term, taking the
 * GPU's side of a bin edge it lies close to (kind-2 overrides, see the header):
 * edge i is at t_obs i / n_bins, i = 1 .. n_bins; the side decides between
 * bin i - 1 and bin i (or nothing past t_obs). */
static int edge_side_bin(const orc_cfg *cfg, double t, int b, const orc_overrides *ov, int64_t q,
                         int64_t step, int32_t *n_bad)
{
    int ei = (int)floor(t * (double)cfg->n_bins / cfg->t_obs + 0.5);
    if (ei < 1) ei = 1;
    if (ei > cfg->n_bins) ei = cfg->n_bins;
    const double e = bin_edge(cfg, ei);
    const double d = fabs(t - e);
    int side = -1;
    if (ov)
        for (int64_t i = ov->off[q]; i < ov->off[q + 1]; ++i)
            if (ov->step[i] == step && ov->kind[i] == 2) side = ov->val[i];
    if (side < 0) {
        if (d <= 0.5 * cfg->edge_window * e && n_bad) ++*n_bad;
        return b;
    }
    /* the GPU logged it within the window of its own clock: the two clocks
     * differ by less than half the window, so a record is consistent up to
     * twice the window from the oracle's event */
    if (d > 2.0 * cfg->edge_window * e) {
        if (n_bad) ++*n_bad;
        return b;
    }
    if (side) return ei < cfg->n_bins ? ei : -1;
    return ei - 1;
}

/* Reverse sweep of the straight-through surrogate for one stored path.
 *
 * kappa (optional, [P]) receives the conditioning of each gradient component:
 * the sum over steps of the magnitudes of the terms that make up that step's
 * contribution, before they cancel.  Alongside the adjoint it carries a
 * magnitude adjoint Lam_X / Lam_t, the running sum of |every increment| of
 * lambda_X / lambda_t, so a term built from v_j . lambda is bounded by
 * sum_q |v_jq| Lam_q.  For parameter i, step k adds, over the channels j of i,
 *   (y~_j / T) (W_j + W_ref + sum_l y~_l W_l) + Lam_t (tau / a0) a_j
 * with W_j = sum_q |v_jq| Lam_q(k+1) and ref the fired channel.  A floating
 * point evaluation with unit roundoff u of the same recursion carries an error
 * of order u * kappa_i in component i, whatever cancellation leaves of it. */
static void adjoint_one(const orc_net *net, const orc_cfg *cfg, const double *k,
                        const path_t *p, const double *dobs, double *grad, double *kappa, double *work,
                        const orc_overrides *ov, int64_t q, int32_t *n_bad)
{
    const int N = net->n_species, M = net->n_reactions, P = net->n_params;
    const int nobs = cfg->n_obs;
    const double T = cfg->temperature;
    const int bins = cfg->obs_kind == ORC_OBS_BINS;
    const int grid = cfg->obs_kind == ORC_OBS_GRID;
    const int tail = cfg->obs_kind == ORC_OBS_TAIL;
    /* tail observation: states tail_lo .. n_steps enter the means */
    const int64_t tail_lo = tail ? cfg->n_steps - cfg->n_bins + 1 : 0;
    const double inv_dt = bins ? (double)cfg->n_bins / cfg->t_obs : 0.0;
    double *lamX = work;              /* [N] */
    double *dX = lamX + N;            /* [N] */
    double *a = dX + N;               /* [M] */
    double *y = a + M;                /* [M] */
    double *w = y + M;                /* [M] */
    double *g = w + M;                /* [M] */
    double *ones = g + M;             /* [n_obs] */
    double *LamX = ones + nobs;       /* [N]  magnitude adjoint */
    double *dXa = LamX + N;           /* [N] */
    double *Wa = dXa + N;             /* [M] */
    for (int o = 0; o < nobs; ++o) ones[o] = 1.0;
    memset(grad, 0, sizeof(double) * P);
    if (kappa) memset(kappa, 0, sizeof(double) * P);
    memset(lamX, 0, sizeof(double) * N);
    memset(LamX, 0, sizeof(double) * N);
    double lamt = 0.0, Lamt = 0.0;

    const int64_t n = p->n;
    /* direct dependence of L on the final state */
    if (bins) {
        /* lamX[s_o] += sum_b dobs[b][o] * |[t_n, t_obs) & bin_b| / dt */
        double *tmp = calloc((size_t)cfg->n_bins * nobs, sizeof(double));
        add_interval(cfg, p->t[n], cfg->t_obs, ones, tmp);
        for (int b = 0; b < cfg->n_bins; ++b)
            for (int o = 0; o < nobs; ++o) {
                const double d = dobs[(size_t)b * nobs + o] * tmp[(size_t)b * nobs + o] * inv_dt;
                lamX[cfg->obs_species[o]] += d;
                LamX[cfg->obs_species[o]] += fabs(d);
            }
        free(tmp);
    } else if (grid) {
        /* grid times at or after the last event see the final state */
        for (int g = grid_first_at_or_after(cfg, p->t[n]); g < cfg->n_bins; ++g)
            for (int o = 0; o < nobs; ++o) {
                lamX[cfg->obs_species[o]] += dobs[(size_t)g * nobs + o];
                LamX[cfg->obs_species[o]] += fabs(dobs[(size_t)g * nobs + o]);
            }
    } else if (tail) {
        /* the tail states at or after the last event are the final state and clock */
        const int64_t first = n > tail_lo ? n : tail_lo;
        const double wf = (double)(cfg->n_steps + 1 - first) / (double)cfg->n_bins;
        if (wf > 0.0) {
            for (int o = 0; o < nobs; ++o) {
                lamX[cfg->obs_species[o]] += dobs[o] * wf;
                LamX[cfg->obs_species[o]] += fabs(dobs[o] * wf);
            }
            lamt += dobs[nobs] * wf;
            Lamt += fabs(dobs[nobs] * wf);
        }
    } else {
        for (int o = 0; o < nobs; ++o) {
            lamX[cfg->obs_species[o]] += dobs[o];
            LamX[cfg->obs_species[o]] += fabs(dobs[o]);
        }
    }

    double *tmp = bins ? calloc((size_t)cfg->n_bins * nobs, sizeof(double)) : NULL;
    for (int64_t kk = n - 1; kk >= 0; --kk) {
        const int32_t *Xk = p->X + (size_t)kk * N;
        const int32_t *Xk1 = p->X + (size_t)(kk + 1) * N;
        const double tk = p->t[kk], tk1 = p->t[kk + 1];
        const double *E = p->E + (size_t)kk * (M + 1);

        /* direct dL/dt_{k+1}: t_{k+1} ends the interval at X_k and starts the one at X_{k+1} */
        if (bins) {
            int b = bin_of(cfg, tk1);
            if (cfg->edge_window > 0.0)
                b = edge_side_bin(cfg, tk1, b, ov, q, kk, n_bad);
            if (b >= 0)
                for (int o = 0; o < nobs; ++o) {
                    int s = cfg->obs_species[o];
                    const double d = dobs[(size_t)b * nobs + o] * (double)(Xk[s] - Xk1[s]) * inv_dt;
                    lamt += d;
                    Lamt += fabs(d);
                }
        }

        /* grid times in [t_k, t_{k+1}): obs = X_k + f (X_{k+1} - X_k) with
         * f = (t_g - t_k)/(t_{k+1} - t_k); the X_{k+1} and t_{k+1} parts
         * enter the adjoints of step k+1 before this step uses them */
        int g_lo = 0, g_hi = 0;
        if (grid) {
            g_lo = grid_first_at_or_after(cfg, tk);
            g_hi = grid_first_at_or_after(cfg, tk1);
            for (int g = g_lo; g < g_hi; ++g) {
                const double f = (grid_time(cfg, g) - tk) / (tk1 - tk);
                for (int o = 0; o < nobs; ++o) {
                    const int s = cfg->obs_species[o];
                    const double d = dobs[(size_t)g * nobs + o];
                    const double dt_ = d * (double)(Xk1[s] - Xk[s]) * (-f / (tk1 - tk));
                    lamX[s] += d * f;
                    lamt += dt_;
                    LamX[s] += fabs(d * f);
                    Lamt += fabs(dt_);
                }
            }
        }

        double a0 = 0.0;
        for (int j = 0; j < M; ++j) {
            a[j] = k[j] * mass_action_h(net->reactant + 2 * j, Xk);
            a0 += a[j];
        }
        const double tau = p->tau[kk];

        /* soft sample of Eq. (3) with the forward's Gumbel noise G_j = -ln(E_j) */
        double zmax = -INFINITY;
        for (int j = 0; j < M; ++j)
            if (a[j] > 0.0) {
                double z = (log(a[j]) - log(E[1 + j])) / T;
                y[j] = z;
                if (z > zmax) zmax = z;
            }
        double zs = 0.0;
        for (int j = 0; j < M; ++j) {
            y[j] = a[j] > 0.0 ? exp(y[j] - zmax) : 0.0;
            zs += y[j];
        }
        for (int j = 0; j < M; ++j) y[j] /= zs;

        /* w_j = v_j . lamX(k+1);  g_j = dL/d ln a_j through sum_j y~_j v_j */
        double wbar = 0.0;
        for (int j = 0; j < M; ++j) {
            const int32_t *v = net->stoich + (size_t)j * N;
            double s = 0.0;
            for (int q = 0; q < N; ++q) s += (double)v[q] * lamX[q];
            w[j] = s;
            wbar += y[j] * s;
        }
        for (int j = 0; j < M; ++j) g[j] = a[j] > 0.0 ? y[j] * (w[j] - wbar) / T : 0.0;

        /* waiting-time path: d tau = -(tau/a0) d a0 (Sec. 3.1) */
        const double c = lamt * (-tau / a0);

        for (int j = 0; j < M; ++j) grad[net->rate_index[j]] += g[j] + c * a[j];

        if (kappa) {
            /* magnitudes of the step's terms (see the comment above) */
            int jref = p->j[kk];
            double wy = 0.0;
            for (int j = 0; j < M; ++j) {
                const int32_t *v = net->stoich + (size_t)j * N;
                double s = 0.0;
                for (int q = 0; q < N; ++q) s += fabs((double)v[q]) * LamX[q];
                Wa[j] = s;
                wy += y[j] * s;
            }
            for (int j = 0; j < M; ++j)
                kappa[net->rate_index[j]] += (a[j] > 0.0 ? y[j] * (Wa[j] + Wa[jref] + wy) / T : 0.0) +
                                             Lamt * (tau / a0) * a[j];
        }

        memset(dX, 0, sizeof(double) * N);
        memset(dXa, 0, sizeof(double) * N);
        for (int j = 0; j < M; ++j) {
            if (a[j] > 0.0) add_grad_log_h(net->reactant + 2 * j, Xk, g[j], dX);
            add_grad_h(net->reactant + 2 * j, Xk, c * k[j], dX);
            if (kappa) {
                if (a[j] > 0.0) add_abs_grad_log_h(net->reactant + 2 * j, Xk, fabs(g[j]), dXa);
                add_abs_grad_h(net->reactant + 2 * j, Xk, fabs(c) * k[j], dXa);
            }
        }
        /* direct dL/dX_k from the interval [t_k, t_{k+1}) */
        if (bins) {
            memset(tmp, 0, sizeof(double) * (size_t)cfg->n_bins * nobs);
            add_interval(cfg, tk, tk1, ones, tmp);
            for (int b = 0; b < cfg->n_bins; ++b)
                for (int o = 0; o < nobs; ++o) {
                    const double d = dobs[(size_t)b * nobs + o] * tmp[(size_t)b * nobs + o] * inv_dt;
                    dX[cfg->obs_species[o]] += d;
                    dXa[cfg->obs_species[o]] += fabs(d);
                }
        }
        /* the X_k and t_k parts of this interval's grid times */
        if (grid)
            for (int g = g_lo; g < g_hi; ++g) {
                const double f = (grid_time(cfg, g) - tk) / (tk1 - tk);
                for (int o = 0; o < nobs; ++o) {
                    const int s = cfg->obs_species[o];
                    const double d = dobs[(size_t)g * nobs + o];
                    const double dt_ = d * (double)(Xk1[s] - Xk[s]) * ((f - 1.0) / (tk1 - tk));
                    dX[s] += d * (1.0 - f);
                    lamt += dt_;
                    dXa[s] += fabs(d * (1.0 - f));
                    Lamt += fabs(dt_);
                }
            }
        /* X_k and t_k as tail states */
        if (tail && kk >= tail_lo) {
            const double inv_m = 1.0 / (double)cfg->n_bins;
            for (int o = 0; o < nobs; ++o) {
                dX[cfg->obs_species[o]] += dobs[o] * inv_m;
                dXa[cfg->obs_species[o]] += fabs(dobs[o] * inv_m);
            }
            lamt += dobs[nobs] * inv_m;
            Lamt += fabs(dobs[nobs] * inv_m);
        }
        for (int q = 0; q < N; ++q) {
            lamX[q] += dX[q];
            LamX[q] += dXa[q];
        }
    }
    free(tmp);
}

int orc_adjoint(const orc_net *net, const orc_cfg *cfg, const double *theta,
                int64_t n_traj, const uint32_t *traj_ids, const int32_t *x0,
                const orc_overrides *ov, const double *d_obs,
                int32_t *x_final, double *t_final, int32_t *steps_done, double *obs,
                double *grad, const orc_stats *stats, int n_threads)
{
    return orc_adjoint_kappa(net, cfg, theta, n_traj, traj_ids, x0, ov, d_obs, x_final, t_final,
                             steps_done, obs, grad, NULL, stats, n_threads);
}

int orc_adjoint_kappa(const orc_net *net, const orc_cfg *cfg, const double *theta,
                      int64_t n_traj, const uint32_t *traj_ids, const int32_t *x0,
                      const orc_overrides *ov, const double *d_obs,
                      int32_t *x_final, double *t_final, int32_t *steps_done, double *obs,
                      double *grad, double *kappa, const orc_stats *stats, int n_threads)
{
    if (check_args(net, cfg) || n_traj < 0) return -1;
    /* the straight-through backward needs the Gumbel noise of the race */
    if (cfg->selection != ORC_SELECT_GUMBEL_MAX) return -1;
    const int N = net->n_species, M = net->n_reactions, P = net->n_params, W = obs_width(cfg);
    double *k = malloc(sizeof(double) * M);
    if (!k) return -1;
    rates_from_theta(net, theta, k);
    int err = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads) reduction(|:err)
#endif
    {
        path_t path;
        memset(&path, 0, sizeof(path));
        double *scratch = malloc(sizeof(double) * (2 * M + 1 + cfg->n_obs + 1));
        double *work = malloc(sizeof(double) * (4 * N + 5 * M + cfg->n_obs + 1));
        if (!scratch || !work) err |= 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t q = 0; q < n_traj; ++q) {
            if (!scratch || !work) continue;
            int32_t *X = x_final + (size_t)q * N;
            memcpy(X, x0 + (size_t)q * N, sizeof(int32_t) * N);
            double *o = obs + (size_t)q * W;
            memset(o, 0, sizeof(double) * W);
            traj_stats_t st;
            double t;
            int64_t n = simulate_one(net, cfg, k, traj_ids ? traj_ids[q] : (uint32_t)q, X, &t,
                                     ov, q, o, &path, NULL, &st, scratch);
            if (n < 0) { err |= 1; continue; }
            t_final[q] = t;
            steps_done[q] = (int32_t)n;
            finish_obs(cfg, X, o);
            int32_t edge_bad = 0;
            adjoint_one(net, cfg, k, &path, d_obs + (size_t)q * W, grad + (size_t)q * P,
                        kappa ? kappa + (size_t)q * P : NULL, work, ov, q, &edge_bad);
            st.n_bad += edge_bad;
            store_stats(stats, q, &st);
        }
        path_free(&path);
        free(scratch);
        free(work);
    }
    free(k);
    return err ? -1 : 0;
}

int64_t orc_trace(const orc_net *net, const orc_cfg *cfg, const double *theta,
                  uint32_t traj_id, const int32_t *x0, int64_t cap,
                  int32_t *X, double *t, double *tau, int32_t *j, double *a,
                  double *u, double *margin)
{
    if (check_args(net, cfg) || cap < 0) return -1;
    const int N = net->n_species, M = net->n_reactions;
    orc_cfg c = *cfg;
    if (c.n_steps > cap) c.n_steps = cap;
    double *k = malloc(sizeof(double) * M);
    double *scratch = malloc(sizeof(double) * (2 * M + 1 + c.n_obs + 1));
    double *obs = calloc((size_t)(c.obs_kind != ORC_OBS_FINAL ? c.n_bins * c.n_obs : 1) + 1,
                         sizeof(double));
    int32_t *Xw = malloc(sizeof(int32_t) * N);
    int64_t n = -1;
    if (k && scratch && obs && Xw) {
        rates_from_theta(net, theta, k);
        memcpy(Xw, x0, sizeof(int32_t) * N);
        trace_t tr = {cap, X, t, tau, j, a, u, margin};
        traj_stats_t st;
        double tf;
        n = simulate_one(net, &c, k, traj_id, Xw, &tf, NULL, 0, obs, NULL, &tr, &st, scratch);
    }
    free(k); free(scratch); free(obs); free(Xw);
    return n;
}
