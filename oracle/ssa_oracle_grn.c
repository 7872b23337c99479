/*
 * FP64 CPU oracle of the gene-regulatory network classifier (Sec. 4.3,
 * Fig. 4A of the paper) simulated by the direct method with Gumbel-max
 * selection, and of its straight-through adjoint.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this directory: the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg are its only
 * users.  It shares no code with the HIP library.
 *
 * What is computed:
 *   - Regulated production (Sec. 4.3, Fig. 4A): a gene is ON with probability
 *     sigmoid(E), E = b + sum_k w_k x_k over its regulators; its production
 *     propensity is beta times that probability.  Every gene decays with
 *     first-order rate delta = delta_min + exp(psi), which keeps delta above
 *     the paper's minimum decay rate.
 *   - The input layer is the image: its pixels are fixed factor levels, so the
 *     hidden genes see the constant E = u_h = b_h + sum_i W_hi x_i.  The
 *     contraction is taken on bfloat16-rounded W and x (products and sum exact
 *     here).  The output genes see v_o = c_o + sum_h U_oh H_h, which changes
 *     with the hidden counts.
 *   - Direct method, exponential race and soft sample exactly as for the
 *     mass-action networks (Sec. 2, Sec. 3.2, Eq. 3); the adjoint is the
 *     reverse recursion of the frozen straight-through surrogate (Eqs. 5-7,
 *     Fig. 1), with d ln a_j / d(parameters, state) of the regulated kinetics.
 *     The observation (final output counts) does not depend on event times,
 *     so the waiting-time path carries no gradient here.
 *   - The relaxed forward of Eq. 4 (the first phase of the two-phase training
 *     of Sec. 3.5): the state is real and every step moves it by the soft
 *     sample's expected change; its adjoint differentiates that whole map.
 */
#include "ssa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int64_t orc_grn_n_params(const orc_grn *net)
{
    const int64_t I = net->n_in, H = net->n_hid, O = net->n_out;
    return H * I + H + O * H + O + H + O;
}

int64_t orc_grn_n_compact(const orc_grn *net)
{
    const int64_t H = net->n_hid, O = net->n_out;
    return H + O * H + O + H + O;
}

float orc_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
        u |= 0x00400000u;                      /* NaN: keep it, quiet */
    } else {
        uint32_t lsb = (u >> 16) & 1u;          /* round half to even */
        u += 0x7FFFu + lsb;
    }
    u &= 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

void orc_grn_hidden_input(const orc_grn *net, const double *theta, const double *x_img,
                          int64_t n_images, double *u)
{
    const int I = net->n_in, H = net->n_hid;
    const double *W = theta, *b = theta + (size_t)H * I;
    for (int64_t m = 0; m < n_images; ++m)
        for (int h = 0; h < H; ++h) {
            /* each product of two bf16 values is exact in FP64; with n_in <= 2^20
             * terms of at most 16 significant bits each, the sum is exact too
             * unless the magnitudes span more than ~2^30 */
            double s = 0.0;
            for (int i = 0; i < I; ++i)
                s += (double)orc_bf16((float)W[(size_t)h * I + i]) *
                     (double)orc_bf16((float)x_img[(size_t)m * I + i]);
            u[(size_t)m * H + h] = b[h] + s;
        }
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Parameter views of theta. */
typedef struct {
    int H, O, M, N;
    const double *U, *c;          /* [O][H], [O] */
    double *delta, *dfac;         /* [H+O]: delta, d ln delta / d psi = exp(psi)/delta */
    double beta;
} grn_par_t;

static int par_init(const orc_grn *net, const double *theta, grn_par_t *p)
{
    const int I = net->n_in, H = net->n_hid, O = net->n_out;
    p->H = H; p->O = O; p->M = 2 * H + 2 * O; p->N = H + O;
    p->beta = net->beta;
    const double *base = theta + (size_t)H * I + H;
    p->U = base;
    p->c = base + (size_t)O * H;
    const double *psi = p->c + O;
    p->delta = malloc(sizeof(double) * (H + O));
    p->dfac = malloc(sizeof(double) * (H + O));
    if (!p->delta || !p->dfac) return -1;
    for (int g = 0; g < H + O; ++g) {
        double e = exp(psi[g]);
        p->delta[g] = net->delta_min + e;
        p->dfac[g] = e / p->delta[g];
    }
    return 0;
}

static void par_free(grn_par_t *p) { free(p->delta); free(p->dfac); }

/* All M propensities at state X = (H, O); v[o] receives the output
 * pre-activations, sh[h] = sigmoid(u_h) is precomputed. */
static double propensities(const grn_par_t *p, const double *sh, const int32_t *X,
                           double *v, double *a)
{
    const int H = p->H, O = p->O;
    double a0 = 0.0;
    for (int h = 0; h < H; ++h) {
        a[h] = p->beta * sh[h];
        a[H + h] = p->delta[h] * (double)X[h];
    }
    for (int o = 0; o < O; ++o) {
        double s = p->c[o];
        for (int h = 0; h < H; ++h) s += p->U[(size_t)o * H + h] * (double)X[h];
        v[o] = s;
        a[2 * H + o] = p->beta * sigmoid(s);
        a[2 * H + O + o] = p->delta[H + o] * (double)X[H + o];
    }
    for (int j = 0; j < p->M; ++j) a0 += a[j];
    return a0;
}

/* Species touched by channel j and the change (+1 production, -1 decay). */
static void channel_effect(const grn_par_t *p, int j, int *species, int *delta)
{
    const int H = p->H, O = p->O;
    if (j < H) { *species = j; *delta = 1; }
    else if (j < 2 * H) { *species = j - H; *delta = -1; }
    else if (j < 2 * H + O) { *species = H + (j - 2 * H); *delta = 1; }
    else { *species = H + (j - 2 * H - O); *delta = -1; }
}

typedef struct {
    double min_margin;
    int32_t n_near, n_resync, n_bad;
} grn_stats_t;

/* Forward of one trajectory; if jpath != NULL the fired channels are kept
 * (capacity cfg->n_steps), if tpath != NULL the clock [n+1]. */
static int64_t simulate_grn(const grn_par_t *p, const orc_cfg *cfg, const double *sh,
                            uint32_t traj_id, int32_t *X, double *t_out,
                            const orc_overrides *ov, int64_t q, int32_t *jpath, double *tpath,
                            int64_t cap, grn_stats_t *st, double *u, double *a, double *v)
{
    const int M = p->M;
    double t = 0.0;
    int64_t p_ov = ov ? ov->off[q] : 0, p_end = ov ? ov->off[q + 1] : 0;
    st->min_margin = INFINITY;
    st->n_near = st->n_resync = st->n_bad = 0;
    if (tpath) tpath[0] = 0.0;
    int64_t k = 0;
    for (; k < cfg->n_steps && k < cap; ++k) {
        double a0 = propensities(p, sh, X, v, a);
        if (!(a0 > 0.0)) break;
        orc_step_uniforms(cfg->seed, cfg->purpose, cfg->epoch, traj_id, (uint32_t)k, M + 1, u);
        double tau = -log(u[0]) / a0;

        int ov_clock = -1, ov_react = -1;
        while (p_ov < p_end && ov->step[p_ov] < k) ++p_ov;
        for (int64_t e = p_ov; e < p_end && ov->step[e] == k; ++e) {
            if (ov->kind[e] == 1) ov_clock = ov->val[e];
            else ov_react = ov->val[e];
        }
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
        double r1 = INFINITY, r2 = INFINITY;
        for (int j = 0; j < M; ++j) {
            if (!(a[j] > 0.0)) continue;
            double r = -log(u[1 + j]) / a[j];
            if (r < r1) { r2 = r1; r1 = r; jbest = j; }
            else if (r < r2) { r2 = r; }
        }
        double margin = isfinite(r2) ? (r2 - r1) / r1 : INFINITY;
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
        int s, d;
        channel_effect(p, jbest, &s, &d);
        X[s] += d;
        t += tau;
        if (jpath) jpath[k] = jbest;
        if (tpath) tpath[k + 1] = t;
    }
    *t_out = t;
    return k;
}

/*
 * Reverse sweep of the frozen surrogate.  X holds the final state on entry
 * (it is walked back to X_0); jpath the fired channels.  g_c receives
 * [du | dU | dc | dpsi].
 */
static void adjoint_grn(const grn_par_t *p, const orc_cfg *cfg, const double *sh,
                        uint32_t traj_id, int32_t *X, const int32_t *jpath, int64_t n,
                        const double *dobs, double *g_c, double *u, double *a, double *v,
                        double *y, double *w, double *lam)
{
    const int H = p->H, O = p->O, M = p->M, N = p->N;
    const double T = cfg->temperature;
    double *du = g_c, *dU = du + H, *dc = dU + (size_t)O * H, *dpsi = dc + O;
    memset(g_c, 0, sizeof(double) * (size_t)(H + O * H + O + H + O));
    for (int s = 0; s < H; ++s) lam[s] = 0.0;
    for (int o = 0; o < O; ++o) lam[H + o] = dobs[o];   /* L depends on O_n only */
    double *dlam = lam + N;                              /* [N] */

    for (int64_t k = n - 1; k >= 0; --k) {
        int s, d;
        channel_effect(p, jpath[k], &s, &d);
        X[s] -= d;                                       /* X_k from X_{k+1} */
        propensities(p, sh, X, v, a);
        orc_step_uniforms(cfg->seed, cfg->purpose, cfg->epoch, traj_id, (uint32_t)k, M + 1, u);

        /* soft sample of Eq. (3) with the forward's noise G_j = -ln(-ln u_{1+j}) */
        double zmax = -INFINITY;
        for (int j = 0; j < M; ++j)
            if (a[j] > 0.0) {
                y[j] = (log(a[j]) - log(-log(u[1 + j]))) / T;
                if (y[j] > zmax) zmax = y[j];
            }
        double zs = 0.0;
        for (int j = 0; j < M; ++j) {
            y[j] = a[j] > 0.0 ? exp(y[j] - zmax) : 0.0;
            zs += y[j];
        }
        /* w_j = v_j . lambda_{k+1}: +lambda for production, -lambda for decay */
        double wbar = 0.0;
        for (int j = 0; j < M; ++j) {
            y[j] /= zs;
            int sp, dd;
            channel_effect(p, j, &sp, &dd);
            w[j] = (double)dd * lam[sp];
            wbar += y[j] * w[j];
        }
        memset(dlam, 0, sizeof(double) * N);
        for (int j = 0; j < M; ++j) {
            if (!(a[j] > 0.0)) continue;
            /* g_j = dL / d ln a_j */
            double g = y[j] * (w[j] - wbar) / T;
            if (j < H) {                                 /* d ln a / d u_h = 1 - sigmoid(u_h) */
                du[j] += g * (1.0 - sh[j]);
            } else if (j < 2 * H) {                      /* a = delta_h H_h */
                int h = j - H;
                dpsi[h] += g * p->dfac[h];
                dlam[h] += g / (double)X[h];
            } else if (j < 2 * H + O) {                  /* a = beta sigmoid(v_o) */
                int o = j - 2 * H;
                double e = g * (1.0 - sigmoid(v[o]));    /* dL / d v_o */
                dc[o] += e;
                for (int h = 0; h < H; ++h) {
                    dU[(size_t)o * H + h] += e * (double)X[h];
                    dlam[h] += e * p->U[(size_t)o * H + h];
                }
            } else {                                     /* a = delta_o O_o */
                int o = j - 2 * H - O;
                dpsi[H + o] += g * p->dfac[H + o];
                dlam[H + o] += g / (double)X[H + o];
            }
        }
        for (int q = 0; q < N; ++q) lam[q] += dlam[q];
    }
}

static int grn_args_ok(const orc_grn *net, const orc_cfg *cfg)
{
    if (!net || !cfg || net->n_in < 0 || net->n_hid <= 0 || net->n_out <= 0) return 0;
    if (!(net->beta > 0.0) || !(net->delta_min >= 0.0) || !(cfg->temperature > 0.0)) return 0;
    return 1;
}

int orc_grn_run(const orc_grn *net, const orc_cfg *cfg, const double *theta,
                const double *u_hid, int64_t n_traj, const uint32_t *traj_ids,
                const int32_t *image_of, const int32_t *x0, const orc_overrides *ov,
                const double *d_obs, int32_t *x_final, double *t_final, int32_t *steps_done,
                double *obs, double *grad_c, const orc_stats *stats, int n_threads)
{
    if (!grn_args_ok(net, cfg) || n_traj < 0 || !u_hid || !image_of) return -1;
    grn_par_t p;
    if (par_init(net, theta, &p)) { par_free(&p); return -1; }
    const int H = p.H, O = p.O, M = p.M, N = p.N;
    const int64_t C = orc_grn_n_compact(net);
    const int64_t cap = cfg->n_steps;
    int err = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads) reduction(|:err)
#endif
    {
        double *buf = malloc(sizeof(double) * (size_t)(H + (M + 1) + M + O + M + M + 2 * N));
        int32_t *jpath = d_obs ? malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1)) : NULL;
        if (!buf || (d_obs && !jpath)) err |= 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t q = 0; q < n_traj; ++q) {
            if (!buf || (d_obs && !jpath)) continue;
            double *sh = buf, *u = sh + H, *a = u + (M + 1), *v = a + M, *y = v + O, *w = y + M,
                   *lam = w + M;
            const double *urow = u_hid + (size_t)image_of[q] * H;
            for (int h = 0; h < H; ++h) sh[h] = sigmoid(urow[h]);
            int32_t *X = x_final + (size_t)q * N;
            memcpy(X, x0 + (size_t)q * N, sizeof(int32_t) * N);
            const uint32_t id = traj_ids ? traj_ids[q] : (uint32_t)q;
            grn_stats_t st;
            double t;
            int64_t n = simulate_grn(&p, cfg, sh, id, X, &t, ov, q, jpath, NULL,
                                     cap, &st, u, a, v);
            t_final[q] = t;
            steps_done[q] = (int32_t)n;
            for (int o = 0; o < O; ++o) obs[(size_t)q * O + o] = (double)X[H + o];
            if (stats) {
                if (stats->min_margin) stats->min_margin[q] = st.min_margin;
                if (stats->n_near) stats->n_near[q] = st.n_near;
                if (stats->n_resync) stats->n_resync[q] = st.n_resync;
                if (stats->n_bad) stats->n_bad[q] = st.n_bad;
                if (stats->bin_edge_dist) stats->bin_edge_dist[q] = INFINITY;
            }
            if (d_obs) {
                int32_t *Xw = malloc(sizeof(int32_t) * N);
                if (!Xw) { err |= 1; continue; }
                memcpy(Xw, X, sizeof(int32_t) * N);
                adjoint_grn(&p, cfg, sh, id, Xw, jpath, n, d_obs + (size_t)q * O,
                            grad_c + (size_t)q * C, u, a, v, y, w, lam);
                free(Xw);
            }
        }
        free(buf);
        free(jpath);
    }
    par_free(&p);
    return err ? -1 : 0;
}

int64_t orc_grn_trace(const orc_grn *net, const orc_cfg *cfg, const double *theta,
                      const double *u_row, uint32_t traj_id, const int32_t *x0, int64_t cap,
                      int32_t *j, double *t)
{
    if (!grn_args_ok(net, cfg) || cap < 0 || !u_row) return -1;
    grn_par_t p;
    if (par_init(net, theta, &p)) { par_free(&p); return -1; }
    const int H = p.H, O = p.O, M = p.M, N = p.N;
    double *buf = malloc(sizeof(double) * (size_t)(H + (M + 1) + M + O));
    int32_t *X = malloc(sizeof(int32_t) * N);
    int64_t n = -1;
    if (buf && X) {
        double *sh = buf, *u = sh + H, *a = u + (M + 1), *v = a + M;
        for (int h = 0; h < H; ++h) sh[h] = sigmoid(u_row[h]);
        memcpy(X, x0, sizeof(int32_t) * N);
        grn_stats_t st;
        double tf;
        n = simulate_grn(&p, cfg, sh, traj_id, X, &tf, NULL, 0, j, t, cap, &st, u, a, v);
    }
    free(buf);
    free(X);
    par_free(&p);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Relaxed (soft) forward of the gene network (Sec. 3.3, Eq. 4)              */
/* ------------------------------------------------------------------------ */

/* Propensities at a real-valued state: a relaxed count at or below zero gives
 * its decay channel a zero propensity (the channel is out of the soft sample,
 * as an exhausted reactant puts a channel out of the hard process). */
static double soft_propensities(const grn_par_t *p, const double *sh, const double *X, double *v, double *a)
{
    const int H = p->H, O = p->O;
    double a0 = 0.0;
    for (int h = 0; h < H; ++h) {
        a[h] = p->beta * sh[h];
        a[H + h] = X[h] > 0.0 ? p->delta[h] * X[h] : 0.0;
    }
    for (int o = 0; o < O; ++o) {
        double s = p->c[o];
        for (int h = 0; h < H; ++h) s += p->U[(size_t)o * H + h] * X[h];
        v[o] = s;
        a[2 * H + o] = p->beta * sigmoid(s);
        a[2 * H + O + o] = X[H + o] > 0.0 ? p->delta[H + o] * X[H + o] : 0.0;
    }
    for (int j = 0; j < p->M; ++j) a0 += a[j];
    return a0;
}

/* Soft sample of Eq. (3): y_j = softmax_j((ln a_j + G_j) / T) over the
 * channels with a_j > 0, G_j = -ln(-ln u_{1+j}). */
static void soft_sample(int M, const double *a, const double *u, double T, double *y)
{
    double zmax = -INFINITY;
    for (int j = 0; j < M; ++j)
        if (a[j] > 0.0) {
            y[j] = (log(a[j]) - log(-log(u[1 + j]))) / T;
            if (y[j] > zmax) zmax = y[j];
        }
    double zs = 0.0;
    for (int j = 0; j < M; ++j) {
        y[j] = a[j] > 0.0 ? exp(y[j] - zmax) : 0.0;
        zs += y[j];
    }
    for (int j = 0; j < M; ++j) y[j] /= zs;
}

/* Relaxed path of one trajectory: X_{k+1} = X_k + sum_j y_j v_j (Eq. 4),
 * t_{k+1} = t_k - ln(u_0) / a0(X_k).  X [(n_steps + 1)][N] receives the
 * states (X[0] = x0), t [n_steps + 1] the clock.  Returns the steps taken. */
static int64_t simulate_grn_soft(const grn_par_t *p, const orc_cfg *cfg, const double *sh,
                                 uint32_t traj_id, double *X, double *t, double *u, double *a,
                                 double *v, double *y)
{
    const int M = p->M, N = p->N;
    t[0] = 0.0;
    int64_t k = 0;
    for (; k < cfg->n_steps; ++k) {
        const double *Xk = X + (size_t)k * N;
        double *Xn = X + (size_t)(k + 1) * N;
        const double a0 = soft_propensities(p, sh, Xk, v, a);
        if (!(a0 > 0.0)) break;
        orc_step_uniforms(cfg->seed, cfg->purpose, cfg->epoch, traj_id, (uint32_t)k, M + 1, u);
        soft_sample(M, a, u, cfg->temperature, y);
        memcpy(Xn, Xk, sizeof(double) * N);
        for (int j = 0; j < M; ++j) {
            int s, d;
            channel_effect(p, j, &s, &d);
            Xn[s] += (double)d * y[j];
        }
        t[k + 1] = t[k] - log(u[0]) / a0;
    }
    return k;
}

/* Reverse sweep of the relaxed map (every step differentiated, no stop
 * gradient): lambda_k = lambda_{k+1} + sum_j g_j grad_X ln a_j(X_k) with
 * g_j = y_j (w_j - sum_l y_l w_l) / T and w_j = v_j . lambda_{k+1}, the
 * Jacobian of Eq. 4's update transposed.  The parameters get
 * sum_k sum_j g_j d ln a_j / d(parameter).  X: the stored path. */
static void adjoint_grn_soft(const grn_par_t *p, const orc_cfg *cfg, const double *sh, uint32_t traj_id,
                             const double *X, int64_t n, const double *dobs, double *g_c, double *u,
                             double *a, double *v, double *y, double *w, double *lam)
{
    const int H = p->H, O = p->O, M = p->M, N = p->N;
    const double T = cfg->temperature;
    double *du = g_c, *dU = du + H, *dc = dU + (size_t)O * H, *dpsi = dc + O;
    memset(g_c, 0, sizeof(double) * (size_t)(H + O * H + O + H + O));
    for (int s = 0; s < H; ++s) lam[s] = 0.0;
    for (int o = 0; o < O; ++o) lam[H + o] = dobs[o];
    double *dlam = lam + N;
    for (int64_t k = n - 1; k >= 0; --k) {
        const double *Xk = X + (size_t)k * N;
        soft_propensities(p, sh, Xk, v, a);
        orc_step_uniforms(cfg->seed, cfg->purpose, cfg->epoch, traj_id, (uint32_t)k, M + 1, u);
        soft_sample(M, a, u, T, y);
        double wbar = 0.0;
        for (int j = 0; j < M; ++j) {
            int sp, dd;
            channel_effect(p, j, &sp, &dd);
            w[j] = (double)dd * lam[sp];
            wbar += y[j] * w[j];
        }
        memset(dlam, 0, sizeof(double) * N);
        for (int j = 0; j < M; ++j) {
            if (!(a[j] > 0.0)) continue;
            const double g = y[j] * (w[j] - wbar) / T;
            if (j < H) {
                du[j] += g * (1.0 - sh[j]);
            } else if (j < 2 * H) {
                const int h = j - H;
                dpsi[h] += g * p->dfac[h];
                dlam[h] += g / Xk[h];
            } else if (j < 2 * H + O) {
                const int o = j - 2 * H;
                const double e = g * (1.0 - sigmoid(v[o]));
                dc[o] += e;
                for (int h = 0; h < H; ++h) {
                    dU[(size_t)o * H + h] += e * Xk[h];
                    dlam[h] += e * p->U[(size_t)o * H + h];
                }
            } else {
                const int o = j - 2 * H - O;
                dpsi[H + o] += g * p->dfac[H + o];
                dlam[H + o] += g / Xk[H + o];
            }
        }
        for (int q = 0; q < N; ++q) lam[q] += dlam[q];
    }
}

int orc_grn_soft_run(const orc_grn *net, const orc_cfg *cfg, const double *theta, const double *u_hid,
                     int64_t n_traj, const uint32_t *traj_ids, const int32_t *image_of, const double *x0,
                     const double *d_obs, double *x_final, double *t_final, double *obs, double *grad_c,
                     int n_threads)
{
    if (!grn_args_ok(net, cfg) || n_traj < 0 || !u_hid || !image_of || !x0 || cfg->n_steps < 0 ||
        cfg->n_steps > ((int64_t)1 << 28) || isfinite(cfg->t_end))
        return -1;
    grn_par_t p;
    if (par_init(net, theta, &p)) { par_free(&p); return -1; }
    const int H = p.H, O = p.O, M = p.M, N = p.N;
    const int64_t C = orc_grn_n_compact(net), n_steps = cfg->n_steps;
    int err = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads) reduction(|:err)
#endif
    {
        double *buf = malloc(sizeof(double) * (size_t)(H + (M + 1) + M + O + M + M + 2 * N));
        double *X = malloc(sizeof(double) * (size_t)(n_steps + 1) * N);
        double *t = malloc(sizeof(double) * (size_t)(n_steps + 1));
        if (!buf || !X || !t) err |= 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t q = 0; q < n_traj; ++q) {
            if (!buf || !X || !t) continue;
            double *sh = buf, *u = sh + H, *a = u + (M + 1), *v = a + M, *y = v + O, *w = y + M, *lam = w + M;
            const double *urow = u_hid + (size_t)image_of[q] * H;
            for (int h = 0; h < H; ++h) sh[h] = sigmoid(urow[h]);
            memcpy(X, x0 + (size_t)q * N, sizeof(double) * N);
            const uint32_t id = traj_ids ? traj_ids[q] : (uint32_t)q;
            const int64_t n = simulate_grn_soft(&p, cfg, sh, id, X, t, u, a, v, y);
            memcpy(x_final + (size_t)q * N, X + (size_t)n * N, sizeof(double) * N);
            t_final[q] = t[n];
            for (int o = 0; o < O; ++o) obs[(size_t)q * O + o] = X[(size_t)n * N + H + o];
            if (d_obs)
                adjoint_grn_soft(&p, cfg, sh, id, X, n, d_obs + (size_t)q * O, grad_c + (size_t)q * C,
                                 u, a, v, y, w, lam);
        }
        free(buf);
        free(X);
        free(t);
    }
    par_free(&p);
    return err ? -1 : 0;
}

int64_t orc_grn_soft_trace(const orc_grn *net, const orc_cfg *cfg, const double *theta, const double *u_row,
                           uint32_t traj_id, const double *x0, int64_t cap, double *X, double *t)
{
    if (!grn_args_ok(net, cfg) || cap < 0 || !u_row || isfinite(cfg->t_end)) return -1;
    grn_par_t p;
    if (par_init(net, theta, &p)) { par_free(&p); return -1; }
    const int H = p.H, O = p.O, M = p.M, N = p.N;
    orc_cfg c = *cfg;
    if (c.n_steps > cap) c.n_steps = cap;
    double *buf = malloc(sizeof(double) * (size_t)(H + (M + 1) + M + O + M));
    int64_t n = -1;
    if (buf) {
        double *sh = buf, *u = sh + H, *a = u + (M + 1), *v = a + M, *y = v + O;
        for (int h = 0; h < H; ++h) sh[h] = sigmoid(u_row[h]);
        memcpy(X, x0, sizeof(double) * N);
        n = simulate_grn_soft(&p, &c, sh, traj_id, X, t, u, a, v, y);
    }
    free(buf);
    par_free(&p);
    return n;
}
