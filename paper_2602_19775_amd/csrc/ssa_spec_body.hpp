// Lane-mode kernels specialised to one network topology.  The network comes
// in as a type NET with compile-time tables:
//   N, M, NOBS                       species, channels, observed species
//   S1[M], S2[M], HOMO[M], MULT[M]   a_j = k_j MULT[j] X[S1[j]] (X[S2[j]] - HOMO[j]);
//                                    index N is a register that always holds 1
//   RATE[M]                          parameter slot of channel j
//   V[M][N]                          change vectors
//   OBS[NOBS]                        observed species
// so every species index is a constant and the state, its adjoint and the
// per-channel values live in plain registers.  The library compiles one such
// kernel pair per topology at plan time (hipRTC); rates, states and all run
// settings stay runtime inputs.
//
// Forward (Sec. 2, Sec. 3.2): a_j, a0, tau = E_0/a0, j* = argmin_j E_j/a_j
// (= argmax_j ln a_j + G_j with G_j = -ln E_j), X += v_j*, t += tau (FP64),
// exact bin integrals of the observed species (Sec. 4.4) or the path linearly
// interpolated between its event points on a uniform time grid (Sec. 4.1),
// checkpoints every K steps and the compact choice tape.
// Backward (Sec. 3.1, Eqs. 3-7, Fig. 1): reverse sweep with the noise,
// propensities and waiting times regenerated from the Philox counters.
#pragma once

#include "ssa_device.hpp"
#include "ssa_plan.hpp"

namespace ssa {
namespace spec {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kFold = 32;   // FP32 adjoint increments are folded into FP64 this often
// register arrays of the observed species need at least one slot
constexpr int obs_cap(int n) { return n > 0 ? n : 1; }

__device__ __forceinline__ double bin_edge(double t_obs, int b, int n_bins)
{
    return t_obs * (double)b / (double)n_bins;
}

// Grid time g of an n-point grid spanning [0, t_obs].
__device__ __forceinline__ double grid_time(double t_obs, int g, int n)
{
    return t_obs * (double)g / (double)(n - 1);
}

// v_j[s] for a runtime channel j.
template <class NET>
__device__ __forceinline__ int delta_of(int j, int s)
{
    int d = 0;
#pragma unroll
    for (int q = 0; q < NET::M; ++q)
        if (NET::V[q][s] != 0) d = (j == q) ? NET::V[q][s] : d;
    return d;
}

// Runs of bins of a trajectory-major observation block, filled by the whole
// wave: lane l holds the bins [lo_l, hi_l) of its own row, all with its held
// counts x (scaled: the bin integral of the held state divided by the bin
// width, computed as the per-bin accumulation computes it; otherwise the
// count itself).  One lane's run at a time, 64 consecutive values a store, so
// a row's cache lines are written whole instead of one value per lane and
// store.  Every lane of the wave must be active.
template <class NET>
__device__ __forceinline__ void fill_runs(double *blk, int64_t first, int64_t npts, int lo, int hi,
                                          const int (&X)[NET::N + 1], bool scaled, double t_obs, int n_bins,
                                          double inv_dt)
{
    constexpr int NOBS = NET::NOBS;
    if constexpr (NOBS > 0) {
        const int lane = threadIdx.x & 63;
        uint64_t m = ballot(hi > lo);
        while (m != 0ull) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            const int rlo = __builtin_amdgcn_readlane(lo, l), rhi = __builtin_amdgcn_readlane(hi, l);
            int xv[NOBS];
#pragma unroll
            for (int o = 0; o < NOBS; ++o) xv[o] = __builtin_amdgcn_readlane(X[NET::OBS[o]], l);
            double *row = blk + (first + l) * npts * NOBS;
            for (int64_t q = (int64_t)rlo * NOBS + lane; q < (int64_t)rhi * NOBS; q += 64) {
                const int b = (int)(q / NOBS), o = (int)(q - (int64_t)b * NOBS);
                int x = xv[0];
#pragma unroll
                for (int u = 1; u < NOBS; ++u) x = o == u ? xv[u] : x;
                row[q] = scaled ? ((double)x * fmax(bin_edge(t_obs, b + 1, n_bins) - bin_edge(t_obs, b, n_bins),
                                                    0.0)) * inv_dt
                                : (double)x;
            }
        }
    }
}

// Fixed-point scale of the single-bin values the ensemble-mean forward sums.
constexpr double kFixScale = 4294967296.0;   // 2^32
// Largest observed count the ensemble-mean forward sums exactly: 64 lanes add
// into one slot, so a count below 2^25 keeps the int32 difference arrays and
// the int64 fixed-point sums (count * 2^32 each) within range.  A larger one
// raises the overflow flag.
constexpr double kEnsMaxCount = 33554432.0;  // 2^25

// The ensemble-mean forward's additions for one lane: the value of a single
// bin fb (the bin an interval completes or the one the path stops in; -1 for
// none) in fixed point with 2^-32 resolution, and the run [lo, hi) of whole
// bins holding the count x as +x at lo and -x at hi in a difference array of
// counts (dsc for bins an interval crosses, whose values are the count times
// the bin width over the nominal width; dun for the held tail, whose values
// are the count).  Integer additions commute, so the wave's sums do not depend
// on the order in which its lanes reach them.  Returns true when a value is
// too large to be summed exactly (kEnsMaxCount); it is then left out.
template <class NET>
__device__ __forceinline__ bool ens_add(long long *sfp, int *dsc, int *dun, int fb,
                                        const double (&fv)[obs_cap(NET::NOBS)], int lo, int hi,
                                        const int (&X)[NET::N + 1], bool scaled)
{
    constexpr int NOBS = NET::NOBS;
    bool big = false;
    if (fb >= 0) {
#pragma unroll
        for (int o = 0; o < NOBS; ++o) {
            const bool ok = fabs(fv[o]) < kEnsMaxCount;
            big = big || !ok;
            if (ok)
                atomicAdd((unsigned long long *)&sfp[fb * NOBS + o],
                          (unsigned long long)(long long)rint(fv[o] * kFixScale));
        }
    }
    if (hi > lo) {
        int *d = scaled ? dsc : dun;
#pragma unroll
        for (int o = 0; o < NOBS; ++o) {
            const int x = X[NET::OBS[o]];
            const bool ok = x > -(int)kEnsMaxCount && x < (int)kEnsMaxCount;
            big = big || !ok;
            if (ok) {
                atomicAdd(&d[lo * NOBS + o], x);
                atomicAdd(&d[hi * NOBS + o], -x);
            }
        }
    }
    return big;
}

// The wave's row of sums [bin][obs]: each lane takes a contiguous chunk of
// bins, the difference arrays are summed over the chunks before it (an
// exclusive scan over the lanes), and each bin's sum is the fixed-point part
// plus the crossed-bin counts times the bin width over the nominal width plus
// the tail counts.  Every lane of the wave must be active.
template <class NET>
__device__ __forceinline__ void ens_row(double *row, const long long *sfp, const int *dsc, const int *dun,
                                        int n_bins, double t_obs, double inv_dt)
{
    constexpr int NOBS = NET::NOBS;
    const int lane = threadIdx.x & 63;
    const int per = (n_bins + 63) / 64;
    const int b0 = min(lane * per, n_bins), b1 = min(b0 + per, n_bins);
#pragma unroll
    for (int o = 0; o < NOBS; ++o) {
        int ts = 0, tu = 0;
        for (int b = b0; b < b1; ++b) {
            ts += dsc[b * NOBS + o];
            tu += dun[b * NOBS + o];
        }
        int cs = ts, cu = tu;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int as = __shfl_up(cs, off), au = __shfl_up(cu, off);
            if (lane >= off) { cs += as; cu += au; }
        }
        int ps = cs - ts, pu = cu - tu;
        for (int b = b0; b < b1; ++b) {
            ps += dsc[b * NOBS + o];
            pu += dun[b * NOBS + o];
            const double w = fmax(bin_edge(t_obs, b + 1, n_bins) - bin_edge(t_obs, b, n_bins), 0.0);
            row[b * NOBS + o] = (double)sfp[b * NOBS + o] * (1.0 / kFixScale) + ((double)ps * w) * inv_dt + (double)pu;
        }
    }
}

__device__ __forceinline__ void log_tie(const RunParams &p, uint32_t g, int k, int chosen, int second,
                                     float margin, int kind)
{
    if (!p.ties) return;
    const uint32_t idx = atomicAdd(p.n_ties, 1u);
    if (idx < p.tie_cap) {
        TieRec r;
        r.traj = g; r.step = (uint32_t)k; r.chosen = chosen; r.second = second;
        r.margin = margin; r.kind = kind;
        p.ties[idx] = r;
    }
}

template <class NET>
struct Blocks {
    static constexpr int NB = (NET::M + 1 + 3) / 4;
    static constexpr int W = 4 * NB;
};

// Philox words of step k (word 0: tau, word 1+j: channel j).
template <class NET, int NW = Blocks<NET>::W>
__device__ __forceinline__ void words(uint32_t k, uint32_t tid, uint32_t pe, uint32_t k0, uint32_t k1,
                                      uint32_t (&wd)[NW])
{
#pragma unroll
    for (int b = 0; b < NW / 4; ++b) {
        const Philox::Out o = Philox::block((uint32_t)b, k, tid, pe, k0, k1);
        wd[4 * b] = o.x;
        wd[4 * b + 1] = o.y;
        wd[4 * b + 2] = o.z;
        wd[4 * b + 3] = o.w;
    }
}

// a_j and (optionally) A1 = c_j X[S1], A2 = c_j (X[S2] - HOMO): da_j/dX[S2], da_j/dX[S1].
template <class NET, bool DERIV>
__device__ __forceinline__ float propensities(const float (&c)[NET::M], const int (&X)[NET::N + 1],
                                              float (&a)[NET::M], float (&A1)[NET::M], float (&A2)[NET::M])
{
    float a0 = 0.f;
#pragma unroll
    for (int j = 0; j < NET::M; ++j) {
        const float x1 = (float)X[NET::S1[j]];
        const float x2 = (float)(X[NET::S2[j]] - NET::HOMO[j]);
        const float u1 = c[j] * x1;
        // a homodimer at X = 0 gives 0 * (-1) = -0; |.| keeps it +0 so that
        // its reciprocal is +inf and the channel never wins the race
        a[j] = fabsf(u1 * x2);
        if (DERIV) {
            A1[j] = u1;
            A2[j] = c[j] * x2;
        }
        a0 += a[j];
    }
    return a0;
}

// X += sign * v_j for a per-lane channel j.
template <class NET>
__device__ __forceinline__ void apply(int (&X)[NET::N + 1], int j, int sign)
{
#pragma unroll
    for (int s = 0; s < NET::N; ++s) {
        int d = 0;
#pragma unroll
        for (int q = 0; q < NET::M; ++q)
            if (NET::V[q][s] != 0) d = (j == q) ? NET::V[q][s] : d;
        X[s] += sign * d;
    }
}

template <class NET>
__device__ __forceinline__ void rates(const RunParams &p, const NetDev &nd, float (&c)[NET::M])
{
#pragma unroll
    for (int j = 0; j < NET::M; ++j) c[j] = expf(p.theta[nd.param_off + NET::RATE[j]]) * NET::MULT[j];
}

// --------------------------------------------------------------------------
// GRID: the grid observation (the other kinds are runtime cases of GRID = false).
// CDF: the channel is the standard direct method's inverse-CDF draw from word 1
// (Sec. 2) instead of the Gumbel-max race; such a run has no backward.
// TMB: bin observations in the trajectory-major layout, whose whole bins are
// filled by the wave (the other kernels take either layout through strides).
// ENS (with TMB, or with GRID): only the ensemble means are kept; each wave
// sums its trajectories' bins or grid points in LDS (integer additions, so in
// any order) and stores one row of sums for its tile.
template <class NET, bool HAS_T_END, bool GRID, bool CDF = false, bool TMB = false, bool ENS = false>
__device__ void forward_run(const RunParams &p)
{
    constexpr int N = NET::N, M = NET::M, NOBS = NET::NOBS, NO = obs_cap(NET::NOBS);
    const int wid = uniform_i((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int item_idx = blockIdx.x * kWaves + wid;
    if (item_idx >= p.n_items) return;
    const LaneItem it = p.items[item_idx];
    const NetDev nd = p.nets[it.net];

    float c[M];
    rates<NET>(p, nd, c);

    const bool valid = lane < it.count;
    const int64_t B = nd.B;
    const int64_t i = it.first + (valid ? lane : 0);
    const int64_t g = nd.traj_off + i;
    const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);

    int X[N + 1];
#pragma unroll
    for (int s = 0; s < N; ++s) X[s] = p.x0[nd.state_off + s * B + i];
    X[N] = 1;

    const bool bins = !GRID && p.obs_kind == 1 && NOBS > 0;
    constexpr bool grid = GRID && NOBS > 0;
    const int n_bins = p.n_bins;
    const double t_obs = nd.t_obs;
    int bin = bins ? 0 : n_bins;
    double bin_hi = bins ? bin_edge(t_obs, 1, n_bins) : INFINITY;
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;
    // tail observation: the states k + 1 >= n_steps - n_bins + 1 (the last
    // n_bins of the run) are summed, counts and clock
    const bool tail = !GRID && p.obs_kind == 3;
    const int tail_k = tail ? p.n_steps - n_bins : 0x7FFFFFFF;
    double tacc[NO], tacc_t = 0.0;
#pragma unroll
    for (int o = 0; o < NO; ++o) tacc[o] = 0.0;
    // observation block [point][obs][B], or [B][point][obs] trajectory-major;
    // the tail observation is [obs + clock][B]
    const int64_t npts = (p.obs_kind != 0 && !tail) ? n_bins : 1;
    const int64_t orow = p.obs_tm ? (int64_t)NOBS : (int64_t)NOBS * B, ocol = p.obs_tm ? 1 : B;
    double *obs_base = p.obs + (tail ? nd.obst_off : nd.obsb_off * npts);
    double *obs_lane = obs_base + (p.obs_tm ? i * npts * NOBS : i);
    // ensemble-mean forward: the wave's fixed-point single-bin sums and its
    // two difference arrays of counts in LDS, cleared here
    extern __shared__ long long s_ens[];
    const int ens_w = n_bins * NOBS;
    long long *sfp = ENS ? s_ens + (int64_t)wid * (2 * ens_w + NOBS) : nullptr;
    int *dsc = ENS ? (int *)(sfp + ens_w) : nullptr;
    int *dun = ENS ? dsc + ens_w + NOBS : nullptr;
    if (ENS) {
        for (int q = lane; q < ens_w; q += 64) sfp[q] = 0;
        for (int q = lane; q < ens_w + NOBS; q += 64) { dsc[q] = 0; dun[q] = 0; }
    }
    // grid observation: next grid point gi, at time grid_t >= t
    int gi = 0;
    double grid_t = grid ? 0.0 : INFINITY;
    const double inv_dt = bins ? (double)n_bins / t_obs : 0.0;
    // bin-edge log: an event time outside (e_lo, e_hi), the current bin
    // narrowed by kEdgeLog at both edges, takes the rare path
    const bool edge_log = bins && p.ties != nullptr;
    double e_lo = -INFINITY, e_hi = edge_log ? bin_hi * (1.0 - kEdgeLog) : INFINITY;

    const int bits = p.tape_bits;
    const int spw = bits ? 32 / bits : 0;
    const int tshift = spw ? __builtin_ctz(spw) : 0;
    uint32_t tword = 0u;

    double t = 0.0;
    bool active = valid;
    int n_done = 0;
    uint32_t flags = 0u;
    int64_t ck_idx = 0;

    // The step body is one straight-line block for every lane: the state
    // updates are predicated on `fire`, and the Philox words of step k+1 are
    // generated inside step k, so the scheduler can interleave that chain
    // with the dependent propensity -> race -> update chain of step k.
    // Per-step bookkeeping stays out of the body: checkpoints are written
    // per segment, the tape word is stored per word, and lanes that stop
    // (absorbing state, t_end) go through the rare path.
    constexpr int NW = CDF ? 4 : Blocks<NET>::W;   // the inverse CDF draws from block 0 only
    uint32_t wd[NW];
    words<NET, NW>(0u, tid, pe, p.seed_lo, p.seed_hi, wd);
    int k = 0;
    bool any = ballot(active) != 0ull;
    while (any && k < p.n_steps) {
      if (p.ck_x) {
          if (active) {
#pragma unroll
              for (int s = 0; s < N; ++s) p.ck_x[ck_idx * p.state_total + nd.state_off + s * B + i] = X[s];
              p.ck_t[ck_idx * p.traj_total + g] = t;
          }
          ck_idx += 1;
      }
      const int seg_end = p.ck_x ? min(k + p.K, p.n_steps) : p.n_steps;
      while (any && k < seg_end) {
        const int word_end = spw ? min((k | (spw - 1)) + 1, seg_end) : seg_end;
        uint32_t shift = spw ? (uint32_t)(bits * (k & (spw - 1))) : 0u;
        for (; k < word_end; ++k) {
        float a[M], A1[M], A2[M];
        const float a0 = propensities<NET, false>(c, X, a, A1, A2);
        const float tau = neglog_u(wd[0]) * fast_rcp(a0);
        const double tn = t + (double)tau;
        float r[M];
        float r1 = INFINITY, r2 = INFINITY;
        int j1 = 0;
        float cdf_gap = INFINITY;     // inverse CDF: distance of u a0 from the nearest interior boundary
        int cdf_side = 0;             // ... and the channel across it
        if (!CDF) {
            // exponential race: smallest and second smallest E_j / a_j
#pragma unroll
            for (int j = 0; j < M; ++j) {
                r[j] = neglog_u(wd[1 + j]) * fast_rcp(a[j]);    // a_j = 0 gives +inf: never fires
                const bool lt = r[j] < r1;
                r2 = lt ? r1 : fminf(r2, r[j]);
                j1 = lt ? j : j1;
                r1 = fminf(r1, r[j]);
            }
        } else {
            // first j whose cumulative propensity (summed in a0's order) exceeds u a0
            const float target = lattice_u(wd[1]) * a0;
            float cs = 0.f;
            bool found = false;
            int last = 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                cs += a[j];
                const bool cross = !found && cs > target;
                j1 = cross ? j : j1;
                found = found || cross;
                last = a[j] > 0.f ? j : last;
                const float d = fabsf(cs - target);
                const bool closer = a[j] > 0.f && cs < a0 && d < cdf_gap;
                cdf_side = closer ? (cs > target ? j + 1 : j) : cdf_side;
                cdf_gap = closer ? d : cdf_gap;
            }
            j1 = found ? j1 : last;
        }
        uint32_t wn[NW];
        words<NET, NW>((uint32_t)(k + 1), tid, pe, p.seed_lo, p.seed_hi, wn);

        const bool live = active && a0 > 0.f;           // a0 = 0: absorbing state
        const bool fire = live && (!HAS_T_END || tn <= p.t_end);
        const bool in_bin = fire && tn <= bin_hi;       // the interval ends inside the current bin
        const double w_obs = in_bin ? (double)tau : 0.0;
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[o] += (double)X[NET::OBS[o]] * w_obs;
        const bool clock_tie = HAS_T_END && live && fabs(tn - p.t_end) <= kClockTieLog * p.t_end;
        const bool near_tie = fire && (CDF ? cdf_gap <= kTieLog * a0 : r2 <= r1 * (1.f + kTieLog));
        const bool crossing = fire && !in_bin && bin < n_bins;
        const bool gcross = grid && fire && grid_t < tn;    // grid points in [t, t + tau)
        const bool odd = active && !(a0 >= 0.f);
        const bool stop = active && !fire;
        const bool edgy = fire && (tn >= e_hi || tn <= e_lo);   // implies crossing when edge_log
        if (ballot(clock_tie || near_tie || crossing || gcross || odd || stop || edgy) != 0ull) {
            if (ballot(stop) != 0ull) any = ballot(fire) != 0ull;
            if (odd) flags |= kFlagNonFinite;
            if (clock_tie)
                log_tie(p, (uint32_t)g, k, fire ? 1 : 0, 0, (float)((tn - p.t_end) / p.t_end), 1);
            if (near_tie) {
                if (CDF) {
                    log_tie(p, (uint32_t)g, k, j1, cdf_side == j1 ? cdf_side - 1 : cdf_side, cdf_gap / a0, 0);
                } else {
                    int j2 = -1;
                    float best = INFINITY;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if (j != j1 && r[j] < best) { best = r[j]; j2 = j; }
                    log_tie(p, (uint32_t)g, k, j1, j2, (r2 - r1) / r1, 0);
                }
            }
            // bins the interval completes
            int run_lo = 0, run_hi = 0, fb = -1;
            double fv[NO];
            if (TMB && crossing) {
                // the first one carries the accumulated integral; the whole
                // bins after it go to the wave-wide fill; the last bin the
                // interval reaches into is found from an estimate and exact
                // comparisons with the edges themselves
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    acc[o] += (double)X[NET::OBS[o]] * fmax(bin_hi - t, 0.0);
                    fv[o] = acc[o] * inv_dt;
                    if (!ENS && o < NOBS) obs_lane[bin * orow + o * ocol] = fv[o];
                    acc[o] = 0.0;
                }
                fb = bin;
                int b = bin + 1;
                if (b < n_bins) {
                    const double est = ceil(tn * (double)n_bins / t_obs) - 1.0;
                    b = !(est > (double)b) ? b : est >= (double)n_bins ? n_bins : (int)est;
                    while (b > bin + 1 && tn <= bin_edge(t_obs, b, n_bins)) --b;
                    while (b < n_bins && tn > bin_edge(t_obs, b + 1, n_bins)) ++b;
                }
                run_lo = bin + 1;
                run_hi = b;
                if (b < n_bins) {
#pragma unroll
                    for (int o = 0; o < NO; ++o) acc[o] += (double)X[NET::OBS[o]] * (tn - bin_edge(t_obs, b, n_bins));
                }
                bin = b;
                bin_hi = b < n_bins ? bin_edge(t_obs, b + 1, n_bins) : INFINITY;
            }
            if (ENS) {
                if (ens_add<NET>(sfp, dsc, dun, fb, fv, run_lo, run_hi, X, true)) flags |= kFlagOverflow;
            } else if (TMB) {
                fill_runs<NET>(obs_base, it.first, npts, run_lo, run_hi, X, true, t_obs, n_bins, inv_dt);
            }
            if (!TMB && crossing) {
                double t0 = t;
                while (bin < n_bins) {
                    const double hi = bin_hi;
                    if (tn <= hi) {
#pragma unroll
                        for (int o = 0; o < NO; ++o) acc[o] += (double)X[NET::OBS[o]] * (tn - t0);
                        break;
                    }
#pragma unroll
                    for (int o = 0; o < NO; ++o) {
                        acc[o] += (double)X[NET::OBS[o]] * fmax(hi - t0, 0.0);
                        if (o < NOBS) obs_lane[bin * orow + o * ocol] = acc[o] * inv_dt;
                        acc[o] = 0.0;
                    }
                    t0 = fmax(t0, hi);
                    bin += 1;
                    bin_hi = bin < n_bins ? bin_edge(t_obs, bin + 1, n_bins) : INFINITY;
                }
            }
            if (edge_log && edgy) {
                // the edges around the bin holding t + tau (edge i is at t_obs i / n_bins)
                const int bl = bin < n_bins ? bin : n_bins;
                const double lo = bl >= 1 ? bin_edge(t_obs, bl, n_bins) : -INFINITY;
                const double hi = bl < n_bins ? bin_edge(t_obs, bl + 1, n_bins) : INFINITY;
                int ei = -1;
                double e = 0.0;
                if (bl >= 1 && fabs(tn - lo) <= kEdgeLog * lo) { ei = bl; e = lo; }
                else if (bl < n_bins && fabs(tn - hi) <= kEdgeLog * hi) { ei = bl + 1; e = hi; }
                if (ei >= 1) log_tie(p, (uint32_t)g, k, tn >= e ? 1 : 0, ei, (float)((tn - e) / e), 2);
                e_lo = bl >= 1 ? lo * (1.0 + kEdgeLog) : -INFINITY;
                e_hi = bl < n_bins ? hi * (1.0 - kEdgeLog) : INFINITY;
            }
            if (gcross) {
                // interpolate between (t, X) and (t + tau, X + v_j)
                const double inv_tau = 1.0 / (double)tau;
                while (grid_t < tn) {
                    const double f = (grid_t - t) * inv_tau;
#pragma unroll
                    for (int o = 0; o < NOBS; ++o) {
                        const double v = (double)X[NET::OBS[o]] + f * (double)delta_of<NET>(j1, NET::OBS[o]);
                        if (ENS) {
                            if (fabs(v) < kEnsMaxCount)
                                atomicAdd((unsigned long long *)&sfp[gi * NOBS + o],
                                          (unsigned long long)(long long)rint(v * kFixScale));
                            else
                                flags |= kFlagOverflow;
                        } else
                            obs_lane[gi * orow + o * ocol] = v;
                    }
                    gi += 1;
                    grid_t = gi < n_bins ? grid_time(t_obs, gi, n_bins) : INFINITY;
                }
            }
        }
        tword |= fire ? (uint32_t)j1 << shift : 0u;
        shift += (uint32_t)bits;
        apply<NET>(X, fire ? j1 : -1, +1);
        t = fire ? tn : t;
        n_done += fire ? 1 : 0;
        active = fire;
        if (k >= tail_k) {
            // state k + 1 (held by a lane that stopped)
#pragma unroll
            for (int o = 0; o < NOBS; ++o) tacc[o] += (double)X[NET::OBS[o]];
            tacc_t += t;
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) wd[q] = wn[q];
        if (!any) {
            ++k;
            break;
        }
        }
        // a completed tape word
        if (spw && (k & (spw - 1)) == 0) {
            if (valid) p.tape[(int64_t)((k - 1) >> tshift) * p.traj_total + g] = tword;
            tword = 0u;
        }
      }
    }
    // hold the last state up to t_obs: the rest of the current bin, then every
    // later bin, whose average is the last state itself
    if (ENS && grid) {
        // grid points at or after the last event hold the last state
        const bool tail = valid && gi < n_bins;
        double fv[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) fv[o] = 0.0;
        if (ens_add<NET>(sfp, dsc, dun, -1, fv, tail ? gi : 0, tail ? n_bins : 0, X, false)) flags |= kFlagOverflow;
    } else if (ENS) {
        const bool tail = valid && bin < n_bins;
        double fv[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o)
            fv[o] = (acc[o] + (double)X[NET::OBS[o]] * fmax(fmin(bin_hi, t_obs) - t, 0.0)) * inv_dt;
        if (ens_add<NET>(sfp, dsc, dun, tail ? bin : -1, fv, tail ? bin + 1 : 0, tail ? n_bins : 0, X, false))
            flags |= kFlagOverflow;
    }
    if (ENS) {
        // every lane's additions land before the row is read back
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        ens_row<NET>(p.tile_sums + nd.tobs_off * n_bins + (int64_t)(it.first >> 6) * n_bins * NOBS, sfp, dsc, dun,
                     n_bins, t_obs, inv_dt);
    } else if (TMB) {
        fill_runs<NET>(obs_base, it.first, npts, valid && bin < n_bins ? bin + 1 : 0,
                       valid && bin < n_bins ? n_bins : 0, X, false, t_obs, n_bins, inv_dt);
    }
    if (!valid) return;
    if (spw && (k & (spw - 1)) != 0) p.tape[(int64_t)(k >> tshift) * p.traj_total + g] = tword;
    if (tail) {
        // the tail states past the last step every lane of the wave stopped at hold the last one
        const int rem = p.n_steps - max(k, tail_k);
        if (rem > 0) {
#pragma unroll
            for (int o = 0; o < NOBS; ++o) tacc[o] += (double)rem * (double)X[NET::OBS[o]];
            tacc_t += (double)rem * t;
        }
        const double inv_m = 1.0 / (double)n_bins;
#pragma unroll
        for (int o = 0; o < NOBS; ++o) obs_lane[o * B] = tacc[o] * inv_m;
        obs_lane[NOBS * B] = tacc_t * inv_m;
    }
    if (!ENS && bin < n_bins) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            acc[o] += (double)X[NET::OBS[o]] * fmax(fmin(bin_hi, t_obs) - t, 0.0);
            if (o < NOBS) obs_lane[bin * orow + o * ocol] = acc[o] * inv_dt;
        }
        // rows from the top down, so the wave's lanes store the same row
        // together whatever bin each of them stopped in
        if (!TMB)
            for (int bb = n_bins - 1; bb > bin; --bb)
#pragma unroll
                for (int o = 0; o < NOBS; ++o) obs_lane[bb * orow + o * ocol] = (double)X[NET::OBS[o]];
    }
    if (p.obs_kind == 0) {
#pragma unroll
        for (int o = 0; o < NOBS; ++o) obs_lane[o * ocol] = (double)X[NET::OBS[o]];
    }
    // grid points after the last event hold the last state
    if (grid && !ENS)
        for (int gg = n_bins - 1; gg >= gi; --gg)
#pragma unroll
            for (int o = 0; o < NOBS; ++o) obs_lane[gg * orow + o * ocol] = (double)X[NET::OBS[o]];
#pragma unroll
    for (int s = 0; s < N; ++s) {
        p.x_final[nd.state_off + s * B + i] = X[s];
        if (X[s] < 0) flags |= kFlagOverflow;
    }
    p.t_final[g] = t;
    p.steps_done[g] = n_done;
    if (flags) atomicOr(p.flags, flags);
}

template <class NET, bool GRID, bool CDF = false, bool TMB = false, bool ENS = false>
__device__ void forward(const RunParams &p)
{
    if (p.t_end < INFINITY) forward_run<NET, true, GRID, CDF, TMB, ENS>(p);
    else forward_run<NET, false, GRID, CDF, TMB, ENS>(p);
}

// --------------------------------------------------------------------------
// Forward-mode tangents (SSA_BWD_TANGENT).  For a network with few channels
// the forward carries, for every channel rate q, the tangents dX/d ln k_q and
// dt/d ln k_q of the straight-through surrogate along the path it fires, and
// writes d obs / d ln k_q; the gradient of any loss is then the contraction of
// those with dL/dobs, and no reverse sweep, checkpoint or tape is needed.  The
// surrogate is the one the backward differentiates (Eq. 5):
//   X_{k+1} = X_k + sum_j v_j (y_j + y~_j - stopgrad(y~_j)),
//   t_{k+1} = t_k + E_0 / a0(X_k),
// so per step d y~_j = y~_j (dz_j - sum_i y~_i dz_i) with
// dz_j = d ln a_j / T, d tau = -(tau / a0) d a0, and the bin averages move
// with the state tangents inside each interval and with the clock tangents
// at its ends.  Forward and reverse accumulation of one function's
// derivative agree; the rounding differs.  Final and bin observations
// (point-major), step-limited runs.
template <class NET>
constexpr bool tangent_fits()
{
    return NET::M <= kTanMaxChannels && NET::N * NET::M <= kTanMaxStateTangents;
}

template <class NET>
__device__ void forward_tangent(const RunParams &p)
{
    if constexpr (tangent_fits<NET>()) {
    constexpr int N = NET::N, M = NET::M, NOBS = NET::NOBS, NO = obs_cap(NET::NOBS);
    const int wid = uniform_i((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int item_idx = blockIdx.x * kWaves + wid;
    if (item_idx >= p.n_items) return;
    const LaneItem it = p.items[item_idx];
    const NetDev nd = p.nets[it.net];

    float c[M];
    rates<NET>(p, nd, c);

    const bool valid = lane < it.count;
    const int64_t B = nd.B;
    const int64_t i = it.first + (valid ? lane : 0);
    const int64_t g = nd.traj_off + i;
    const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);
    const float T = run_temperature(p);
    const float invT = 1.0f / T;

    int X[N + 1];
#pragma unroll
    for (int s = 0; s < N; ++s) X[s] = p.x0[nd.state_off + s * B + i];
    X[N] = 1;
    // tangents: the initial state does not depend on the rates
    double dX[N][M], dt[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
        dt[q] = 0.0;
#pragma unroll
        for (int s = 0; s < N; ++s) dX[s][q] = 0.0;
    }

    const bool bins = p.obs_kind == 1 && NOBS > 0;
    const int n_bins = p.n_bins;
    const double t_obs = nd.t_obs;
    int bin = bins ? 0 : n_bins;
    double bin_hi = bins ? bin_edge(t_obs, 1, n_bins) : INFINITY;
    double acc[NO], dacc[NO][M];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        acc[o] = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) dacc[o][q] = 0.0;
    }
    const int64_t npts = p.obs_kind != 0 ? n_bins : 1;
    double *obs_lane = p.obs + nd.obsb_off * npts + i;
    double *tan_lane = p.tangent + nd.tanw_off * npts + i;
    const int64_t orow = (int64_t)NOBS * B;
    const int64_t trow = (int64_t)NOBS * M * B;     // [point][obs][channel][B]
    const double inv_dt = bins ? (double)n_bins / t_obs : 0.0;
    const bool edge_log = bins && p.ties != nullptr;
    double e_lo = -INFINITY, e_hi = edge_log ? bin_hi * (1.0 - kEdgeLog) : INFINITY;

    double t = 0.0;
    bool active = valid;
    int n_done = 0;
    uint32_t flags = 0u;

    constexpr int NW = Blocks<NET>::W;
    uint32_t wd[NW];
    words<NET, NW>(0u, tid, pe, p.seed_lo, p.seed_hi, wd);
    bool any = ballot(active) != 0ull;
    int k = 0;
    for (; any && k < p.n_steps; ++k) {
        float a[M], A1[M], A2[M];
        const float a0 = propensities<NET, true>(c, X, a, A1, A2);
        const float tau = neglog_u(wd[0]) * fast_rcp(a0);
        const double tn = t + (double)tau;
        float r[M];
        float r1 = INFINITY, r2 = INFINITY;
        int j1 = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            r[j] = neglog_u(wd[1 + j]) * fast_rcp(a[j]);
            const bool lt = r[j] < r1;
            r2 = lt ? r1 : fminf(r2, r[j]);
            j1 = lt ? j : j1;
            r1 = fminf(r1, r[j]);
        }
        uint32_t wn[NW];
        words<NET, NW>((uint32_t)(k + 1), tid, pe, p.seed_lo, p.seed_hi, wn);

        const bool fire = active && a0 > 0.f;
        const bool in_bin = fire && tn <= bin_hi;
        const bool near_tie = fire && r2 <= r1 * (1.f + kTieLog);
        const bool crossing = fire && !in_bin && bin < n_bins;
        const bool odd = active && !(a0 >= 0.f);
        const bool stop = active && !fire;
        const bool edgy = fire && (tn >= e_hi || tn <= e_lo);

        // tangents of this step: d a_j / d ln k_q at X_k, the soft sample and
        // its derivative, d tau
        float dXf[N + 1][M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
#pragma unroll
            for (int s = 0; s < N; ++s) dXf[s][q] = (float)dX[s][q];
            dXf[N][q] = 0.f;
        }
        float y[M], ysum = 0.f;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const float rho = r[j] == r1 ? 1.0f : r1 * fast_rcp(r[j]);      // a_j = 0: r = inf, rho = 0
            float w = rho;
            if (T == 0.5f) w = rho * rho;
            else if (T != 1.0f) w = rho > 0.f ? exp2f(log2f(rho) * invT) : 0.f;
            y[j] = w;
            ysum += w;
        }
        const float rys = fast_rcp(ysum);
        const float rcp_a0 = fast_rcp(a0);
        float dtau[M], dy[M][M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            // dy_j = y~_j sum_i y~_i (dz_j - dz_i), with the differences taken
            // against the fired channel first: the fired channel's y~ is close
            // to 1 at low T, and dz_j - sum_i y~_i dz_i would cancel
            float da0 = 0.f;
            float dz[M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const float da = (j == q ? a[j] : 0.f) + A2[j] * dXf[NET::S1[j]][q] + A1[j] * dXf[NET::S2[j]][q];
                da0 += da;
                dz[j] = a[j] > 0.f ? da * fast_rcp(a[j]) * invT : 0.f;
            }
            float dzref = dz[0];
#pragma unroll
            for (int j = 1; j < M; ++j) dzref = j == j1 ? dz[j] : dzref;
            float zbar = 0.f;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                dz[j] -= dzref;
                zbar += y[j] * rys * dz[j];
            }
            dtau[q] = -tau * rcp_a0 * da0;
#pragma unroll
            for (int j = 0; j < M; ++j) dy[j][q] = y[j] * rys * (dz[j] - zbar);
        }

        if (ballot(near_tie || crossing || odd || stop || edgy) != 0ull) {
            if (ballot(stop) != 0ull) any = ballot(fire) != 0ull;
            if (odd) flags |= kFlagNonFinite;
            if (near_tie) {
                int j2 = -1;
                float best = INFINITY;
#pragma unroll
                for (int j = 0; j < M; ++j)
                    if (j != j1 && r[j] < best) { best = r[j]; j2 = j; }
                log_tie(p, (uint32_t)g, k, j1, j2, (r2 - r1) / r1, 0);
            }
            if (crossing) {
                // the bins the interval completes: their averages and tangents
                double t0 = t;
                bool first = true;
                while (bin < n_bins) {
                    const double hi = bin_hi;
                    if (tn <= hi) {
#pragma unroll
                        for (int o = 0; o < NO; ++o) {
                            const double xo = (double)X[NET::OBS[o]];
                            acc[o] += xo * (tn - t0);
#pragma unroll
                            for (int q = 0; q < M; ++q)
                                dacc[o][q] += (double)dXf[NET::OBS[o]][q] * (tn - t0) +
                                              xo * (first ? (double)dtau[q] : dt[q] + (double)dtau[q]);
                        }
                        break;
                    }
                    const double seg = fmax(hi - t0, 0.0);
#pragma unroll
                    for (int o = 0; o < NO; ++o) {
                        const double xo = (double)X[NET::OBS[o]];
                        acc[o] += xo * seg;
                        if (o < NOBS) obs_lane[bin * orow + o * B] = acc[o] * inv_dt;
                        acc[o] = 0.0;
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            dacc[o][q] += (double)dXf[NET::OBS[o]][q] * seg - (first && seg > 0.0 ? xo * dt[q] : 0.0);
                            if (o < NOBS) tan_lane[bin * trow + (o * M + q) * B] = dacc[o][q] * inv_dt;
                            dacc[o][q] = 0.0;
                        }
                    }
                    first = false;
                    t0 = fmax(t0, hi);
                    bin += 1;
                    bin_hi = bin < n_bins ? bin_edge(t_obs, bin + 1, n_bins) : INFINITY;
                }
            }
            if (edge_log && edgy) {
                const int bl = bin < n_bins ? bin : n_bins;
                const double lo = bl >= 1 ? bin_edge(t_obs, bl, n_bins) : -INFINITY;
                const double hi = bl < n_bins ? bin_edge(t_obs, bl + 1, n_bins) : INFINITY;
                int ei = -1;
                double e = 0.0;
                if (bl >= 1 && fabs(tn - lo) <= kEdgeLog * lo) { ei = bl; e = lo; }
                else if (bl < n_bins && fabs(tn - hi) <= kEdgeLog * hi) { ei = bl + 1; e = hi; }
                if (ei >= 1) log_tie(p, (uint32_t)g, k, tn >= e ? 1 : 0, ei, (float)((tn - e) / e), 2);
                e_lo = bl >= 1 ? lo * (1.0 + kEdgeLog) : -INFINITY;
                e_hi = bl < n_bins ? hi * (1.0 - kEdgeLog) : INFINITY;
            }
        }
        if (in_bin) {
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const double xo = (double)X[NET::OBS[o]];
                acc[o] += xo * (double)tau;
#pragma unroll
                for (int q = 0; q < M; ++q)
                    dacc[o][q] += (double)(dXf[NET::OBS[o]][q] * tau) + xo * (double)dtau[q];
            }
        }
        if (fire) {
#pragma unroll
            for (int s = 0; s < N; ++s)
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    float dv = 0.f;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if (NET::V[j][s] != 0) dv += (float)NET::V[j][s] * dy[j][q];
                    dX[s][q] += (double)dv;
                }
#pragma unroll
            for (int q = 0; q < M; ++q) dt[q] += (double)dtau[q];
        }
        apply<NET>(X, fire ? j1 : -1, +1);
        t = fire ? tn : t;
        n_done += fire ? 1 : 0;
        active = fire;
#pragma unroll
        for (int q = 0; q < NW; ++q) wd[q] = wn[q];
    }
    if (!valid) return;
    if (bin < n_bins) {
        // hold the last state up to t_obs: the rest of the current bin, then
        // every later bin, whose average is the last state itself
        const double seg = fmax(fmin(bin_hi, t_obs) - t, 0.0);
#pragma unroll
        for (int o = 0; o < NOBS; ++o) {
            const double xo = (double)X[NET::OBS[o]];
            obs_lane[bin * orow + o * B] = (acc[o] + xo * seg) * inv_dt;
#pragma unroll
            for (int q = 0; q < M; ++q)
                tan_lane[bin * trow + (o * M + q) * B] =
                    (dacc[o][q] + dX[NET::OBS[o]][q] * seg - (seg > 0.0 ? xo * dt[q] : 0.0)) * inv_dt;
        }
        for (int bb = n_bins - 1; bb > bin; --bb)
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                obs_lane[bb * orow + o * B] = (double)X[NET::OBS[o]];
#pragma unroll
                for (int q = 0; q < M; ++q) tan_lane[bb * trow + (o * M + q) * B] = dX[NET::OBS[o]][q];
            }
    }
    if (p.obs_kind == 0) {
#pragma unroll
        for (int o = 0; o < NOBS; ++o) {
            obs_lane[o * B] = (double)X[NET::OBS[o]];
#pragma unroll
            for (int q = 0; q < M; ++q) tan_lane[(o * M + q) * B] = dX[NET::OBS[o]][q];
        }
    }
#pragma unroll
    for (int s = 0; s < N; ++s) {
        p.x_final[nd.state_off + s * B + i] = X[s];
        if (X[s] < 0) flags |= kFlagOverflow;
    }
    p.t_final[g] = t;
    p.steps_done[g] = n_done;
    if (flags) atomicOr(p.flags, flags);
    }
}

// --------------------------------------------------------------------------
// TMODE: 2 -> T = 1/2 (y~ ~ rho^2), 1 -> T = 1 (y~ ~ rho), 0 -> y~ ~ rho^(1/T).
// RECOMPUTE: the choices of a segment come from re-running it into LDS
// instead of the tape.
constexpr int kRecSteps = 64;   // recompute mode: steps of a segment kept in LDS

// SH: bin observations with one dL/dobs block shared by the trajectories,
// whose per-species prefix sums over the bins (p.dobs_prefix) give the
// contribution of every whole bin an interval spans in one difference.
template <class NET, int TMODE, bool RECOMPUTE, bool GRID, bool SH = false>
__device__ void backward_run(const RunParams &p, uint8_t (*s_tape)[kRecSteps][64])
{
    constexpr int N = NET::N, M = NET::M, NOBS = NET::NOBS, NO = obs_cap(NET::NOBS);

    const int wid = uniform_i((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int item_idx = blockIdx.x * kWaves + wid;
    if (item_idx >= p.n_items) return;
    const LaneItem it = p.items[item_idx];
    const NetDev nd = p.nets[it.net];

    float c[M];
    rates<NET>(p, nd, c);

    const bool valid = lane < it.count;
    const int64_t B = nd.B;
    const int64_t i = it.first + (valid ? lane : 0);
    const int64_t g = nd.traj_off + i;
    const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);
    const float invT = 1.0f / run_temperature(p);

    const int n = valid ? p.steps_done[g] : 0;
    int kmax = n;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) kmax = max(kmax, __shfl_xor(kmax, off));
    kmax = uniform_i(kmax);
    // smallest step count of the wave's valid lanes (lanes past the tile count nothing)
    int nmin = valid ? n : kmax;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) nmin = min(nmin, __shfl_xor(nmin, off));
    nmin = uniform_i(nmin);

    int X[N + 1];
#pragma unroll
    for (int s = 0; s < N; ++s) X[s] = valid ? p.x_final[nd.state_off + s * B + i] : 0;
    X[N] = 1;
    double t = valid ? p.t_final[g] : 0.0;

    const bool bins = !GRID && p.obs_kind == 1 && NOBS > 0;
    constexpr bool grid = GRID && NOBS > 0;
    const int n_bins = p.n_bins;
    const double t_obs = nd.t_obs;
    const double inv_dt = bins ? (double)n_bins / t_obs : 0.0;
    // tail observation: the states X_k, k >= tail_lo, enter the means
    const bool tail = !GRID && p.obs_kind == 3;
    const int tail_lo = tail ? p.n_steps - n_bins + 1 : 0x7FFFFFFF;
    // dL/dobs in the observation layout, or one block per network shared by
    // its trajectories
    const int64_t npts = (p.obs_kind != 0 && !tail) ? n_bins : 1;
    const bool dtm = p.obs_tm || p.dobs_shared;
    const int64_t drow = dtm ? (int64_t)NOBS : (int64_t)NOBS * B, dcol = dtm ? 1 : B;
    const double *dobs_lane = p.d_obs + (tail ? nd.obst_off + i
                                         : p.dobs_shared ? nd.obsw_off * npts
                                         : nd.obsb_off * npts + (p.obs_tm ? i * npts * NOBS : i));
    // tail: dL/dobs over the tail length, per observed count and for the clock
    float tdo[NO];
    double tdt = 0.0;
#pragma unroll
    for (int o = 0; o < NO; ++o) tdo[o] = 0.f;
    // prefix sums [obs][n_bins + 1] of the shared block (SH)
    const double *pre = SH ? p.dobs_prefix + nd.obsw_off * (int64_t)(n_bins + 1) : nullptr;

    // adjoint of the state: FP64 accumulator, FP32 increments folded every kFold steps
    double lam[N];
    float lam32[N], dlam[N];
#pragma unroll
    for (int s = 0; s < N; ++s) { lam[s] = 0.0; dlam[s] = 0.f; }
    double lam_t = 0.0;
    double dth[M];
    float dth32[M];
#pragma unroll
    for (int j = 0; j < M; ++j) { dth[j] = 0.0; dth32[j] = 0.f; }

    // reverse-time bin tracker; doi = dL/dobs of the current bin / bin width
    int rbin = n_bins;
    double rlo = t_obs;
    double doi[NO];
    float doi32[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) { doi[o] = 0.0; doi32[o] = 0.f; }
    if (valid) {
        if (bins && t < t_obs) {
            // the bin holding the last event's time: an estimate, then exact
            // comparisons with the bin edges themselves
            const double est = floor(t * (double)n_bins / t_obs);
            int b = !(est > 0.0) ? 0 : est >= (double)n_bins ? n_bins - 1 : (int)est;
            while (b > 0 && t < bin_edge(t_obs, b, n_bins)) --b;
            while (b + 1 < n_bins && t >= bin_edge(t_obs, b + 1, n_bins)) ++b;
            // later bins average the held final state: their dL/dobs go to it whole
            if (SH) {
#pragma unroll
                for (int o = 0; o < NOBS; ++o)
                    lam[NET::OBS[o]] += pre[o * (n_bins + 1) + n_bins] - pre[o * (n_bins + 1) + b + 1];
            } else {
                for (int bb = n_bins - 1; bb > b; --bb)
#pragma unroll
                    for (int o = 0; o < NOBS; ++o) lam[NET::OBS[o]] += dobs_lane[bb * drow + o * dcol];
            }
            // and the part of bin b after the last event
            rbin = b;
            rlo = b > 0 ? bin_edge(t_obs, b, n_bins) : -INFINITY;
            const double hi = b + 1 < n_bins ? bin_edge(t_obs, b + 1, n_bins) : t_obs;
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                doi[o] = o < NOBS ? dobs_lane[b * drow + o * dcol] * inv_dt : 0.0;
                doi32[o] = (float)doi[o];
            }
#pragma unroll
            for (int o = 0; o < NOBS; ++o) lam[NET::OBS[o]] += doi[o] * (hi - t);
        } else if (p.obs_kind == 0) {
#pragma unroll
            for (int o = 0; o < NOBS; ++o) lam[NET::OBS[o]] += dobs_lane[o * dcol];
        } else if (tail) {
            // X_n, t_n and the held copies of them among the tail states
            const double inv_m = 1.0 / (double)n_bins;
            const int first = max(n, tail_lo);
            const double wf = (double)(p.n_steps + 1 - first) * inv_m;
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                const double d = dobs_lane[o * B];
                tdo[o] = (float)(d * inv_m);
                if (wf > 0.0) lam[NET::OBS[o]] += d * wf;
            }
            const double dt_ = dobs_lane[NOBS * B];
            tdt = dt_ * inv_m;
            if (wf > 0.0) lam_t += dt_ * wf;
        }
    }
    // grid observation: the points at or after the last event see the final
    // state; gh counts the points below the current clock, glo is the time of
    // the highest of them (the next one the reverse sweep meets)
    int gh = 0;
    double glo = -INFINITY;
    double gd[NO];                     // dL/dobs of grid point gh - 1, loaded ahead
#pragma unroll
    for (int o = 0; o < NO; ++o) gd[o] = 0.0;
    if (grid) {
        if (valid) {
            // first grid index whose time is >= t: an estimate, then exact
            // comparisons with the grid times themselves
            const double est = ceil(t * (double)(n_bins - 1) / t_obs);
            gh = !(est > 0.0) ? 0 : est > (double)n_bins ? n_bins : (int)est;
            while (gh > 0 && grid_time(t_obs, gh - 1, n_bins) >= t) --gh;
            while (gh < n_bins && grid_time(t_obs, gh, n_bins) < t) ++gh;
            for (int g = gh; g < n_bins; ++g)
#pragma unroll
                for (int o = 0; o < NOBS; ++o) lam[NET::OBS[o]] += dobs_lane[g * drow + o * dcol];
        }
        glo = gh > 0 ? grid_time(t_obs, gh - 1, n_bins) : -INFINITY;
        if (gh > 0)
#pragma unroll
            for (int o = 0; o < NOBS; ++o) gd[o] = dobs_lane[(gh - 1) * drow + o * dcol];
    }
#pragma unroll
    for (int s = 0; s < N; ++s) lam32[s] = (float)lam[s];

    const int spw = p.tape_bits ? 32 / p.tape_bits : 1;
    const int tshift = __builtin_ctz(spw);
    const uint32_t tmask = p.tape_bits ? ((1u << p.tape_bits) - 1u) : 0u;
    const int n_seg = (kmax + p.K - 1) / p.K;
    int fold_left = kFold;

    for (int cseg = n_seg - 1; cseg >= 0; --cseg) {
        const int k_lo = cseg * p.K;
        const int k_hi = min(k_lo + p.K, kmax);
        if (RECOMPUTE) {
            int Xr[N + 1];
            if (k_lo < n) {
#pragma unroll
                for (int s = 0; s < N; ++s)
                    Xr[s] = p.ck_x[(int64_t)cseg * p.state_total + nd.state_off + s * B + i];
            } else {
#pragma unroll
                for (int s = 0; s < N; ++s) Xr[s] = X[s];
            }
            Xr[N] = 1;
            for (int k = k_lo; k < k_hi; ++k) {
                if (k >= n) continue;
                float a[M], A1[M], A2[M];
                propensities<NET, false>(c, Xr, a, A1, A2);
                uint32_t wd[Blocks<NET>::W];
                words<NET>((uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, wd);
                float r1 = INFINITY;
                int j1 = 0;
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const float rj = neglog_u(wd[1 + j]) * fast_rcp(a[j]);
                    j1 = rj < r1 ? j : j1;
                    r1 = fminf(r1, rj);
                }
                s_tape[wid][k - k_lo][lane] = (uint8_t)j1;
                apply<NET>(Xr, j1, +1);
            }
        }
        if (k_hi < n) {
            const int64_t c1 = cseg + 1;
#pragma unroll
            for (int s = 0; s < N; ++s) X[s] = p.ck_x[c1 * p.state_total + nd.state_off + s * B + i];
            t = p.ck_t[c1 * p.traj_total + g];
        }
        uint32_t tword = 0u;
        int tword_idx = -1;
        // one reverse step k for a lane that fired it: X_{k+1} -> X_k and the
        // adjoint recursion; e holds -ln u of the words of step k (e[0] for
        // the waiting time, e[1 + q] for channel q)
        auto sweep = [&](int k, int j, const float (&e)[M + 1]) {
                int Xn[NOBS > 0 ? NOBS : 1];
    #pragma unroll
                for (int o = 0; o < NOBS; ++o) Xn[o] = X[NET::OBS[o]];
                apply<NET>(X, j, -1);        // X_{k+1} -> X_k

                float a[M], A1[M], A2[M];
                const float a0 = propensities<NET, true>(c, X, a, A1, A2);
                const float rcp_a0 = fast_rcp(a0);
                const float tau = e[0] * rcp_a0;
                const double t_k = t - (double)tau;

                // direct dL/dt_{k+1} (doi is 0 past the observation window)
                if (bins) {
    #pragma unroll
                    for (int o = 0; o < NOBS; ++o)
                        lam_t += doi[o] * (double)(X[NET::OBS[o]] - Xn[o]);
                }
                // grid points in [t_k, t_{k+1}) see X_k + f (X_{k+1} - X_k),
                // f = (t_g - t_k) / tau: their X_{k+1} and t_{k+1} parts join
                // the adjoints this step reads, the X_k and t_k parts are
                // added after it
                float gx[NO];
    #pragma unroll
                for (int o = 0; o < NO; ++o) gx[o] = 0.f;
                double glt = 0.0;
                if (grid && ballot(gh > 0 && glo >= t_k) != 0ull) {
                    const double inv_tau = 1.0 / (double)tau;
                    while (gh > 0 && glo >= t_k) {
                        const double f = (glo - t_k) * inv_tau;
    #pragma unroll
                        for (int o = 0; o < NOBS; ++o) {
                            const double d = gd[o];
                            const double ddv = d * (double)(Xn[o] - X[NET::OBS[o]]) * inv_tau;
                            dlam[NET::OBS[o]] += (float)(d * f);
                            lam_t -= ddv * f;
                            gx[o] += (float)(d * (1.0 - f));
                            glt += ddv * (f - 1.0);
                        }
                        gh -= 1;
                        glo = gh > 0 ? grid_time(t_obs, gh - 1, n_bins) : -INFINITY;
                        if (gh > 0)
    #pragma unroll
                            for (int o = 0; o < NOBS; ++o) gd[o] = dobs_lane[(gh - 1) * drow + o * dcol];
                    }
                }
                // soft sample y~ in ratio form: y~_q ~ (r_j / r_q)^(1/T) with j
                // the fired channel; a_q = 0 gives r_q = +inf and y~_q = 0
                // without a branch
                float r[M], ra[M];
    #pragma unroll
                for (int q = 0; q < M; ++q) {
                    const float rq = fast_rcp(a[q]);
                    ra[q] = a[q] > 0.f ? rq : 0.f;
                    r[q] = e[1 + q] * rq;
                }
                float rref = r[0];
    #pragma unroll
                for (int q = 1; q < M; ++q) rref = (q == j) ? r[q] : rref;
                float y[M];
    #pragma unroll
                for (int q = 0; q < M; ++q) y[q] = rref * fast_rcp(r[q]);
                if (TMODE == 2) {
    #pragma unroll
                    for (int q = 0; q < M; ++q) y[q] = y[q] * y[q];
                } else if (TMODE == 0) {
    #pragma unroll
                    for (int q = 0; q < M; ++q) y[q] = y[q] > 0.f ? exp2f(log2f(y[q]) * invT) : 0.f;
                }
                float ysum = 0.f;
    #pragma unroll
                for (int q = 0; q < M; ++q) ysum += y[q];
                const float rys = fast_rcp(ysum);
                // w_q = v_q . lambda(k+1)
                float wv[M];
    #pragma unroll
                for (int q = 0; q < M; ++q) {
                    float s = 0.f;
    #pragma unroll
                    for (int sp = 0; sp < N; ++sp)
                        if (NET::V[q][sp] != 0) s += (float)NET::V[q][sp] * (lam32[sp] + dlam[sp]);
                    wv[q] = s;
                }
                float wref = wv[0];
    #pragma unroll
                for (int q = 1; q < M; ++q) wref = (q == j) ? wv[q] : wref;
                float wbar = 0.f;
    #pragma unroll
                for (int q = 0; q < M; ++q) {
                    y[q] *= rys;
                    wbar += y[q] * (wv[q] - wref);
                }
                const float cc = (float)lam_t * (-tau * rcp_a0);
    #pragma unroll
                for (int q = 0; q < M; ++q) {
                    const float gq = y[q] * ((wv[q] - wref) - wbar) * invT;
                    dth32[q] += gq + cc * a[q];
                    const float coef = gq * ra[q] + cc;
                    if (NET::S1[q] < N) dlam[NET::S1[q]] += coef * A2[q];
                    if (NET::S2[q] < N) dlam[NET::S2[q]] += coef * A1[q];
                }
                // direct dL/dX_k over [t_k, t_{k+1}); crossing a bin edge is rare
                if (bins) {
                    double hi = t < t_obs ? t : t_obs;
                    // below the first bin's edge rlo is -inf: nothing left to cross
                    if (SH && ballot(t_k < rlo) != 0ull) {
                        if (t_k < rlo) {
                            // the rest of the current bin, then the bin b that
                            // holds t_k (an estimate, then exact comparisons
                            // with the edges), and the whole bins between from
                            // the prefix sums (width / bin width = 1)
                            if (rbin < n_bins) {
                                const double seg = fmax(hi - rlo, 0.0);
    #pragma unroll
                                for (int o = 0; o < NOBS; ++o) dlam[NET::OBS[o]] += (float)(doi[o] * seg);
                            }
                            const double est = floor(t_k * (double)n_bins / t_obs);
                            int b = !(est > 0.0) ? 0 : est >= (double)(rbin - 1) ? rbin - 1 : (int)est;
                            while (b > 0 && t_k < bin_edge(t_obs, b, n_bins)) --b;
                            while (b + 1 < rbin && t_k >= bin_edge(t_obs, b + 1, n_bins)) ++b;
                            if (rbin > b + 1) {
    #pragma unroll
                                for (int o = 0; o < NOBS; ++o)
                                    dlam[NET::OBS[o]] += (float)(pre[o * (n_bins + 1) + rbin] -
                                                                 pre[o * (n_bins + 1) + b + 1]);
                            }
                            hi = b + 1 == rbin ? fmin(hi, rlo) : bin_edge(t_obs, b + 1, n_bins);
                            rbin = b;
                            rlo = b > 0 ? bin_edge(t_obs, b, n_bins) : -INFINITY;
    #pragma unroll
                            for (int o = 0; o < NO; ++o) {
                                doi[o] = o < NOBS ? dobs_lane[rbin * drow + o * dcol] * inv_dt : 0.0;
                                doi32[o] = (float)doi[o];
                            }
                        }
                    } else if (!SH && ballot(t_k < rlo) != 0ull)
                    while (t_k < rlo) {
                        if (rbin < n_bins) {
                            const double seg = fmax(hi - rlo, 0.0);
    #pragma unroll
                            for (int o = 0; o < NOBS; ++o) dlam[NET::OBS[o]] += (float)(doi[o] * seg);
                        }
                        hi = fmin(hi, rlo);
                        rbin -= 1;
                        rlo = rbin > 0 ? bin_edge(t_obs, rbin, n_bins) : -INFINITY;
    #pragma unroll
                        for (int o = 0; o < NO; ++o) {
                            doi[o] = o < NOBS ? dobs_lane[rbin * drow + o * dcol] * inv_dt : 0.0;
                            doi32[o] = (float)doi[o];
                        }
                    }
                    const float seg = fmaxf((float)(hi - t_k), 0.f);
    #pragma unroll
                    for (int o = 0; o < NOBS; ++o) dlam[NET::OBS[o]] += seg * doi32[o];
                }
                if (grid) {
    #pragma unroll
                    for (int o = 0; o < NOBS; ++o) dlam[NET::OBS[o]] += gx[o];
                    lam_t += glt;
                }
                // X_k and t_k as tail states
                if (k >= tail_lo) {
    #pragma unroll
                    for (int o = 0; o < NOBS; ++o) dlam[NET::OBS[o]] += tdo[o];
                    lam_t += tdt;
                }
            t = t_k;
        };
        auto choice = [&](int k) -> int {
            if (RECOMPUTE) return (int)s_tape[wid][k - k_lo][lane];
            const int widx = k >> tshift;
            if (widx != tword_idx) {
                tword = p.tape[(int64_t)widx * p.traj_total + g];
                tword_idx = widx;
            }
            return (int)((tword >> (p.tape_bits * (k & (spw - 1)))) & tmask);
        };
        // the FP32 increments go into the FP64 accumulators once kFold steps
        // have been swept since the last fold
        auto fold = [&](int steps) {
            fold_left -= steps;
            if (fold_left <= 0) {
#pragma unroll
                for (int s = 0; s < N; ++s) {
                    lam[s] += (double)dlam[s];
                    dlam[s] = 0.f;
                    lam32[s] = (float)lam[s];
                }
#pragma unroll
                for (int j = 0; j < M; ++j) { dth[j] += (double)dth32[j]; dth32[j] = 0.f; }
                fold_left = kFold;
            }
        };
        // steps some lanes of the wave never fired (they ended early): masked
        const int k_split = max(min(k_hi, nmin), k_lo);
        for (int k = k_hi - 1; k >= k_split; --k) {
            const int j = choice(k);
            if (k < n) {
                uint32_t w[Blocks<NET>::W];
                words<NET>((uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, w);
                float e[M + 1];
#pragma unroll
                for (int q = 0; q <= M; ++q) e[q] = neglog_u(w[q]);
                sweep(k, j, e);
            }
            fold(1);
        }
        // steps every lane fired: straight-line body, the noise of step k-1
        // (Philox words and their logarithms) computed while step k is swept;
        // the choices are read one tape word (or, recomputing, one segment)
        // at a time
        if (k_split > k_lo) {
            float ed[M + 1];
            {
                uint32_t wd[Blocks<NET>::W];
                words<NET>((uint32_t)(k_split - 1), tid, pe, p.seed_lo, p.seed_hi, wd);
#pragma unroll
                for (int q = 0; q <= M; ++q) ed[q] = neglog_u(wd[q]);
            }
            int k = k_split - 1;
            // the tape word of the next (lower) block is loaded one block ahead
            uint32_t tw_next = RECOMPUTE ? 0u : p.tape[(int64_t)(k >> tshift) * p.traj_total + g];
            while (k >= k_lo) {
                const int w_lo = RECOMPUTE ? k_lo : max(k & ~(spw - 1), k_lo);
                const uint32_t tw = tw_next;
                if (!RECOMPUTE && w_lo > k_lo)
                    tw_next = p.tape[(int64_t)((w_lo - 1) >> tshift) * p.traj_total + g];
                int shift = RECOMPUTE ? 0 : p.tape_bits * (k & (spw - 1));
                const int steps = k - w_lo + 1;
                for (; k >= w_lo; --k) {
                    const int j = RECOMPUTE ? (int)s_tape[wid][k - k_lo][lane] : (int)((tw >> shift) & tmask);
                    shift -= p.tape_bits;
                    uint32_t wn[Blocks<NET>::W];
                    words<NET>((uint32_t)(k - 1), tid, pe, p.seed_lo, p.seed_hi, wn);
                    float en[M + 1];
#pragma unroll
                    for (int q = 0; q <= M; ++q) en[q] = neglog_u(wn[q]);
                    sweep(k, j, ed);
#pragma unroll
                    for (int q = 0; q <= M; ++q) ed[q] = en[q];
                }
                fold(steps);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) dth[j] += (double)dth32[j];
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < M; ++q) p.partials[nd.part_off + q * B + i] = dth[q];
}

template <class NET, bool GRID, bool SH = false>
__device__ void backward(const RunParams &p)
{
    __shared__ uint8_t s_tape[kWaves][kRecSteps][64];
    const float invT = 1.0f / run_temperature(p);
    if (p.recompute) {
        if (invT == 2.0f) backward_run<NET, 2, true, GRID, SH>(p, s_tape);
        else if (invT == 1.0f) backward_run<NET, 1, true, GRID, SH>(p, s_tape);
        else backward_run<NET, 0, true, GRID, SH>(p, s_tape);
    } else {
        if (invT == 2.0f) backward_run<NET, 2, false, GRID, SH>(p, s_tape);
        else if (invT == 1.0f) backward_run<NET, 1, false, GRID, SH>(p, s_tape);
        else backward_run<NET, 0, false, GRID, SH>(p, s_tape);
    }
}

}  // namespace spec
}  // namespace ssa
