// Lane-mode kernels: one trajectory per lane, for networks with few species
// and channels.  The state X lives in vector registers (indexed with
// wave-uniform species numbers), the channel descriptors are wave-uniform and
// come through the scalar cache, and the packed change vectors sit in LDS
// because the fired channel differs from lane to lane.
//
// Forward (Sec. 2; Gumbel-max selection of Sec. 3.2): per step
//   a_j = k_j h_j(X), a0 = sum a_j, tau = E_0/a0, j* = argmin_j E_j/a_j
// with E_w = -ln u_w from the Philox stream, which picks the same channel as
// argmax_j [ln a_j + G_j], G_j = -ln E_j.  The clock t is accumulated in FP64
// and so are the exact bin integrals of the observed species (Sec. 4.4).
//
// Backward (Sec. 3.1, Eqs. 3-7, Fig. 1): reverse sweep of every checkpoint
// segment.  The fired channels come from the forward's compact tape or from
// re-running the segment; the noise, propensities and waiting times are
// regenerated from the Philox counters, so nothing else per step is stored.
#include "ssa_device.hpp"
#include "ssa_lane.hpp"

#include <math.h>

namespace ssa {

namespace {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kObsMax = 4;

__device__ __forceinline__ double bin_edge(double t_obs, int b, int n_bins)
{
    return t_obs * (double)b / (double)n_bins;
}

__device__ void log_tie(const RunParams &p, uint32_t g, int k, int chosen, int second, float margin,
                        int kind)
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

// Everything a wave needs about its network, read once.
template <int NMAX, int MMAX>
struct WaveNet {
    int N, M, nob;
    float c[MMAX];       // k_j * mult_j, k_j = exp(theta)
    int osp[kObsMax];    // observed species (NMAX = unused)
    const ReactDesc *rd;
};

template <int NMAX, int MMAX>
__device__ __forceinline__ void load_wave_net(const RunParams &p, const NetDev &nd, WaveNet<NMAX, MMAX> &w)
{
    w.N = nd.N;
    w.M = nd.M;
    w.nob = nd.n_obs;
    w.rd = p.rd + nd.react_off;
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        float c = 0.f;
        if (j < nd.M) {
            const ReactDesc r = w.rd[j];
            c = expf(p.theta[nd.param_off + r.rate]) * r.mult;
        }
        w.c[j] = c;
    }
#pragma unroll
    for (int o = 0; o < kObsMax; ++o)
        w.osp[o] = o < nd.n_obs ? uniform_i(p.obs_sp[nd.obs_sp_off + o]) : NMAX;
}

template <int NMAX>
__device__ __forceinline__ int slot(int s)
{
    return s == kNoSpecies ? NMAX : s;
}

// Wave-uniform fields of channel j, read as whole dwords (scalar loads).
struct Chan {
    int s1, s2, homodimer;
};

template <int NMAX>
__device__ __forceinline__ Chan chan(const ReactDesc *rd, int j)
{
    const uint32_t w0 = (uint32_t)uniform_i(*reinterpret_cast<const int32_t *>(rd + j));
    Chan c;
    c.s1 = slot<NMAX>((int)(w0 & 0xFFu));
    c.s2 = slot<NMAX>((int)((w0 >> 8) & 0xFFu));
    c.homodimer = (int)((w0 >> 16) & 0xFFu);
    return c;
}

__device__ __forceinline__ int chan_csr(const ReactDesc *rd, int j)
{
    return uniform_i(rd[j].csr);
}

// a_j = (c_j X[s1]) (X[s2] - homodimer); returns a0.  A1 = c_j X[s1] and
// A2 = c_j (X[s2] - homodimer) are the partial derivatives da_j/dX[s2] and
// da_j/dX[s1].
template <int NMAX, int MMAX, bool DERIV>
__device__ __forceinline__ float propensities(const WaveNet<NMAX, MMAX> &w, const int (&X)[NMAX + 1],
                                              float (&a)[MMAX], float (&A1)[MMAX], float (&A2)[MMAX])
{
    float a0 = 0.f;
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        float aj = 0.f;
        if (j < w.M) {
            const Chan r = chan<NMAX>(w.rd, j);
            const float x1 = (float)X[r.s1];
            const float x2 = (float)(X[r.s2] - r.homodimer);
            const float u1 = w.c[j] * x1;
            aj = u1 * x2;
            if (DERIV) {
                A1[j] = u1;
                A2[j] = w.c[j] * x2;
            }
        } else if (DERIV) {
            A1[j] = 0.f;
            A2[j] = 0.f;
        }
        a[j] = aj;
        a0 += aj;
    }
    return a0;
}

// Philox words of step k: word 0 for tau, word 1+j for channel j.
template <int MMAX>
__device__ __forceinline__ void step_words(int M, uint32_t k, uint32_t tid, uint32_t pe, uint32_t k0,
                                           uint32_t k1, uint32_t (&wd)[4 * ((MMAX + 4) / 4)])
{
    constexpr int NB = (MMAX + 4) / 4;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        Philox::Out o{0u, 0u, 0u, 0u};
        if (4 * b < M + 1) o = Philox::block((uint32_t)b, k, tid, pe, k0, k1);
        wd[4 * b] = o.x;
        wd[4 * b + 1] = o.y;
        wd[4 * b + 2] = o.z;
        wd[4 * b + 3] = o.w;
    }
}

// Exponential race: the smallest and second smallest r_j = E_j / a_j.
template <int MMAX>
__device__ __forceinline__ int race(int M, const float (&a)[MMAX], const uint32_t (&wd)[4 * ((MMAX + 4) / 4)],
                                    float (&r)[MMAX], float &r1, float &r2)
{
    int j1 = 0;
    r1 = INFINITY;
    r2 = INFINITY;
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        float rj = INFINITY;
        if (j < M && a[j] > 0.f) rj = neglog_u(wd[1 + j]) * fast_rcp(a[j]);
        r[j] = rj;
        const bool lt = rj < r1;
        r2 = lt ? r1 : fminf(r2, rj);
        j1 = lt ? j : j1;
        r1 = fminf(r1, rj);
    }
    return j1;
}

template <int MMAX>
__device__ __forceinline__ int second_index(int M, const float (&r)[MMAX], int j1)
{
    int j2 = -1;
    float best = INFINITY;
#pragma unroll
    for (int j = 0; j < MMAX; ++j)
        if (j < M && j != j1 && r[j] < best) { best = r[j]; j2 = j; }
    return j2;
}

// X += sign * v_j for the packed change vector of channel j (LDS).
template <int NMAX>
__device__ __forceinline__ void apply_change(int (&X)[NMAX + 1], const uint32_t *rows, int j, int sign)
{
    constexpr int WPR = (NMAX + 7) / 8;
#pragma unroll
    for (int q = 0; q < WPR; ++q) {
        const uint32_t word = rows[j * WPR + q];
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (8 * q + s < NMAX) X[8 * q + s] += sign * nibble(word, s);
    }
}

struct Bins {
    int bin;
    double hi;       // upper edge of the current bin
};

// Adds the interval [t0, t1) of a path at values xo into the bin integrals,
// writing every bin it completes.  close = true completes all bins up to t_obs.
template <int NMAX>
__device__ void bins_add(double t0, double t1, const double (&xo)[kObsMax], int nob, Bins &bs,
                         double (&acc)[kObsMax], double *obs_lane, int64_t B, int n_bins, double t_obs,
                         bool close)
{
    if (bs.bin >= n_bins) return;
    if (!close && t1 <= bs.hi) {
#pragma unroll
        for (int o = 0; o < kObsMax; ++o) acc[o] += xo[o] * (t1 - t0);
        return;
    }
    const double inv_dt = (double)n_bins / t_obs;
    while (bs.bin < n_bins) {
        const double hi = bs.hi;
        if (!close && t1 <= hi) {
#pragma unroll
            for (int o = 0; o < kObsMax; ++o) acc[o] += xo[o] * (t1 - t0);
            return;
        }
        const double seg = fmax(hi - t0, 0.0);
#pragma unroll
        for (int o = 0; o < kObsMax; ++o) {
            acc[o] += xo[o] * seg;
            if (o < nob) obs_lane[((int64_t)bs.bin * nob + o) * B] = acc[o] * inv_dt;
            acc[o] = 0.0;
        }
        t0 = fmax(t0, hi);
        bs.bin += 1;
        bs.hi = bs.bin < n_bins ? bin_edge(t_obs, bs.bin + 1, n_bins) : INFINITY;
    }
}

template <int NMAX>
__device__ __forceinline__ void observe(const int (&X)[NMAX + 1], const int (&osp)[kObsMax],
                                        double (&xo)[kObsMax])
{
#pragma unroll
    for (int o = 0; o < kObsMax; ++o) xo[o] = (double)X[osp[o]];
}

}  // namespace

// --------------------------------------------------------------------------
// Forward
// --------------------------------------------------------------------------
template <int NMAX, int MMAX>
__global__ __launch_bounds__(kBlock) void fwd_lane_kernel(RunParams p)
{
    constexpr int WPR = (NMAX + 7) / 8;
    constexpr int NB = (MMAX + 4) / 4;
    __shared__ uint32_t s_rows[kWaves][MMAX * WPR];

    const int wid = uniform_i((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int item_idx = blockIdx.x * kWaves + wid;
    const bool have = item_idx < p.n_items;
    const LaneItem it = p.items[have ? item_idx : 0];
    const NetDev nd = p.nets[it.net];
    if (have)
        for (int q = lane; q < nd.M * WPR; q += 64) s_rows[wid][q] = p.rows[nd.rows_off + q];
    __syncthreads();
    if (!have) return;
    const uint32_t *rows = s_rows[wid];

    WaveNet<NMAX, MMAX> w;
    load_wave_net(p, nd, w);

    const bool valid = lane < it.count;
    const int64_t B = nd.B;
    const int64_t i = it.first + (valid ? lane : 0);
    const int64_t g = nd.traj_off + i;
    const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);

    int X[NMAX + 1];
#pragma unroll
    for (int s = 0; s < NMAX; ++s) X[s] = (s < w.N) ? p.x0[nd.state_off + s * B + i] : 0;
    X[NMAX] = 1;

    const bool bins = p.obs_kind == 1 && w.nob > 0;
    const int n_bins = p.n_bins;
    const double t_obs = nd.t_obs;
    Bins bs{0, bins ? bin_edge(t_obs, 1, n_bins) : INFINITY};
    if (!bins) bs.bin = n_bins;
    // bin-edge log: an event time outside (e_lo, e_hi), the current bin
    // narrowed by kEdgeLog at both edges, is compared with the edges
    const bool edge_log = bins && p.ties != nullptr;
    double e_lo = -INFINITY, e_hi = edge_log ? bs.hi * (1.0 - kEdgeLog) : INFINITY;
    double acc[kObsMax] = {0.0, 0.0, 0.0, 0.0};
    double *obs_lane = p.obs + nd.obsb_off * (p.obs_kind == 1 ? n_bins : 1) + i;

    const int spw = p.tape_bits ? 32 / p.tape_bits : 0;
    const int tshift = spw ? __builtin_ctz(spw) : 0;
    uint32_t tword = 0u;
    const bool has_t_end = p.t_end < INFINITY;

    double t = 0.0;
    bool active = valid;
    int n_done = 0;
    uint32_t flags = 0u;

    int ck_left = 0;         // steps until the next checkpoint
    int64_t ck_idx = 0;
    for (int k = 0; k < p.n_steps; ++k) {
        if (ballot(active) == 0ull) break;
        if (!active) continue;
        if (p.ck_x) {
            if (ck_left == 0) {
#pragma unroll
                for (int s = 0; s < NMAX; ++s)
                    if (s < w.N) p.ck_x[ck_idx * p.state_total + nd.state_off + s * B + i] = X[s];
                p.ck_t[ck_idx * p.traj_total + g] = t;
                ck_idx += 1;
                ck_left = p.K;
            }
            ck_left -= 1;
        }
        float a[MMAX], A1[MMAX], A2[MMAX];
        const float a0 = propensities<NMAX, MMAX, false>(w, X, a, A1, A2);
        if (!(a0 > 0.f)) {                       // absorbing state (or a non-finite rate)
            if (!(a0 == 0.f)) flags |= kFlagNonFinite;
            active = false;
            continue;
        }
        uint32_t wd[4 * NB];
        step_words<MMAX>(w.M, (uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, wd);
        const float tau = neglog_u(wd[0]) * fast_rcp(a0);
        const double tn = t + (double)tau;
        if (has_t_end) {
            const bool fire = tn <= p.t_end;
            if (fabs(tn - p.t_end) <= kClockTieLog * p.t_end)
                log_tie(p, (uint32_t)g, k, fire ? 1 : 0, 0, (float)((tn - p.t_end) / p.t_end), 1);
            if (!fire) {
                active = false;
                continue;
            }
        }
        float r[MMAX], r1, r2;
        const int j = race<MMAX>(w.M, a, wd, r, r1, r2);
        if (r2 <= r1 * (1.f + kTieLog))
            log_tie(p, (uint32_t)g, k, j, second_index<MMAX>(w.M, r, j), (r2 - r1) / r1, 0);
        if (bs.bin < n_bins) {
            double xo[kObsMax];
            observe<NMAX>(X, w.osp, xo);
            bins_add<NMAX>(t, tn, xo, w.nob, bs, acc, obs_lane, B, n_bins, t_obs, false);
        }
        if (edge_log && (tn >= e_hi || tn <= e_lo)) {
            // the edges around the bin holding t + tau (edge b is at t_obs b / n_bins)
            const int bl = bs.bin < n_bins ? bs.bin : n_bins;
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
        if (spw) {
            const int pos = k & (spw - 1);
            tword |= (uint32_t)j << (p.tape_bits * pos);
            if (pos == spw - 1) {
                p.tape[(int64_t)(k >> tshift) * p.traj_total + g] = tword;
                tword = 0u;
            }
        }
        apply_change<NMAX>(X, rows, j, +1);
        t = tn;
        n_done = k + 1;
    }
    if (!valid) return;
    if (spw && (n_done & (spw - 1)) != 0) p.tape[(int64_t)(n_done >> tshift) * p.traj_total + g] = tword;
    if (bs.bin < n_bins) {
        double xo[kObsMax];
        observe<NMAX>(X, w.osp, xo);
        bins_add<NMAX>(t, t_obs, xo, w.nob, bs, acc, obs_lane, B, n_bins, t_obs, true);
    }
    if (p.obs_kind == 0) {
#pragma unroll
        for (int o = 0; o < kObsMax; ++o)
            if (o < w.nob) obs_lane[(int64_t)o * B] = (double)X[w.osp[o]];
    }
#pragma unroll
    for (int s = 0; s < NMAX; ++s) {
        if (s < w.N) {
            p.x_final[nd.state_off + s * B + i] = X[s];
            if (X[s] < 0) flags |= kFlagOverflow;
        }
    }
    p.t_final[g] = t;
    p.steps_done[g] = n_done;
    if (flags) atomicOr(p.flags, flags);
}

// --------------------------------------------------------------------------
// Backward
// --------------------------------------------------------------------------

// Reverse-time bin tracker: the bin holding the current (later) time t, its
// lower edge and the cached d_obs values of that bin.
struct RevBins {
    int bin;         // n_bins when t >= t_obs
    double lo;
    double dob[kObsMax];
};

__device__ __forceinline__ void rev_load(RevBins &rb, const double *dobs_lane, int nob, int64_t B)
{
#pragma unroll
    for (int o = 0; o < kObsMax; ++o)
        rb.dob[o] = (o < nob) ? dobs_lane[((int64_t)rb.bin * nob + o) * B] : 0.0;
}

template <int NMAX, int MMAX>
__global__ __launch_bounds__(kBlock) void bwd_lane_kernel(RunParams p)
{
    constexpr int WPR = (NMAX + 7) / 8;
    constexpr int NB = (MMAX + 4) / 4;
    constexpr int KMAX_REC = 64;           // recompute mode: steps per segment kept in LDS
    __shared__ uint32_t s_rows[kWaves][MMAX * WPR];
    __shared__ uint8_t s_tape[kWaves][KMAX_REC][64];

    const int wid = uniform_i((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int item_idx = blockIdx.x * kWaves + wid;
    const bool have = item_idx < p.n_items;
    const LaneItem it = p.items[have ? item_idx : 0];
    const NetDev nd = p.nets[it.net];
    if (have)
        for (int q = lane; q < nd.M * WPR; q += 64) s_rows[wid][q] = p.rows[nd.rows_off + q];
    __syncthreads();
    if (!have) return;
    const uint32_t *rows = s_rows[wid];

    WaveNet<NMAX, MMAX> w;
    load_wave_net(p, nd, w);

    const bool valid = lane < it.count;
    const int64_t B = nd.B;
    const int64_t i = it.first + (valid ? lane : 0);
    const int64_t g = nd.traj_off + i;
    const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);
    const float invT = 1.0f / run_temperature(p);
    const bool invT_is_2 = invT == 2.0f, invT_is_1 = invT == 1.0f;

    const int n = valid ? p.steps_done[g] : 0;
    // wave-uniform number of steps to sweep
    int kmax = n;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) kmax = max(kmax, __shfl_xor(kmax, off));
    kmax = uniform_i(kmax);

    // state at the end of the path
    int X[NMAX + 1];
#pragma unroll
    for (int s = 0; s < NMAX; ++s) X[s] = (s < w.N && valid) ? p.x_final[nd.state_off + s * B + i] : 0;
    X[NMAX] = 1;
    double t = valid ? p.t_final[g] : 0.0;

    const bool bins = p.obs_kind == 1 && w.nob > 0;
    const int n_bins = p.n_bins;
    const double t_obs = nd.t_obs;
    const double inv_dt = bins ? (double)n_bins / t_obs : 0.0;
    const double *dobs_lane = p.d_obs + nd.obsb_off * (p.obs_kind == 1 ? n_bins : 1) + i;

    // adjoint of the state: FP64 base plus an FP32 per-segment increment
    double lam[NMAX + 1];
    float dlam[NMAX + 1];
#pragma unroll
    for (int s = 0; s <= NMAX; ++s) { lam[s] = 0.0; dlam[s] = 0.f; }
    double lam_t = 0.0;
    double dth[MMAX];
    float dth_seg[MMAX];
#pragma unroll
    for (int j = 0; j < MMAX; ++j) { dth[j] = 0.0; dth_seg[j] = 0.f; }

    RevBins rb;
    rb.bin = n_bins;
    rb.lo = t_obs;
#pragma unroll
    for (int o = 0; o < kObsMax; ++o) rb.dob[o] = 0.0;
    if (valid) {
        if (bins) {
            // direct dependence on the final state: the hold [t_n, t_obs)
            double hi = t_obs;
            while (rb.bin > 0 && t < rb.lo) {
                rb.bin -= 1;
                rb.lo = bin_edge(t_obs, rb.bin, n_bins);
                rev_load(rb, dobs_lane, w.nob, B);
                const double seg = hi - fmax(t, rb.lo);
#pragma unroll
                for (int o = 0; o < kObsMax; ++o)
                    if (o < w.nob) lam[w.osp[o]] += rb.dob[o] * seg * inv_dt;
                hi = rb.lo;
            }
        } else if (p.obs_kind == 0) {
#pragma unroll
            for (int o = 0; o < kObsMax; ++o)
                if (o < w.nob) lam[w.osp[o]] += dobs_lane[(int64_t)o * B];
        }
    }

    const int spw = p.tape_bits ? 32 / p.tape_bits : 1;
    const int tshift = __builtin_ctz(spw);
    const uint32_t tmask = p.tape_bits ? ((1u << p.tape_bits) - 1u) : 0u;
    const int n_seg = (kmax + p.K - 1) / p.K;
    uint32_t flags = 0u;

    for (int c = n_seg - 1; c >= 0; --c) {
        const int k_lo = c * p.K;
        const int k_hi = min(k_lo + p.K, kmax);
        if (p.recompute) {
            // re-run the segment from its checkpoint to recover the fired channels
            int Xr[NMAX + 1];
            if (k_lo < n) {
#pragma unroll
                for (int s = 0; s < NMAX; ++s)
                    Xr[s] = (s < w.N) ? p.ck_x[(int64_t)c * p.state_total + nd.state_off + s * B + i] : 0;
            } else {
#pragma unroll
                for (int s = 0; s < NMAX; ++s) Xr[s] = X[s];
            }
            Xr[NMAX] = 1;
            for (int k = k_lo; k < k_hi; ++k) {
                if (k >= n) continue;
                float a[MMAX], A1[MMAX], A2[MMAX];
                const float a0 = propensities<NMAX, MMAX, false>(w, Xr, a, A1, A2);
                (void)a0;
                uint32_t wd[4 * NB];
                step_words<MMAX>(w.M, (uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, wd);
                float r[MMAX], r1, r2;
                const int j = race<MMAX>(w.M, a, wd, r, r1, r2);
                s_tape[wid][k - k_lo][lane] = (uint8_t)j;
                apply_change<NMAX>(Xr, rows, j, +1);
            }
        }
        // resynchronise with the checkpoint that ends this segment
        if (k_hi < n && p.ck_x) {
            const int64_t c1 = c + 1;
#pragma unroll
            for (int s = 0; s < NMAX; ++s)
                if (s < w.N) X[s] = p.ck_x[c1 * p.state_total + nd.state_off + s * B + i];
            t = p.ck_t[c1 * p.traj_total + g];
        }
        uint32_t tword = 0u;
        int tword_idx = -1;
        for (int k = k_hi - 1; k >= k_lo; --k) {
            if (k >= n) continue;
            int j;
            if (p.recompute) {
                j = s_tape[wid][k - k_lo][lane];
            } else {
                const int widx = k >> tshift;
                if (widx != tword_idx) {
                    tword = p.tape[(int64_t)widx * p.traj_total + g];
                    tword_idx = widx;
                }
                j = (int)((tword >> (p.tape_bits * (k & (spw - 1)))) & tmask);
            }
            // X_{k+1} -> X_k
            int Xp[NMAX + 1];
#pragma unroll
            for (int s = 0; s <= NMAX; ++s) Xp[s] = X[s];
            apply_change<NMAX>(X, rows, j, -1);

            float a[MMAX], A1[MMAX], A2[MMAX];
            const float a0 = propensities<NMAX, MMAX, true>(w, X, a, A1, A2);
            uint32_t wd[4 * NB];
            step_words<MMAX>(w.M, (uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, wd);
            const float E0 = neglog_u(wd[0]);
            const float rcp_a0 = fast_rcp(a0);
            const float tau = E0 * rcp_a0;
            const double t_k = t - (double)tau;

            // direct dL/dt_{k+1}: t_{k+1} closes the interval at X_k and opens the one at X_{k+1}
            if (bins && rb.bin < n_bins) {
#pragma unroll
                for (int o = 0; o < kObsMax; ++o)
                    if (o < w.nob) lam_t += rb.dob[o] * (double)(X[w.osp[o]] - Xp[w.osp[o]]) * inv_dt;
            }

            // soft sample y~ of Eq. (3) in ratio form: y~_j ~ (r_min / r_j)^(1/T)
            float r[MMAX], ra[MMAX];
            float rmin = INFINITY;
            int jmin = 0;
#pragma unroll
            for (int q = 0; q < MMAX; ++q) {
                float rq = INFINITY, raq = 0.f;
                if (q < w.M && a[q] > 0.f) {
                    raq = fast_rcp(a[q]);
                    rq = neglog_u(wd[1 + q]) * raq;
                }
                r[q] = rq;
                ra[q] = raq;
                jmin = rq < rmin ? q : jmin;
                rmin = fminf(rmin, rq);
            }
            float y[MMAX];
            float ysum = 0.f;
#pragma unroll
            for (int q = 0; q < MMAX; ++q) {
                // r[q] = inf for inactive channels gives rho = 0
                y[q] = rmin * fast_rcp(r[q]);
            }
            if (invT_is_2) {
#pragma unroll
                for (int q = 0; q < MMAX; ++q) y[q] = y[q] * y[q];
            } else if (!invT_is_1) {
#pragma unroll
                for (int q = 0; q < MMAX; ++q) y[q] = y[q] > 0.f ? exp2f(log2f(y[q]) * invT) : 0.f;
            }
#pragma unroll
            for (int q = 0; q < MMAX; ++q) ysum += y[q];
            const float rys = fast_rcp(ysum);
            // w_q = v_q . lambda(k+1), shifted by w_jmin to keep y~(w - wbar) accurate
            float wv[MMAX];
#pragma unroll
            for (int q = 0; q < MMAX; ++q) {
                float s = 0.f;
                if (q < w.M) {
                    const int csr = chan_csr(w.rd, q);
                    const int beg = csr & 0xFFFFFF, cnt = (int)((uint32_t)csr >> 24);
                    for (int e = 0; e < cnt; ++e) {
                        const int32_t ent = uniform_i(p.csr[beg + e]);
                        const int sp = csr_species(ent);
                        s += (float)csr_delta(ent) * ((float)lam[sp] + dlam[sp]);
                    }
                }
                wv[q] = s;
            }
            float wref = 0.f;
#pragma unroll
            for (int q = 0; q < MMAX; ++q) wref = (q == jmin) ? wv[q] : wref;
            float wbar = 0.f;
#pragma unroll
            for (int q = 0; q < MMAX; ++q) {
                y[q] *= rys;
                wbar += y[q] * (wv[q] - wref);
            }
            // waiting-time path: d tau = -(tau / a0) d a0
            const float cc = (float)(lam_t * (double)(-tau * rcp_a0));
#pragma unroll
            for (int q = 0; q < MMAX; ++q) {
                if (q < w.M) {
                    const float gq = y[q] * ((wv[q] - wref) - wbar) * invT;   // dL/d ln a_q (soft path)
                    dth_seg[q] += gq + cc * a[q];
                    const float coef = gq * ra[q] + cc;                       // multiplies d a_q / dX
                    const Chan rd = chan<NMAX>(w.rd, q);
                    dlam[rd.s1] += coef * A2[q];
                    dlam[rd.s2] += coef * A1[q];
                }
            }
            // direct dL/dX_k from the interval [t_k, t_{k+1})
            if (bins) {
                double hi = fmin(t, t_obs);
                while (t_k < rb.lo && rb.bin > 0) {
                    if (rb.bin < n_bins) {
                        const double seg = fmax(hi - rb.lo, 0.0);
#pragma unroll
                        for (int o = 0; o < kObsMax; ++o)
                            if (o < w.nob) lam[w.osp[o]] += rb.dob[o] * seg * inv_dt;
                    }
                    hi = fmin(hi, rb.lo);
                    rb.bin -= 1;
                    rb.lo = bin_edge(t_obs, rb.bin, n_bins);
                    rev_load(rb, dobs_lane, w.nob, B);
                }
                if (rb.bin < n_bins) {
                    const double seg = fmax(hi - t_k, 0.0);
#pragma unroll
                    for (int o = 0; o < kObsMax; ++o)
                        if (o < w.nob) lam[w.osp[o]] += rb.dob[o] * seg * inv_dt;
                }
            }
            if (!(a0 > 0.f) || !(tau >= 0.f)) flags |= kFlagNonFinite;
            t = t_k;
        }
        // fold the segment's FP32 increments into the FP64 accumulators
#pragma unroll
        for (int s = 0; s <= NMAX; ++s) { lam[s] += (double)dlam[s]; dlam[s] = 0.f; }
#pragma unroll
        for (int q = 0; q < MMAX; ++q) { dth[q] += (double)dth_seg[q]; dth_seg[q] = 0.f; }
    }
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < MMAX; ++q)
        if (q < w.M) p.partials[nd.part_off + q * B + i] = dth[q];
    if (flags) atomicOr(p.flags, flags);
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
template <int NMAX, int MMAX>
static hipError_t launch_lane(const RunParams &p, bool backward, hipStream_t stream)
{
    const int blocks = (p.n_items + kWaves - 1) / kWaves;
    if (blocks == 0) return hipSuccess;
    if (backward)
        hipLaunchKernelGGL((bwd_lane_kernel<NMAX, MMAX>), dim3(blocks), dim3(kBlock), 0, stream, p);
    else
        hipLaunchKernelGGL((fwd_lane_kernel<NMAX, MMAX>), dim3(blocks), dim3(kBlock), 0, stream, p);
    return hipGetLastError();
}

hipError_t lane_launch(int lane_class, const RunParams &p, bool backward, hipStream_t stream)
{
    switch (lane_class) {
    case kLane_N4_M4: return launch_lane<4, 4>(p, backward, stream);
    case kLane_N8_M8: return launch_lane<8, 8>(p, backward, stream);
    case kLane_N8_M16: return launch_lane<8, 16>(p, backward, stream);
    case kLane_N16_M16: return launch_lane<16, 16>(p, backward, stream);
    case kLane_N16_M32: return launch_lane<16, 32>(p, backward, stream);
    default: return hipErrorInvalidValue;
    }
}

int lane_class_for(int N, int M)
{
    if (N <= 4 && M <= 4) return kLane_N4_M4;
    if (N <= 8 && M <= 8) return kLane_N8_M8;
    if (N <= 8 && M <= 16) return kLane_N8_M16;
    if (N <= 16 && M <= 16) return kLane_N16_M16;
    if (N <= 16 && M <= 32) return kLane_N16_M32;
    return -1;
}

int lane_class_nmax(int cls)
{
    switch (cls) {
    case kLane_N4_M4: return 4;
    case kLane_N8_M8: case kLane_N8_M16: return 8;
    default: return 16;
    }
}

}  // namespace ssa
