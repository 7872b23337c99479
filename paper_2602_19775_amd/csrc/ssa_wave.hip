// Wave-mode kernels: one trajectory per group of L lanes (L = 8, 16, 32 or
// 64; 64/L trajectories per wavefront), for networks with many channels.
// Lane l of a group owns the Philox blocks b = l, l + L, ... of every step,
// i.e. the words 4b..4b+3 and the channels 4b-1..4b+2, so no block is
// generated twice.  The state X of each trajectory sits in LDS; a0 and the
// race (smallest and second smallest E_j/a_j) are reduced across the group
// with cross-lane shuffles.  One persistent launch serves every network of a
// batch: waves pull trajectories from a work counter in cost order.
//
// Forward (Sec. 2, Sec. 3.2) and backward (Sec. 3.1, Eqs. 3-7, Fig. 1) follow
// the lane-mode kernels step for step; the backward's state-adjoint updates
// are gathered per species through incidence lists, so every sum has a fixed
// order and the gradients are bit-reproducible.
#include "ssa_device.hpp"
#include "ssa_wave.hpp"

#include <math.h>

namespace ssa {
namespace wave {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kMaxN = 64;
constexpr int kOne = kMaxN;   // LDS state slot holding the constant 1 (a missing reactant)
constexpr int kObsMax = 4;
constexpr int kFold = 32;

__device__ __forceinline__ double bin_edge(double t_obs, int b, int n_bins)
{
    return t_obs * (double)b / (double)n_bins;
}

// Checkpoints and the choice tape are kept trajectory-major in this mode: a
// group works on one trajectory at a time, so its successive tape words and
// its checkpointed counts share cache lines instead of each touching a line of
// its own.
__device__ __forceinline__ int64_t tape_at(const RunParams &p, int64_t g, int64_t w)
{
    return g * p.tape_words + w;
}

__device__ __forceinline__ int64_t ckx_at(const RunParams &p, const NetDev &nd, int64_t c, int64_t i, int s)
{
    return c * p.state_total + nd.state_off + i * nd.N + s;
}

__device__ __forceinline__ int64_t ckt_at(const RunParams &p, int64_t g, int64_t c)
{
    return g * p.n_ckpt + c;
}

// LDS writes of one lane become visible to the other lanes of its wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int L>
__device__ __forceinline__ float gsum(float v)
{
    return group_sum<L>(v);
}

// (r1, j1, r2) = smallest ratio, its channel (lowest index on exact ties) and
// the second smallest ratio over the group.
template <int L>
__device__ __forceinline__ void grace(float &r1, int &j1, float &r2)
{
    group_race<L>(r1, j1, r2);
}

__device__ void log_tie(const RunParams &p, uint32_t g, int k, int chosen, int second, float margin, int kind)
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

// The channels a lane owns, read once per network.  For the backward also
// the first kVecSlots change-vector entries of each, two per word as
// species | delta << 8 in 16 bits (zero-padded), and its two incidence slots
// as pos1 | pos2 << 16.
template <int L, int BPL>
struct LaneChannels {
    static constexpr int C = 4 * BPL;
    int s1[C], s2[C], homo[C], csr[C], j[C];
    float c[C];
    bool on[C];
    uint32_t ve[C][kVecSlots / 2];
    uint32_t pos[C];
    static constexpr uint32_t kSink = 8 * BPL * L;   // incidence slot that nothing reads

    __device__ void load(const RunParams &p, const NetDev &nd, int gl)
    {
        const ReactDesc *rd = p.rd + nd.react_off;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int b = gl + L * (q >> 2);
            const int w = 4 * b + (q & 3);
            const int jj = w - 1;
            j[q] = jj;
            on[q] = jj >= 0 && jj < nd.M;
            s1[q] = s2[q] = kOne;
            homo[q] = 0;
            csr[q] = 0;
            c[q] = 0.f;
            pos[q] = kSink | (kSink << 16);
#pragma unroll
            for (int e = 0; e < kVecSlots / 2; ++e) ve[q][e] = 0u;
            if (on[q]) {
                const ReactDesc r = rd[jj];
                s1[q] = r.s1 == kNoSpecies ? kOne : r.s1;
                s2[q] = r.s2 == kNoSpecies ? kOne : r.s2;
                homo[q] = r.homodimer;
                csr[q] = r.csr;
                c[q] = expf(p.theta[nd.param_off + r.rate]) * r.mult;
                const int beg = r.csr & 0xFFFFFF, cnt = (int)((uint32_t)r.csr >> 24);
#pragma unroll
                for (int e = 0; e < kVecSlots; ++e) {
                    const int32_t ent = e < cnt ? p.csr[beg + e] : 0;
                    const uint32_t h = ((uint32_t)csr_species(ent) & 0xFFu) | (((uint32_t)csr_delta(ent) & 0xFFu) << 8);
                    ve[q][e >> 1] |= h << (16 * (e & 1));
                }
                const uint32_t pi = (uint32_t)p.chan_inc[nd.react_off + jj];
                const uint32_t p1 = pi & 0xFFFFu, p2 = pi >> 16;
                pos[q] = (p1 == 0xFFFFu ? kSink : p1) | ((p2 == 0xFFFFu ? kSink : p2) << 16);
            }
        }
    }
};

// A network's tables staged in the group's LDS slot:
//   desc[tab_m]        channel j: first entry (relative) | entry count << 24
//   ent[tab_nnz]       change-vector entries, species | delta << 16
//   inc_ptr[kMaxN+1]   species -> range of its incidence slots
struct GroupTab {
    int32_t *desc, *ent, *inc_ptr;

    __device__ GroupTab(int32_t *base, const RunParams &p)
    {
        desc = base;
        ent = desc + p.tab_m;
        inc_ptr = ent + p.tab_nnz;
    }

    __device__ void load(const RunParams &p, const NetDev &nd, int gl, int L)
    {
        const ReactDesc *rd = p.rd + nd.react_off;
        const int base_e = rd[0].csr & 0xFFFFFF;
        const int last = rd[nd.M - 1].csr;
        const int n_ent = (last & 0xFFFFFF) + (int)((uint32_t)last >> 24) - base_e;
        for (int q = gl; q < nd.M; q += L) {
            const int c = rd[q].csr;
            desc[q] = ((c & 0xFFFFFF) - base_e) | (c & (int)0xFF000000);
        }
        for (int e = gl; e < n_ent; e += L) ent[e] = p.csr[base_e + e];
        const int *ip = p.inc_ptr + nd.inc_off;
        for (int s = gl; s <= nd.N; s += L) inc_ptr[s] = ip[s];
    }
};

// Count of species s; a channel's missing reactant reads slot kOne, which
// holds 1 for the whole item.
__device__ __forceinline__ int xval(const int *sx, int s)
{
    return sx[s];
}

template <int L, int BPL>
__device__ __forceinline__ void group_words(int M, int gl, uint32_t k, uint32_t tid, uint32_t pe, uint32_t k0,
                                            uint32_t k1, uint32_t (&wd)[4 * BPL])
{
#pragma unroll
    for (int bb = 0; bb < BPL; ++bb) {
        const int b = gl + L * bb;
        Philox::Out o{0u, 0u, 0u, 0u};
        if (4 * b < M + 1) o = Philox::block((uint32_t)b, k, tid, pe, k0, k1);
        wd[4 * bb] = o.x;
        wd[4 * bb + 1] = o.y;
        wd[4 * bb + 2] = o.z;
        wd[4 * bb + 3] = o.w;
    }
}

// Lane of a group and channel slot that hold channel j: word j + 1 lies in
// Philox block b = (j + 1) / 4, which lane b mod L generates as its slot
// 4 (b / L) + (j + 1) mod 4.
struct Owner {
    int lane;   // lane of the wavefront
    int slot;
};

template <int L, int BPL>
__device__ __forceinline__ Owner owner_of(int j, int grp)
{
    if (L == 64) j = __builtin_amdgcn_readfirstlane(j);   // one trajectory per wave: j is uniform
    const int w = j + 1, b = w >> 2;
    return Owner{grp * L + (b & (L - 1)), 4 * (b / L) + (w & 3)};
}

// v[o.slot] of lane o.lane, for every lane of the group.
template <int L, int C>
__device__ __forceinline__ float from_owner(const float (&v)[C], Owner o)
{
    if (L == 64) {
        // owner and slot are uniform: read every slot of the owner lane into
        // scalars and pick one (a select on the lane's own slots with a
        // uniform index would be lowered to an indexed private array)
        int pick = 0;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int x = __builtin_amdgcn_readlane(__float_as_int(v[q]), o.lane);
            pick = (q == o.slot) ? x : pick;
        }
        return __int_as_float(pick);
    }
    float mine = v[0];
#pragma unroll
    for (int q = 1; q < C; ++q) mine = (q == o.slot) ? v[q] : mine;
    return __shfl(mine, o.lane);
}

// X += sign * v_j through the sparse change vector (lane e applies entry e);
// csr is channel j's descriptor tab.desc[j].
template <int L>
__device__ __forceinline__ void group_apply_desc(const GroupTab &tab, int *sx, int csr, int sign, int gl, bool act)
{
    const int beg = csr & 0xFFFFFF, cnt = (int)((uint32_t)csr >> 24);
    for (int e = gl; e < cnt; e += L) {
        const int32_t ent = tab.ent[beg + e];
        if (act) sx[csr_species(ent)] += sign * csr_delta(ent);
    }
    wave_sync();
}

template <int L>
__device__ __forceinline__ void group_apply(const GroupTab &tab, int *sx, int j, int sign, int gl, bool act)
{
    const int csr = tab.desc[j];
    const int beg = csr & 0xFFFFFF, cnt = (int)((uint32_t)csr >> 24);
    for (int e = gl; e < cnt; e += L) {
        const int32_t ent = tab.ent[beg + e];
        if (act) sx[csr_species(ent)] += sign * csr_delta(ent);
    }
    wave_sync();
}

// --------------------------------------------------------------------------
template <int L, int BPL>
__global__ __launch_bounds__(kBlock) void fwd_kernel(RunParams p)
{
    constexpr int G = 64 / L;                 // trajectories per wavefront
    constexpr int C = 4 * BPL;
    __shared__ int s_x[kWaves][G][kMaxN + 1];   // + the constant-1 slot kOne
    extern __shared__ int32_t s_dyn[];
    const int wid = uniform_i((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane & (L - 1);
    int *sx = s_x[wid][grp];
    GroupTab tab(s_dyn + (wid * G + grp) * p.tab_words, p);
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);
    const bool has_t_end = p.t_end < INFINITY;

    LaneChannels<L, BPL> ch;
    int cached_net = -1;
    for (;;) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(p.work_counter, (uint32_t)G);
        base = (uint32_t)uniform_i((int)__shfl((int)base, 0));
        if (base >= (uint32_t)p.n_items) break;
        const uint32_t item = base + grp;
        const bool have = item < (uint32_t)p.n_items;
        const LaneItem it = p.items[have ? item : 0];
        const NetDev nd = p.nets[it.net];
        if (it.net != cached_net) {
            ch.load(p, nd, gl);
            tab.load(p, nd, gl, L);
            cached_net = it.net;
        }
        const int N = nd.N, M = nd.M;
        const int64_t B = nd.B;
        const int64_t i = it.first;
        const int64_t g = nd.traj_off + i;
        const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
        for (int s = gl; s < N; s += L) sx[s] = have ? p.x0[nd.state_off + s * B + i] : 0;
        if (gl == 0) sx[kOne] = 1;
        wave_sync();
        int osp[kObsMax];
#pragma unroll
        for (int o = 0; o < kObsMax; ++o) osp[o] = o < nd.n_obs ? p.obs_sp[nd.obs_sp_off + o] : kNoSpecies;
        const bool bins = p.obs_kind == 1 && nd.n_obs > 0;
        const int n_bins = p.n_bins;
        const double t_obs = nd.t_obs;
        int bin = bins ? 0 : n_bins;
        double bin_hi = bins ? bin_edge(t_obs, 1, n_bins) : INFINITY;
        // bin-edge log: an event time outside (e_lo, e_hi), the current bin
        // narrowed by kEdgeLog at both edges, is compared with the edges
        const bool edge_log = bins && p.ties != nullptr;
        double e_lo = -INFINITY, e_hi = edge_log ? bin_hi * (1.0 - kEdgeLog) : INFINITY;
        double acc[kObsMax] = {0.0, 0.0, 0.0, 0.0};
        double *obs_lane = p.obs + nd.obsb_off * (p.obs_kind == 1 ? n_bins : 1) + i;
        const double inv_dt = bins ? (double)n_bins / t_obs : 0.0;
        const int spw = p.tape_bits ? 32 / p.tape_bits : 0;
        const int tshift = spw ? __builtin_ctz(spw) : 0;
        uint32_t tword = 0u;
        double t = 0.0;
        bool active = have;
        int n_done = 0;
        uint32_t flags = 0u;
        int ck_left = 0;
        int64_t ck_idx = 0;
        int k = 0;
        for (; k < p.n_steps; ++k) {
            if (ballot(active) == 0ull) break;
            if (p.ck_x) {
                if (ck_left == 0) {
                    if (active) {
                        for (int s = gl; s < N; s += L) p.ck_x[ckx_at(p, nd, ck_idx, i, s)] = sx[s];
                        if (gl == 0) p.ck_t[ckt_at(p, g, ck_idx)] = t;
                    }
                    ck_idx += 1;
                    ck_left = p.K;
                }
                ck_left -= 1;
            }
            // propensities of the lane's channels (every operand index is a
            // valid slot, kOne for a missing reactant or an unused channel
            // slot, so all the reads go out before the first is waited for)
            float a[C];
            float a0 = 0.f;
            int xr1[C], xr2[C];
#pragma unroll
            for (int q = 0; q < C; ++q) {
                xr1[q] = xval(sx, ch.s1[q]);
                xr2[q] = xval(sx, ch.s2[q]);
            }
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const float x1 = (float)xr1[q];
                const float x2 = (float)(xr2[q] - ch.homo[q]);
                a[q] = ch.on[q] ? fabsf((ch.c[q] * x1) * x2) : 0.f;
                a0 += a[q];
            }
            a0 = gsum<L>(a0);
            uint32_t wd[C];
            group_words<L, BPL>(M, gl, (uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, wd);
            float r1 = INFINITY, r2 = INFINITY;
            int j1 = 0x7FFFFFFF;
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const float rq = ch.on[q] ? neglog_u(wd[q]) * fast_rcp(a[q]) : INFINITY;
                const bool lt = rq < r1;
                r2 = lt ? r1 : fminf(r2, rq);
                j1 = lt ? ch.j[q] : j1;
                r1 = fminf(r1, rq);
            }
            grace<L>(r1, j1, r2);
            const float e0 = group_first<L>(neglog_u(wd[0]));
            const float tau = e0 * fast_rcp(a0);
            const double tn = t + (double)tau;
            const bool live = active && a0 > 0.f;
            const bool fire = live && (!has_t_end || tn <= p.t_end);
            if (gl == 0) {
                if (active && !(a0 >= 0.f)) flags |= kFlagNonFinite;
                if (live && has_t_end && fabs(tn - p.t_end) <= kClockTieLog * p.t_end)
                    log_tie(p, (uint32_t)g, k, fire ? 1 : 0, 0, (float)((tn - p.t_end) / p.t_end), 1);
            }
            // second-best channel index for a near-tie record
            if (ballot(fire && r2 <= r1 * (1.f + kTieLog)) != 0ull) {
                const bool nt = fire && r2 <= r1 * (1.f + kTieLog);
                float b2 = INFINITY;
                int j2 = 0x7FFFFFFF;
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    const float rq = ch.on[q] ? neglog_u(wd[q]) * fast_rcp(a[q]) : INFINITY;
                    if (ch.j[q] != j1 && (rq < b2 || (rq == b2 && ch.j[q] < j2))) { b2 = rq; j2 = ch.j[q]; }
                }
                float dummy = INFINITY;
                grace<L>(b2, j2, dummy);
                if (nt && gl == 0) log_tie(p, (uint32_t)g, k, j1, j2, (r2 - r1) / r1, 0);
            }
            if (fire && bin < n_bins) {
                double xo[kObsMax];
#pragma unroll
                for (int o = 0; o < kObsMax; ++o) xo[o] = o < nd.n_obs ? (double)sx[osp[o]] : 0.0;
                double t0 = t;
                while (bin < n_bins) {
                    const double hi = bin_hi;
                    if (tn <= hi) {
#pragma unroll
                        for (int o = 0; o < kObsMax; ++o) acc[o] += xo[o] * (tn - t0);
                        break;
                    }
#pragma unroll
                    for (int o = 0; o < kObsMax; ++o) {
                        acc[o] += xo[o] * fmax(hi - t0, 0.0);
                        if (o < nd.n_obs && gl == 0) obs_lane[((int64_t)bin * nd.n_obs + o) * B] = acc[o] * inv_dt;
                        acc[o] = 0.0;
                    }
                    t0 = fmax(t0, hi);
                    bin += 1;
                    bin_hi = bin < n_bins ? bin_edge(t_obs, bin + 1, n_bins) : INFINITY;
                }
            }
            if (edge_log && fire && (tn >= e_hi || tn <= e_lo)) {
                // the edges around the bin holding t + tau (edge b is at t_obs b / n_bins)
                const int bl = bin < n_bins ? bin : n_bins;
                const double lo = bl >= 1 ? bin_edge(t_obs, bl, n_bins) : -INFINITY;
                const double hi = bl < n_bins ? bin_edge(t_obs, bl + 1, n_bins) : INFINITY;
                int ei = -1;
                double e = 0.0;
                if (bl >= 1 && fabs(tn - lo) <= kEdgeLog * lo) { ei = bl; e = lo; }
                else if (bl < n_bins && fabs(tn - hi) <= kEdgeLog * hi) { ei = bl + 1; e = hi; }
                if (ei >= 1 && gl == 0) log_tie(p, (uint32_t)g, k, tn >= e ? 1 : 0, ei, (float)((tn - e) / e), 2);
                e_lo = bl >= 1 ? lo * (1.0 + kEdgeLog) : -INFINITY;
                e_hi = bl < n_bins ? hi * (1.0 - kEdgeLog) : INFINITY;
            }
            if (spw) {
                const int pos = k & (spw - 1);
                tword |= fire ? (uint32_t)j1 << (p.tape_bits * pos) : 0u;
                if (pos == spw - 1) {
                    if (have && gl == 0) p.tape[tape_at(p, g, k >> tshift)] = tword;
                    tword = 0u;
                }
            }
            group_apply<L>(tab, sx, fire ? j1 : 0, +1, gl, fire);
            t = fire ? tn : t;
            n_done += fire ? 1 : 0;
            active = fire;
        }
        if (have) {
            if (spw && (k & (spw - 1)) != 0 && gl == 0) p.tape[tape_at(p, g, k >> tshift)] = tword;
            if (bin < n_bins) {
                double xo[kObsMax];
#pragma unroll
                for (int o = 0; o < kObsMax; ++o) xo[o] = o < nd.n_obs ? (double)sx[osp[o]] : 0.0;
                double t0 = t;
                while (bin < n_bins) {
                    const double hi = bin_hi;
#pragma unroll
                    for (int o = 0; o < kObsMax; ++o) {
                        acc[o] += xo[o] * fmax(fmin(hi, t_obs) - t0, 0.0);
                        if (o < nd.n_obs && gl == 0) obs_lane[((int64_t)bin * nd.n_obs + o) * B] = acc[o] * inv_dt;
                        acc[o] = 0.0;
                    }
                    t0 = fmax(t0, hi);
                    bin += 1;
                    bin_hi = bin < n_bins ? bin_edge(t_obs, bin + 1, n_bins) : INFINITY;
                }
            }
            if (p.obs_kind == 0 && gl == 0)
                for (int o = 0; o < nd.n_obs; ++o) obs_lane[(int64_t)o * B] = (double)sx[osp[o]];
            for (int s = gl; s < N; s += L) {
                p.x_final[nd.state_off + s * B + i] = sx[s];
                if (sx[s] < 0) flags |= kFlagOverflow;
            }
            if (gl == 0) {
                p.t_final[g] = t;
                p.steps_done[g] = n_done;
            }
        }
        if (flags) atomicOr(p.flags, flags);
        wave_sync();
    }
}

// --------------------------------------------------------------------------
// waves per SIMD the backward's registers are held to
template <int L, int BPL>
constexpr int bwd_waves() { return BPL == 1 && L == 64 ? 3 : BPL == 2 && L < 64 ? 1 : 2; }

// TMODE: 0 for 1/T = 2, 1 for 1/T = 1, 2 for any other temperature
template <int L, int BPL, int TMODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(bwd_waves<L, BPL>())))
void bwd_kernel(RunParams p)
{
    constexpr int G = 64 / L;
    constexpr int C = 4 * BPL;
    constexpr int MMAX = 4 * BPL * L;          // channel slots of a group
    constexpr int KREC = 64;
    __shared__ int s_x[kWaves][G][kMaxN + 1];   // + the constant-1 slot kOne
    __shared__ float s_lam32[kWaves][G][kMaxN];      // FP32 view of lambda (base + increments)
    __shared__ float s_inc[kWaves][G][2 * MMAX + 1];  // per-channel contributions to dlambda[s1], dlambda[s2],
                                                      // in incidence-slot order, + a sink slot
    __shared__ uint16_t s_tape[kWaves][G][KREC];       // channel indices reach 510
    extern __shared__ int32_t s_dyn[];
    const int wid = uniform_i((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane & (L - 1);
    int *sx = s_x[wid][grp];
    float *slam = s_lam32[wid][grp];
    float *sinc = s_inc[wid][grp];
    uint16_t *stape = s_tape[wid][grp];
    GroupTab tab(s_dyn + (wid * G + grp) * p.tab_words, p);
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);
    const float invT = 1.0f / run_temperature(p);

    LaneChannels<L, BPL> ch;
    int cached_net = -1;
    for (;;) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(p.work_counter, (uint32_t)G);
        base = (uint32_t)uniform_i((int)__shfl((int)base, 0));
        if (base >= (uint32_t)p.n_items) break;
        const uint32_t item = base + grp;
        const bool have = item < (uint32_t)p.n_items;
        const LaneItem it = p.items[have ? item : 0];
        const NetDev nd = p.nets[it.net];
        if (it.net != cached_net) {
            ch.load(p, nd, gl);
            tab.load(p, nd, gl, L);
            cached_net = it.net;
        }
        const int N = nd.N, M = nd.M;
        const int64_t B = nd.B;
        const int64_t i = it.first;
        const int64_t g = nd.traj_off + i;
        const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
        const int n = have ? p.steps_done[g] : 0;
        int kmax = n;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) kmax = max(kmax, __shfl_xor(kmax, off));
        kmax = uniform_i(kmax);

        for (int s = gl; s < N; s += L) sx[s] = have ? p.x_final[nd.state_off + s * B + i] : 0;
        if (gl == 0) sx[kOne] = 1;
        double t = have ? p.t_final[g] : 0.0;
        int osp[kObsMax];
#pragma unroll
        for (int o = 0; o < kObsMax; ++o) osp[o] = o < nd.n_obs ? p.obs_sp[nd.obs_sp_off + o] : kNoSpecies;
        const bool bins = p.obs_kind == 1 && nd.n_obs > 0;
        const int n_bins = p.n_bins;
        const double t_obs = nd.t_obs;
        const double inv_dt = bins ? (double)n_bins / t_obs : 0.0;
        const double *dobs_lane = p.d_obs + nd.obsb_off * (p.obs_kind == 1 ? n_bins : 1) + i;

        // lambda of species s = gl + L*m lives in this lane: FP64 base + FP32 increment
        constexpr int SPL = (kMaxN + L - 1) / L;
        double lam[SPL];
        float dlam[SPL];
#pragma unroll
        for (int m = 0; m < SPL; ++m) { lam[m] = 0.0; dlam[m] = 0.f; }
        double lam_t = 0.0;
        double dth[C];
        float dth32[C];
#pragma unroll
        for (int q = 0; q < C; ++q) { dth[q] = 0.0; dth32[q] = 0.f; }

        // direct dependence on the final state
        int rbin = n_bins;
        double rlo = t_obs;
        double dob[kObsMax] = {0.0, 0.0, 0.0, 0.0};
        double lam_obs0[kObsMax] = {0.0, 0.0, 0.0, 0.0};   // contributions to lambda of observed species
        if (have) {
            if (bins) {
                double hi = t_obs;
                while (rbin > 0 && t < rlo) {
                    rbin -= 1;
                    rlo = bin_edge(t_obs, rbin, n_bins);
#pragma unroll
                    for (int o = 0; o < kObsMax; ++o)
                        dob[o] = o < nd.n_obs ? dobs_lane[((int64_t)rbin * nd.n_obs + o) * B] : 0.0;
                    const double seg = hi - fmax(t, rlo);
#pragma unroll
                    for (int o = 0; o < kObsMax; ++o) lam_obs0[o] += dob[o] * seg * inv_dt;
                    hi = rlo;
                }
            } else if (p.obs_kind == 0) {
#pragma unroll
                for (int o = 0; o < kObsMax; ++o)
                    lam_obs0[o] = o < nd.n_obs ? dobs_lane[(int64_t)o * B] : 0.0;
            }
        }
#pragma unroll
        for (int m = 0; m < SPL; ++m) {
            const int s = gl + L * m;
#pragma unroll
            for (int o = 0; o < kObsMax; ++o)
                if (o < nd.n_obs && osp[o] == s) lam[m] += lam_obs0[o];
            if (s < N) slam[s] = (float)lam[m];
        }
        wave_sync();

        const int spw = p.tape_bits ? 32 / p.tape_bits : 1;
        const int tshift = __builtin_ctz(spw);
        const uint32_t tmask = p.tape_bits ? ((1u << p.tape_bits) - 1u) : 0u;
        const int n_seg = (kmax + p.K - 1) / p.K;
        uint32_t flags = 0u;
        int fold_left = kFold;

        for (int cseg = n_seg - 1; cseg >= 0; --cseg) {
            const int k_lo = cseg * p.K;
            const int k_hi = min(k_lo + p.K, kmax);
            if (p.recompute) {
                // re-run the segment from its checkpoint to recover the fired channels
                int xs[SPL];
#pragma unroll
                for (int m = 0; m < SPL; ++m) {
                    const int s = gl + L * m;
                    xs[m] = s < N ? sx[s] : 0;
                }
                if (k_lo < n)
                    for (int s = gl; s < N; s += L)
                        sx[s] = p.ck_x[ckx_at(p, nd, cseg, i, s)];
                wave_sync();
                for (int k = k_lo; k < k_hi; ++k) {
                    const bool on_k = k < n;
                    float a[C];
#pragma unroll
                    for (int q = 0; q < C; ++q) {
                        const float x1 = (float)xval(sx, ch.s1[q]);
                        const float x2 = (float)(xval(sx, ch.s2[q]) - ch.homo[q]);
                        a[q] = ch.on[q] ? fabsf((ch.c[q] * x1) * x2) : 0.f;
                    }
                    uint32_t wd[C];
                    group_words<L, BPL>(M, gl, (uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, wd);
                    float r1 = INFINITY, r2 = INFINITY;
                    int j1 = 0x7FFFFFFF;
#pragma unroll
                    for (int q = 0; q < C; ++q) {
                        const float rq = ch.on[q] ? neglog_u(wd[q]) * fast_rcp(a[q]) : INFINITY;
                        const bool lt = rq < r1;
                        r2 = lt ? r1 : fminf(r2, rq);
                        j1 = lt ? ch.j[q] : j1;
                        r1 = fminf(r1, rq);
                    }
                    grace<L>(r1, j1, r2);
                    if (on_k && gl == 0) stape[k - k_lo] = (uint16_t)j1;
                    group_apply<L>(tab, sx, on_k ? j1 : 0, +1, gl, on_k);
                }
                // back to the state at the segment's end
#pragma unroll
                for (int m = 0; m < SPL; ++m) {
                    const int s = gl + L * m;
                    if (s < N) sx[s] = xs[m];
                }
                wave_sync();
            }
            if (k_hi < n) {
                const int64_t c1 = cseg + 1;
                for (int s = gl; s < N; s += L) sx[s] = p.ck_x[ckx_at(p, nd, c1, i, s)];
                t = p.ck_t[ckt_at(p, g, c1)];
                wave_sync();
            }
            uint32_t tword = 0u, tnext = 0u;
            int tword_idx = -1;
            for (int k = k_hi - 1; k >= k_lo; --k) {
                if (fold_left == 0) {
#pragma unroll
                    for (int m = 0; m < SPL; ++m) {
                        const int s = gl + L * m;
                        lam[m] += (double)dlam[m];
                        dlam[m] = 0.f;
                        if (s < N) slam[s] = (float)lam[m];
                    }
#pragma unroll
                    for (int q = 0; q < C; ++q) { dth[q] += (double)dth32[q]; dth32[q] = 0.f; }
                    fold_left = kFold;
                    wave_sync();
                }
                fold_left -= 1;
                const bool on_k = k < n;
                if (ballot(on_k) == 0ull) continue;
                int j;
                if (p.recompute) {
                    wave_sync();
                    j = stape[k - k_lo];
                } else {
                    // the word of the next (earlier) steps is fetched one word ahead
                    const int widx = k >> tshift;
                    if (widx != tword_idx) {
                        tword = (widx == tword_idx - 1) ? tnext
                                                        : (have ? p.tape[tape_at(p, g, widx)] : 0u);
                        tword_idx = widx;
                        tnext = (have && widx > 0) ? p.tape[tape_at(p, g, widx - 1)] : 0u;
                    }
                    j = (int)((tword >> (p.tape_bits * (k & (spw - 1)))) & tmask);
                }
                // observed counts of X_{k+1}, then X_{k+1} -> X_k (the fired
                // channel's descriptor is read together with the counts)
                const int jcsr = tab.desc[on_k ? j : 0];
                int xn[kObsMax];
#pragma unroll
                for (int o = 0; o < kObsMax; ++o) xn[o] = o < nd.n_obs ? sx[osp[o]] : 0;
                wave_sync();
                group_apply_desc<L>(tab, sx, jcsr, -1, gl, on_k);

                float a[C], A1[C], A2[C];
                float a0 = 0.f;
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    const float x1 = (float)xval(sx, ch.s1[q]);
                    const float x2 = (float)(xval(sx, ch.s2[q]) - ch.homo[q]);
                    const float u1 = ch.c[q] * x1;
                    a[q] = ch.on[q] ? fabsf(u1 * x2) : 0.f;
                    A1[q] = ch.on[q] ? u1 : 0.f;
                    A2[q] = ch.on[q] ? ch.c[q] * x2 : 0.f;
                    a0 += a[q];
                }
                a0 = gsum<L>(a0);
                uint32_t wd[C];
                group_words<L, BPL>(M, gl, (uint32_t)k, tid, pe, p.seed_lo, p.seed_hi, wd);
                const float rcp_a0 = fast_rcp(a0);
                const float e0 = group_first<L>(neglog_u(wd[0]));
                const float tau = e0 * rcp_a0;
                const double t_k = t - (double)tau;
                if (on_k && bins && rbin < n_bins) {
#pragma unroll
                    for (int o = 0; o < kObsMax; ++o)
                        if (o < nd.n_obs) lam_t += dob[o] * (double)(sx[osp[o]] - xn[o]) * inv_dt;
                }
                // soft sample in ratio form, relative to the fired channel j
                // (the race's winner, so every ratio is at most 1)
                float r[C], ra[C];
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    const bool onq = ch.on[q] && a[q] > 0.f;
                    ra[q] = onq ? fast_rcp(a[q]) : 0.f;
                    r[q] = onq ? neglog_u(wd[q]) * ra[q] : INFINITY;
                }
                const Owner own = owner_of<L, BPL>(j, grp);
                const float rref = from_owner<L, C>(r, own);
                float y[C];
                float ys = 0.f;
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    float v = rref * fast_rcp(r[q]);
                    if (TMODE == 0) v = v * v;
                    else if (TMODE == 2) v = v > 0.f ? exp2f(log2f(v) * invT) : 0.f;
                    y[q] = v;
                    ys += v;
                }
                ys = gsum<L>(ys);
                const float rys = fast_rcp(ys);
                // w_q = v_q . lambda(k+1)
                float wv[C];
                if (p.wide_ve) {
#pragma unroll
                    for (int q = 0; q < C; ++q) {
                        float s = 0.f;
                        if (ch.on[q]) {
                            const int d = tab.desc[ch.j[q]];
                            const int beg = d & 0xFFFFFF, cnt = (int)((uint32_t)d >> 24);
                            for (int e = 0; e < cnt; ++e) {
                                const int32_t ent = tab.ent[beg + e];
                                s += (float)csr_delta(ent) * slam[csr_species(ent)];
                            }
                        }
                        wv[q] = s;
                    }
                } else {
                    // padding entries are species 0 with delta 0; the entries
                    // stay packed across the step loop (to save registers)
                    // and are decoded here, two channels at a time with all
                    // their reads of lambda issued before the first is waited
                    // for, then each channel summed in entry order
#pragma unroll
                    for (int q0 = 0; q0 < C; q0 += 2) {
                        uint32_t w[2][kVecSlots / 2];
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int e2 = 0; e2 < kVecSlots / 2; ++e2) {
                                w[h][e2] = ch.ve[q0 + h][e2];
                                asm volatile("" : "+v"(w[h][e2]));
                            }
                        float lv[2][kVecSlots];
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int e = 0; e < kVecSlots; ++e)
                                lv[h][e] = slam[(int)((w[h][e >> 1] >> (16 * (e & 1))) & 0xFFu)];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            float s = 0.f;
#pragma unroll
                            for (int e = 0; e < kVecSlots; ++e) {
                                const int dl = (int)(int8_t)(uint8_t)((w[h][e >> 1] >> (16 * (e & 1) + 8)) & 0xFFu);
                                s += (float)dl * lv[h][e];
                            }
                            wv[q0 + h] = s;
                        }
                    }
                }
                // reference value w_j from the lane owning channel j
                const float wref = from_owner<L, C>(wv, own);
                float wb = 0.f;
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    y[q] *= rys;
                    wb += y[q] * (wv[q] - wref);
                }
                const float wbar = gsum<L>(wb);
                const float cc = (float)(lam_t * (double)(-tau * rcp_a0));
                // per-channel gradient terms and contributions to dlambda
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    const float gq = y[q] * ((wv[q] - wref) - wbar) * invT;
                    const float coef = gq * ra[q] + cc;
                    if (on_k && ch.on[q]) {
                        dth32[q] += gq + cc * a[q];
                        uint32_t ps = ch.pos[q];
                        asm volatile("" : "+v"(ps));
                        sinc[ps & 0xFFFFu] = coef * A2[q];
                        sinc[ps >> 16] = coef * A1[q];
                    }
                }
                wave_sync();
                // gather per species in a fixed order (incidence list)
                if (on_k) {
#pragma unroll
                    for (int m = 0; m < SPL; ++m) {
                        const int s = gl + L * m;
                        if (s < N) {
                            // the species' slots in order, eight reads in flight
                            const int end = tab.inc_ptr[s + 1];
                            int e = tab.inc_ptr[s];
                            float d = 0.f;
                            for (; e + 8 <= end; e += 8) {
                                const float v0 = sinc[e], v1 = sinc[e + 1], v2 = sinc[e + 2], v3 = sinc[e + 3];
                                const float v4 = sinc[e + 4], v5 = sinc[e + 5], v6 = sinc[e + 6], v7 = sinc[e + 7];
                                d = (((((((d + v0) + v1) + v2) + v3) + v4) + v5) + v6) + v7;
                            }
                            for (; e + 4 <= end; e += 4) {
                                const float v0 = sinc[e], v1 = sinc[e + 1], v2 = sinc[e + 2], v3 = sinc[e + 3];
                                d = (((d + v0) + v1) + v2) + v3;
                            }
                            for (; e < end; ++e) d += sinc[e];
                            dlam[m] += d;
                        }
                    }
                }
                // direct dL/dX_k over [t_k, t_{k+1})
                double dobs_x[kObsMax] = {0.0, 0.0, 0.0, 0.0};
                if (on_k && bins) {
                    double hi = fmin(t, t_obs);
                    while (t_k < rlo && rbin > 0) {
                        if (rbin < n_bins) {
                            const double seg = fmax(hi - rlo, 0.0);
#pragma unroll
                            for (int o = 0; o < kObsMax; ++o) dobs_x[o] += dob[o] * seg * inv_dt;
                        }
                        hi = fmin(hi, rlo);
                        rbin -= 1;
                        rlo = bin_edge(t_obs, rbin, n_bins);
#pragma unroll
                        for (int o = 0; o < kObsMax; ++o)
                            dob[o] = o < nd.n_obs ? dobs_lane[((int64_t)rbin * nd.n_obs + o) * B] : 0.0;
                    }
                    if (rbin < n_bins) {
                        const double seg = fmax(hi - t_k, 0.0);
#pragma unroll
                        for (int o = 0; o < kObsMax; ++o) dobs_x[o] += dob[o] * seg * inv_dt;
                    }
                }
#pragma unroll
                for (int m = 0; m < SPL; ++m) {
                    const int s = gl + L * m;
#pragma unroll
                    for (int o = 0; o < kObsMax; ++o)
                        if (o < nd.n_obs && osp[o] == s) dlam[m] += (float)dobs_x[o];
                    if (s < N) slam[s] = (float)lam[m] + dlam[m];
                }
                if (on_k && (!(a0 > 0.f) || !(tau >= 0.f))) flags |= kFlagNonFinite;
                t = on_k ? t_k : t;
                wave_sync();
            }
        }
#pragma unroll
        for (int q = 0; q < C; ++q) dth[q] += (double)dth32[q];
        if (have) {
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (ch.on[q]) p.partials[nd.part_off + (int64_t)ch.j[q] * B + i] = dth[q];
        }
        if (flags) atomicOr(p.flags, flags);
        wave_sync();
    }
}

}  // namespace wave

int wave_class_for(int max_M, int max_lanes)
{
    const int nb = (max_M + 1 + 3) / 4;
    // one block per lane within the cap
    if (nb <= 8 && max_lanes >= 8) return kWave_L8;
    if (nb <= 16 && max_lanes >= 16) return kWave_L16;
    if (nb <= 32 && max_lanes >= 32) return kWave_L32;
    // two blocks per lane at the cap
    if (nb <= 2 * max_lanes) {
        switch (max_lanes) {
        case 8: return kWave_L8x2;
        case 16: return kWave_L16x2;
        case 32: return kWave_L32x2;
        default: break;
        }
    }
    // too large for the cap: the library's own width
    if (nb <= 8) return kWave_L8;
    if (nb <= 16) return kWave_L16;
    if (nb <= 32) return kWave_L32;
    if (nb <= 64) return kWave_L64;
    if (nb <= 128) return kWave_L64x2;
    return -1;
}

int wave_class_lanes(int cls)
{
    switch (cls) {
    case kWave_L8: case kWave_L8x2: return 8;
    case kWave_L16: case kWave_L16x2: return 16;
    case kWave_L32: case kWave_L32x2: return 32;
    default: return 64;
    }
}

int wave_class_bpl(int cls)
{
    return cls == kWave_L64x2 || cls == kWave_L8x2 || cls == kWave_L16x2 || cls == kWave_L32x2 ? 2 : 1;
}

template <int L, int BPL>
static hipError_t launch_wave(const RunParams &p, bool backward, int n_blocks, hipStream_t stream)
{
    const size_t dyn = sizeof(int32_t) * (size_t)p.tab_words * wave::kWaves * (64 / L);
    if (backward) {
        // a temperature read on the device takes the general form
        const float invT = p.d_temperature ? 0.f : 1.0f / p.temperature;
        if (invT == 2.0f)
            hipLaunchKernelGGL((wave::bwd_kernel<L, BPL, 0>), dim3(n_blocks), dim3(wave::kBlock), dyn, stream, p);
        else if (invT == 1.0f)
            hipLaunchKernelGGL((wave::bwd_kernel<L, BPL, 1>), dim3(n_blocks), dim3(wave::kBlock), dyn, stream, p);
        else
            hipLaunchKernelGGL((wave::bwd_kernel<L, BPL, 2>), dim3(n_blocks), dim3(wave::kBlock), dyn, stream, p);
    } else
        hipLaunchKernelGGL((wave::fwd_kernel<L, BPL>), dim3(n_blocks), dim3(wave::kBlock), dyn, stream, p);
    return hipGetLastError();
}

size_t wave_static_lds(int cls, bool backward)
{
    const int L = wave_class_lanes(cls);
    const int G = 64 / L;
    const int bpl = wave_class_bpl(cls);
    size_t b = sizeof(int) * wave::kWaves * G * (wave::kMaxN + 1);
    if (backward)
        b += sizeof(float) * wave::kWaves * G * wave::kMaxN + sizeof(float) * wave::kWaves * G * (2 * 4 * bpl * L + 1) +
             sizeof(uint16_t) * wave::kWaves * G * 64;
    return b;
}

hipError_t wave_launch(int cls, const RunParams &p, bool backward, int n_blocks, hipStream_t stream)
{
    switch (cls) {
    case kWave_L8: return launch_wave<8, 1>(p, backward, n_blocks, stream);
    case kWave_L16: return launch_wave<16, 1>(p, backward, n_blocks, stream);
    case kWave_L32: return launch_wave<32, 1>(p, backward, n_blocks, stream);
    case kWave_L64: return launch_wave<64, 1>(p, backward, n_blocks, stream);
    case kWave_L64x2: return launch_wave<64, 2>(p, backward, n_blocks, stream);
    case kWave_L8x2: return launch_wave<8, 2>(p, backward, n_blocks, stream);
    case kWave_L16x2: return launch_wave<16, 2>(p, backward, n_blocks, stream);
    case kWave_L32x2: return launch_wave<32, 2>(p, backward, n_blocks, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ssa
