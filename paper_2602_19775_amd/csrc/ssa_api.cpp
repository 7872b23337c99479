// C ABI of libssa (declared in include/ssa.h): argument checks, device
// tables, buffer layout and kernel launches.  Nothing here allocates,
// frees or synchronises inside ssa_forward / ssa_backward / ssa_step_batch.
#include "ssa.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ssa_host.hpp"
#include "ssa_jit.hpp"
#include "ssa_lane.hpp"
#include "ssa_wave.hpp"
#include "ssa_misc.hpp"
#include "ssa_plan.hpp"

using namespace ssa;

static_assert(sizeof(TieRec) == sizeof(ssa_tie), "tie record layout");

namespace ssa {

thread_local std::string g_last_error;

ssa_status fail(ssa_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

ssa_status hip_fail(hipError_t e, const char *what)
{
    return fail(SSA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace ssa

namespace {

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * src.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

size_t align_up(size_t x, size_t a)
{
    return (x + a - 1) / a * a;
}

}  // namespace

struct ssa_net {
    int n_networks = 0;
    std::vector<NetDev> nets_h;
    NetDev *nets_d = nullptr;
    ReactDesc *rd_d = nullptr;
    uint32_t *rows_d = nullptr;
    int32_t *csr_d = nullptr;
    int32_t *obs_sp_d = nullptr;
    int32_t *pmap_off_d = nullptr;
    int32_t *pmap_ch_d = nullptr;
    int32_t *param_net_d = nullptr;
    int32_t *inc_ptr_d = nullptr;
    int32_t *chan_inc_d = nullptr;
    // one launch per group: a generic lane class, or a topology-specialised kernel pair
    struct Group {
        bool spec = false;
        int lane_class = -1;
        int wave_class = -1;     // persistent wave-mode launch
        int wave_blocks = 0;
        int tab_m = 0, tab_nnz = 0;   // per-group LDS table capacities
        int wide_ve = 0;              // a channel changes more than kVecSlots species
        SpecKernels kernels;
        int spec_nobs = 0;            // observed species of the group's topology
        LaneItem *items_d = nullptr;
        int n_items = 0;
    };
    std::vector<Group> groups;
    uint32_t *flags_d = nullptr;
    int64_t traj_total = 0, state_total = 0, param_total = 0, obsb_total = 0, part_total = 0,
            ppt_total = 0, obsw_total = 0, tobs_total = 0, obst_total = 0, obstw_total = 0, tanw_total = 0;
    int max_M = 0;
    bool tangent_fit = false;   // every network runs in the specialised mode within the tangent limits
    int64_t max_B = 0;
    int device = 0;
    void *scratch = nullptr;     // this device's copy of the static scratch array
};

// Scratch of ssa_backward_static: a file-scope device array, one copy per
// GPU, in place of the caller's work buffer.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address): ssa_net_create resolves the address of the current device's copy
// once per device and every handle keeps it.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_of_device;

// Device address of `scratch` on `device`, which must be the current device.
hipError_t static_scratch(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_of_device.find(device);
    if (it != g_scratch_of_device.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_of_device[device] = ptr;
    *out = ptr;
    return hipSuccess;
}

}  // namespace

namespace {

// Layout of the caller's checkpoint buffer for a configuration.
struct CkptLayout {
    int32_t n_ckpt = 0;
    int32_t tape_bits = 0;
    int32_t tape_words = 0;
    size_t off_t = 0, off_x = 0, off_tape = 0, bytes = 0;
};

// Tape bits per step: enough for channel indices 0..M-1 (the wave mode runs
// networks of up to 511 channels).
int bits_for(int M)
{
    if (M <= 2) return 1;
    if (M <= 4) return 2;
    if (M <= 16) return 4;
    if (M <= 256) return 8;
    return 16;
}

int resolve_bwd_mode(const ssa_config *cfg)
{
    return cfg->bwd_mode == SSA_BWD_AUTO ? SSA_BWD_TAPE : cfg->bwd_mode;
}

constexpr int kMaxRecomputeSegment = 64;
// values a wave of the ensemble-mean forward sums in LDS (16 bytes each:
// a fixed-point sum and two difference-array counts, plus 8 bytes an observed
// species for the arrays' end slots), and the LDS of a wave (4 waves a block
// within the 64 KiB a workgroup may hold; with at most kObsMax observed
// species the first bound implies the second)
constexpr int64_t kMeanMaxValues = 1000;
constexpr int64_t kMeanLdsPerWave = 16384;

bool bounded_steps(const ssa_config *cfg)
{
    return cfg->n_steps < INT32_MAX;
}

CkptLayout ckpt_layout(const ssa_net *net, const ssa_config *cfg)
{
    CkptLayout L;
    if (!bounded_steps(cfg) || cfg->ckpt_every < 1) return L;
    if (cfg->bwd_mode == SSA_BWD_TANGENT) {
        // no checkpoints or tape: the tangents d obs / d ln k_q
        const int64_t npts = cfg->obs_kind == SSA_OBS_BINS ? cfg->n_bins : 1;
        L.bytes = align_up(sizeof(double) * (size_t)(net->tanw_total * npts), 256);
        if (L.bytes == 0) L.bytes = 256;
        return L;
    }
    L.n_ckpt = (int32_t)(((int64_t)cfg->n_steps + cfg->ckpt_every - 1) / cfg->ckpt_every);
    if (resolve_bwd_mode(cfg) == SSA_BWD_TAPE) {
        L.tape_bits = bits_for(net->max_M);
        const int spw = 32 / L.tape_bits;
        L.tape_words = (int32_t)(((int64_t)cfg->n_steps + spw - 1) / spw + 1);
    }
    size_t off = 0;
    L.off_t = off;
    off = align_up(off + sizeof(double) * (size_t)L.n_ckpt * net->traj_total, 256);
    L.off_x = off;
    off = align_up(off + sizeof(int32_t) * (size_t)L.n_ckpt * net->state_total, 256);
    L.off_tape = off;
    off = align_up(off + sizeof(uint32_t) * (size_t)L.tape_words * net->traj_total, 256);
    L.bytes = off;
    return L;
}

// Work buffer: [header: work counter] then FP64 per-channel partials, then
// the per-chunk sums of the gradient reduction.
constexpr size_t kWorkHeader = 256;

size_t partials_bytes(const ssa_net *net)
{
    return align_up(sizeof(double) * (size_t)net->part_total, 256);
}

size_t grad_work_bytes(const ssa_net *net)
{
    return kWorkHeader + partials_bytes(net) +
           align_up(sizeof(double) * (size_t)net->param_total * reduce_chunks(net->max_B), 256);
}

// values per trajectory of network nd for the observation of cfg
int64_t obs_width(const NetDev &nd, const ssa_config *cfg)
{
    if (cfg->obs_kind == SSA_OBS_TAIL) return (int64_t)nd.n_obs + 1;
    return (int64_t)nd.n_obs * (cfg->obs_kind != SSA_OBS_FINAL ? cfg->n_bins : 1);
}

// first value of network nd in the observation buffer and in the buffer of
// ensemble means, for the observation kind and point count of a query
int64_t obs_block_offset(const NetDev &nd, int32_t obs_kind, int32_t n_bins)
{
    if (obs_kind == SSA_OBS_TAIL) return nd.obst_off;
    return nd.obsb_off * (obs_kind != SSA_OBS_FINAL ? n_bins : 1);
}

int64_t mean_block_offset(const NetDev &nd, int32_t obs_kind, int32_t n_bins)
{
    if (obs_kind == SSA_OBS_TAIL) return nd.obstw_off;
    return nd.obsw_off * (obs_kind != SSA_OBS_FINAL ? n_bins : 1);
}

// values of the whole observation buffer for cfg (0: nothing observed)
int64_t obs_total(const ssa_net *net, const ssa_config *cfg)
{
    return cfg->obs_kind == SSA_OBS_TAIL ? net->obst_total : net->obsb_total;
}

// The ensemble-mean chunk sums follow the gradient region of the work buffer.
size_t mean_work_bytes(const ssa_net *net, const ssa_config *cfg)
{
    size_t m = 0;
    for (const NetDev &nd : net->nets_h)
        m = std::max(m, sizeof(double) * (size_t)obs_mean_chunks(nd.B) * (size_t)obs_width(nd, cfg));
    return align_up(m, 256);
}

// Prefix sums of a shared bin dL/dobs block follow the ensemble-mean region.
size_t prefix_work_bytes(const ssa_net *net, const ssa_config *cfg)
{
    if (!cfg->dobs_shared || cfg->obs_kind != SSA_OBS_BINS) return 0;
    return align_up(sizeof(double) * (size_t)net->obsw_total * (size_t)(cfg->n_bins + 1), 256);
}

// Per-tile sums of the ensemble-mean forward follow the prefix sums.
size_t tile_work_bytes(const ssa_net *net, const ssa_config *cfg)
{
    if (cfg->obs_layout != SSA_OBS_ENSEMBLE_MEAN) return 0;
    return align_up(sizeof(double) * (size_t)net->tobs_total * (size_t)cfg->n_bins, 256);
}

size_t work_bytes_for(const ssa_net *net, const ssa_config *cfg)
{
    return grad_work_bytes(net) + mean_work_bytes(net, cfg) + prefix_work_bytes(net, cfg) +
           tile_work_bytes(net, cfg);
}

double *tile_sums_of(const ssa_net *net, const ssa_config *cfg, void *work)
{
    return (double *)((char *)work + grad_work_bytes(net) + mean_work_bytes(net, cfg) +
                      prefix_work_bytes(net, cfg));
}

ssa_status check_config(const ssa_net *net, const ssa_config *cfg)
{
    if (!net) return fail(SSA_EINVAL, "network handle is NULL");
    if (!cfg) return fail(SSA_EINVAL, "config is NULL");
    if (cfg->n_steps < 0) return fail(SSA_EINVAL, "n_steps must be >= 0");
    if (!(cfg->t_end > 0.0)) return fail(SSA_EINVAL, "t_end must be > 0 (use INFINITY for no limit)");
    if (cfg->obs_kind != SSA_OBS_FINAL && cfg->obs_kind != SSA_OBS_BINS && cfg->obs_kind != SSA_OBS_GRID &&
        cfg->obs_kind != SSA_OBS_TAIL)
        return fail(SSA_EINVAL, "obs_kind must be SSA_OBS_FINAL, SSA_OBS_BINS, SSA_OBS_GRID or SSA_OBS_TAIL");
    if (cfg->obs_kind == SSA_OBS_TAIL) {
        if (!bounded_steps(cfg) || cfg->n_bins < 1 || cfg->n_bins > cfg->n_steps)
            return fail(SSA_EINVAL, "tail observation needs a bounded n_steps and 1 <= n_bins <= n_steps");
        if (cfg->obs_layout != SSA_OBS_POINT_MAJOR || cfg->dobs_shared)
            return fail(SSA_ENOTSUP, "the tail observation runs in the point-major layout with a per-trajectory d_obs");
        if (cfg->selection != SSA_SELECT_GUMBEL_MAX)
            return fail(SSA_ENOTSUP, "the tail observation runs with the Gumbel-max selection");
        for (const auto &gr : net->groups)
            if (gr.n_items && !gr.spec)
                return fail(SSA_ENOTSUP, "the tail observation runs in the topology-specialised lane mode only");
    }
    if (cfg->obs_kind == SSA_OBS_BINS) {
        if (cfg->n_bins < 1) return fail(SSA_EINVAL, "bin observation needs n_bins >= 1");
        for (const NetDev &nd : net->nets_h)
            if (nd.n_obs > 0 && !(nd.t_obs > 0.0) )
                return fail(SSA_EINVAL, "bin observation needs t_obs > 0 for every observed network");
    }
    if (cfg->obs_kind == SSA_OBS_GRID) {
        if (cfg->n_bins < 2) return fail(SSA_EINVAL, "grid observation needs n_bins >= 2 grid points");
        for (const NetDev &nd : net->nets_h)
            if (nd.n_obs > 0 && !(nd.t_obs > 0.0) )
                return fail(SSA_EINVAL, "grid observation needs t_obs > 0 for every observed network");
        for (const auto &gr : net->groups)
            if (gr.n_items && !gr.spec)
                return fail(SSA_ENOTSUP, "grid observation runs in the topology-specialised lane mode only");
    }
    if (!(cfg->temperature > 0.f) || !std::isfinite(cfg->temperature))
        return fail(SSA_EINVAL, "temperature must be finite and > 0");
    if (cfg->ckpt_every < 1) return fail(SSA_EINVAL, "ckpt_every must be >= 1");
    const int mode = resolve_bwd_mode(cfg);
    if (mode != SSA_BWD_TAPE && mode != SSA_BWD_RECOMPUTE && mode != SSA_BWD_TANGENT)
        return fail(SSA_EINVAL, "unknown bwd_mode");
    if (mode == SSA_BWD_TANGENT) {
        if (!net->tangent_fit)
            return fail(SSA_ENOTSUP, "forward-mode tangents need the topology-specialised lane mode and networks of "
                                     "at most 4 channels and 32 species x channels");
        if (cfg->obs_kind != SSA_OBS_FINAL && cfg->obs_kind != SSA_OBS_BINS)
            return fail(SSA_ENOTSUP, "forward-mode tangents run with the final or bin observation");
        if (cfg->obs_layout != SSA_OBS_POINT_MAJOR || cfg->dobs_shared)
            return fail(SSA_ENOTSUP, "forward-mode tangents use the point-major layout with a per-trajectory d_obs");
        if (cfg->t_end != INFINITY) return fail(SSA_ENOTSUP, "forward-mode tangents run step-limited paths (no t_end)");
        if (cfg->selection != SSA_SELECT_GUMBEL_MAX)
            return fail(SSA_ENOTSUP, "forward-mode tangents need the Gumbel-max selection");
        if (!bounded_steps(cfg)) return fail(SSA_EINVAL, "forward-mode tangents need a bounded n_steps");
    }
    if (mode == SSA_BWD_RECOMPUTE && cfg->ckpt_every > kMaxRecomputeSegment)
        return fail(SSA_EINVAL, "recompute mode needs ckpt_every <= 64");
    if (cfg->tie_capacity < 0) return fail(SSA_EINVAL, "tie_capacity must be >= 0");
    if (cfg->obs_layout != SSA_OBS_POINT_MAJOR && cfg->obs_layout != SSA_OBS_TRAJ_MAJOR &&
        cfg->obs_layout != SSA_OBS_ENSEMBLE_MEAN)
        return fail(SSA_EINVAL, "obs_layout must be SSA_OBS_POINT_MAJOR, SSA_OBS_TRAJ_MAJOR or SSA_OBS_ENSEMBLE_MEAN");
    if (cfg->obs_layout == SSA_OBS_ENSEMBLE_MEAN) {
        if (cfg->obs_kind == SSA_OBS_FINAL)
            return fail(SSA_ENOTSUP, "the ensemble-mean forward observes bins or grid points only");
        for (const NetDev &nd : net->nets_h)
            if ((int64_t)nd.n_obs * cfg->n_bins > kMeanMaxValues ||
                16 * (int64_t)nd.n_obs * cfg->n_bins + 8 * (int64_t)nd.n_obs > kMeanLdsPerWave)
                return fail(SSA_ENOTSUP, "the ensemble-mean forward needs n_bins * n_obs <= 1000 and its sums "
                                         "within 16 KiB of LDS a wave");
    }
    if (cfg->obs_layout != SSA_OBS_POINT_MAJOR || cfg->dobs_shared)
        for (const auto &gr : net->groups)
            if (gr.n_items && !gr.spec)
                return fail(SSA_ENOTSUP, "the trajectory-major and ensemble-mean layouts and a shared d_obs "
                                         "run in the topology-specialised lane mode only");
    if (cfg->selection != SSA_SELECT_GUMBEL_MAX && cfg->selection != SSA_SELECT_INVERSE_CDF)
        return fail(SSA_EINVAL, "unknown selection");
    if (cfg->relaxed)
        return fail(SSA_ENOTSUP, "the relaxed forward runs on the gene-network classifier only");
    if (cfg->selection == SSA_SELECT_INVERSE_CDF) {
        if (cfg->obs_layout == SSA_OBS_ENSEMBLE_MEAN)
            return fail(SSA_ENOTSUP, "the inverse-CDF selection writes per-trajectory observations");
        if (cfg->obs_kind == SSA_OBS_GRID)
            return fail(SSA_ENOTSUP, "the inverse-CDF selection runs with the final or bin observation");
        for (const auto &gr : net->groups)
            if (gr.n_items && !gr.spec)
                return fail(SSA_ENOTSUP, "the inverse-CDF selection runs in the topology-specialised lane mode only");
    }
    return SSA_OK;
}

RunParams base_params(const ssa_net *net, const ssa_config *cfg)
{
    RunParams p;
    std::memset(&p, 0, sizeof(p));
    p.nets = net->nets_d;
    p.rd = net->rd_d;
    p.rows = net->rows_d;
    p.csr = net->csr_d;
    p.obs_sp = net->obs_sp_d;
    p.flags = net->flags_d;
    p.seed_lo = (uint32_t)cfg->seed;
    p.seed_hi = (uint32_t)(cfg->seed >> 32);
    p.purpose = cfg->purpose & 0xFFu;
    p.epoch = cfg->epoch;
    p.d_epoch = cfg->d_epoch;
    p.traj_ids = cfg->traj_ids;
    p.n_steps = cfg->n_steps;
    p.t_end = cfg->t_end;
    p.obs_kind = cfg->obs_kind;
    p.n_bins = cfg->obs_kind != SSA_OBS_FINAL ? cfg->n_bins : 0;
    p.K = cfg->ckpt_every;
    p.state_total = net->state_total;
    p.traj_total = net->traj_total;
    p.temperature = cfg->temperature;
    p.d_temperature = cfg->d_temperature;
    p.selection = cfg->selection;
    p.obs_tm = cfg->obs_layout != SSA_OBS_POINT_MAJOR ? 1 : 0;
    p.obs_ens = cfg->obs_layout == SSA_OBS_ENSEMBLE_MEAN ? 1 : 0;
    p.dobs_shared = cfg->dobs_shared ? 1 : 0;
    p.recompute = resolve_bwd_mode(cfg) == SSA_BWD_RECOMPUTE ? 1 : 0;
    p.inc_ptr = net->inc_ptr_d;
    p.chan_inc = net->chan_inc_d;
    return p;
}

ssa_status launch_all_classes(const ssa_net *net, RunParams p, bool backward, hipStream_t stream)
{
    for (const auto &gr : net->groups) {
        if (!gr.n_items) continue;
        p.items = gr.items_d;
        p.n_items = gr.n_items;
        hipError_t e;
        if (gr.wave_class >= 0) {
            p.tab_m = gr.tab_m;
            p.tab_nnz = gr.tab_nnz;
            p.tab_words = gr.tab_m + gr.tab_nnz + (kWaveMaxSpecies + 1);
            p.wide_ve = gr.wide_ve;
            // the persistent kernel pulls work from a counter that starts at 0
            e = launch_fill_u32(p.work_counter, 1, 0u, stream);
            if (e == hipSuccess) e = wave_launch(gr.wave_class, p, backward, gr.wave_blocks, stream);
        } else {
            const size_t mean_lds = !backward && p.obs_ens
                                        ? spec_waves_per_block * (16 * (size_t)p.n_bins * gr.spec_nobs +
                                                                  8 * (size_t)gr.spec_nobs)
                                        : 0;
            e = gr.spec ? spec_launch(gr.kernels, p, backward, mean_lds, stream)
                        : lane_launch(gr.lane_class, p, backward, stream);
        }
        if (e != hipSuccess) return hip_fail(e, backward ? "backward launch" : "forward launch");
    }
    return SSA_OK;
}



// Topology-specialised kernels are used for networks small enough to keep
// their state in registers, and only while a batch has few distinct
// topologies (each costs one runtime compilation).
constexpr int kSpecMaxSpecies = 64;
constexpr int kSpecMaxChannels = 64;
constexpr int kSpecMaxTopologies = 16;
// The library's own choice takes the specialised kernels for networks of at
// most this many channels: past it their unrolled backward spills (kilobytes
// of scratch a lane from about 48 channels) and compiling one topology grows
// from tens of seconds to minutes.  SSA_EXEC_SPEC still accepts up to
// kSpecMaxChannels.
constexpr int kSpecAutoMaxChannels = 32;



}  // namespace

extern "C" {

void ssa_config_default(ssa_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n_steps = INT32_MAX;
    cfg->t_end = INFINITY;
    cfg->obs_kind = SSA_OBS_FINAL;
    cfg->n_bins = 0;
    cfg->temperature = 0.5f;
    cfg->d_temperature = nullptr;
    cfg->selection = SSA_SELECT_GUMBEL_MAX;
    cfg->ckpt_every = 256;
    cfg->bwd_mode = SSA_BWD_AUTO;
    cfg->tie_capacity = 0;
}

const char *ssa_status_string(ssa_status s)
{
    switch (s) {
    case SSA_OK: return "ok";
    case SSA_EINVAL: return "invalid argument";
    case SSA_ESHAPE: return "unsupported network or batch shape";
    case SSA_EWORKSPACE: return "buffer too small";
    case SSA_EOVERFLOW: return "copy number overflow";
    case SSA_ENONFINITE: return "non-finite propensity or clock";
    case SSA_EHIP: return "HIP runtime error";
    case SSA_ENOTSUP: return "not supported";
    }
    return "unknown status";
}

const char *ssa_last_error(void)
{
    return g_last_error.c_str();
}

ssa_status ssa_net_create(const ssa_network_desc *d, ssa_net **out)
{
    g_last_error.clear();
    if (!d || !out) return fail(SSA_EINVAL, "NULL argument");
    *out = nullptr;
    const int nn = d->n_networks;
    if (nn < 1) return fail(SSA_EINVAL, "n_networks must be >= 1");
    if (!d->n_species || !d->n_reactions || !d->n_params || !d->n_traj || !d->n_obs || !d->reactant ||
        !d->rate_index || !d->stoich)
        return fail(SSA_EINVAL, "missing table in network description");

    ssa_net *net = new ssa_net();
    net->n_networks = nn;
    auto bail = [&](ssa_status st, const std::string &m) {
        ssa_net_destroy(net);
        return fail(st, m);
    };

    // ---- validation and the execution plan -------------------------------
    enum { kSpec = 1, kLane = 2, kWave = 3 };
    int max_M = 0, max_N = 0;
    bool all_spec_fit = true, all_lane_fit = true;
    std::vector<std::string> srcs(nn);
    std::map<std::string, SpecKernels> spec_kernels;
    {
        int64_t roff = 0, soff = 0, ooff = 0;
        for (int n = 0; n < nn; ++n) {
            const int N = d->n_species[n], M = d->n_reactions[n], P = d->n_params[n], B = d->n_traj[n];
            const int nob = d->n_obs[n];
            const std::string tag = "network " + std::to_string(n);
            if (N < 1 || M < 1 || P < 1 || B < 0 || nob < 0) return bail(SSA_EINVAL, tag + ": sizes must be positive");
            if (nob > 4) return bail(SSA_ESHAPE, tag + ": at most 4 observed species per network");
            if (nob > 0 && !d->obs_species) return bail(SSA_EINVAL, "obs_species is NULL");
            if (N > 254) return bail(SSA_ESHAPE, tag + ": at most 254 species");
            for (int j = 0; j < M; ++j) {
                const int s1 = d->reactant[2 * (roff + j)], s2 = d->reactant[2 * (roff + j) + 1];
                const int ri = d->rate_index[roff + j];
                if (s1 < -1 || s1 >= N || s2 < -1 || s2 >= N || (s1 < 0 && s2 >= 0))
                    return bail(SSA_EINVAL, tag + ": bad reactant of channel " + std::to_string(j));
                if (ri < 0 || ri >= P) return bail(SSA_EINVAL, tag + ": rate_index out of range");
                int cnt = 0;
                for (int q = 0; q < N; ++q) {
                    const int v = d->stoich[soff + (int64_t)j * N + q];
                    if (v < -8 || v > 7) return bail(SSA_EINVAL, tag + ": change vector entry out of [-8,7]");
                    cnt += v != 0;
                }
                if (cnt > 255) return bail(SSA_ESHAPE, tag + ": change vector too long");
            }
            for (int o = 0; o < nob; ++o) {
                const int sp = d->obs_species[ooff + o];
                if (sp < 0 || sp >= N) return bail(SSA_EINVAL, tag + ": observed species out of range");
            }
            max_M = std::max(max_M, M);
            max_N = std::max(max_N, N);
            if (N > kSpecMaxSpecies || M > kSpecMaxChannels) all_spec_fit = false;
            if (lane_class_for(N, M) < 0) all_lane_fit = false;
            if (all_spec_fit) {
                srcs[n] = spec_source(N, M, d->reactant + 2 * roff, d->rate_index + roff, d->stoich + soff, nob,
                                      d->obs_species ? d->obs_species + ooff : nullptr);
                spec_kernels.emplace(srcs[n], SpecKernels());
                if ((int)spec_kernels.size() > kSpecMaxTopologies) all_spec_fit = false;
            }
            roff += M;
            soff += (int64_t)M * N;
            ooff += nob;
        }
    }
    const int wave_lanes = d->wave_lanes == 0 ? 64 : d->wave_lanes;
    if (wave_lanes != 8 && wave_lanes != 16 && wave_lanes != 32 && wave_lanes != 64)
        return bail(SSA_EINVAL, "wave_lanes must be 0, 8, 16, 32 or 64");
    const bool wave_fit = max_N <= kWaveMaxSpecies && wave_class_for(max_M, wave_lanes) >= 0;
    if (d->exec_mode < SSA_EXEC_AUTO || d->exec_mode > SSA_EXEC_WAVE) return bail(SSA_EINVAL, "unknown exec_mode");
    int mode = d->exec_mode;
    if (mode == kSpec && !all_spec_fit) return bail(SSA_ESHAPE, "specialised lane mode does not fit this batch");
    if (mode == kLane && !all_lane_fit) return bail(SSA_ESHAPE, "generic lane mode does not fit this batch");
    if (mode == kWave && !wave_fit) return bail(SSA_ESHAPE, "wave mode does not fit this batch");
    if (mode == 0) {
        if (all_spec_fit && max_M <= kSpecAutoMaxChannels) mode = kSpec;
        else if (all_lane_fit && nn <= 64) mode = kLane;
        else if (wave_fit) mode = kWave;
        else if (all_lane_fit) mode = kLane;
        else return bail(SSA_ESHAPE, "no execution mode fits this batch (at most 64 species and 511 channels)");
    }
    net->tangent_fit = mode == kSpec && max_M <= kTanMaxChannels;
    for (int n = 0; n < nn && net->tangent_fit; ++n)
        if ((int64_t)d->n_species[n] * d->n_reactions[n] > kTanMaxStateTangents) net->tangent_fit = false;
    if (mode == kSpec) {
        for (auto &kv : spec_kernels) {
            std::string log;
            if (!spec_compile(kv.first, &kv.second, &log)) return bail(SSA_EHIP, log);
        }
    }
    const int wave_cls = mode == kWave ? wave_class_for(max_M, wave_lanes) : -1;
    // wave mode: one persistent launch for the whole batch, or one per
    // lane-group width with each network in the narrowest group that fits it
    // (the library's choice: one launch per width, which keeps lanes busy)
    const bool wave_split = d->wave_split != 0;

    // ---- device tables ---------------------------------------------------
    std::vector<ReactDesc> rd;
    std::vector<uint32_t> rows;
    std::vector<int32_t> csr, obs_sp, pmap_off, pmap_ch, param_net, inc_ptr, chan_inc;
    std::vector<LaneItem> items[kLaneClassCount];
    std::map<int, std::vector<LaneItem>> wave_items;   // by wave class
    std::vector<int> net_nnz, net_ve;
    std::map<std::string, std::vector<LaneItem>> spec_items;
    int64_t roff = 0, soff = 0, ooff = 0;
    for (int n = 0; n < nn; ++n) {
        const int N = d->n_species[n], M = d->n_reactions[n], P = d->n_params[n], B = d->n_traj[n];
        const int nob = d->n_obs[n];
        const int cls = mode == kLane ? lane_class_for(N, M) : -1;
        NetDev nd;
        std::memset(&nd, 0, sizeof(nd));
        nd.N = N; nd.M = M; nd.P = P; nd.n_obs = nob; nd.B = B;
        const int nmax = mode == kLane ? lane_class_nmax(cls) : N;
        nd.wpr = (nmax + 7) / 8;
        nd.react_off = (int32_t)rd.size();
        nd.rows_off = (int32_t)rows.size();
        nd.obs_sp_off = (int32_t)obs_sp.size();
        nd.mode = mode == kLane ? cls : mode == kSpec ? -1 : -2;
        nd.inc_off = (int32_t)inc_ptr.size();
        nd.traj_off = net->traj_total;
        nd.state_off = net->state_total;
        nd.param_off = net->param_total;
        nd.obsb_off = net->obsb_total;
        nd.obsw_off = net->obsw_total;
        nd.tobs_off = net->tobs_total;
        nd.obst_off = net->obst_total;
        nd.obstw_off = net->obstw_total;
        nd.tanw_off = net->tanw_total;
        nd.part_off = net->part_total;
        nd.ppt_off = net->ppt_total;
        nd.t_obs = d->t_obs ? d->t_obs[n] : 0.0;
        std::vector<std::vector<int32_t>> incid(N);
        int max_ve = 0;
        for (int j = 0; j < M; ++j) {
            const int s1 = d->reactant[2 * (roff + j)], s2 = d->reactant[2 * (roff + j) + 1];
            ReactDesc r;
            std::memset(&r, 0, sizeof(r));
            r.s1 = (uint8_t)(s1 < 0 ? kNoSpecies : s1);
            r.s2 = (uint8_t)(s2 < 0 ? kNoSpecies : s2);
            r.homodimer = (uint8_t)(s1 >= 0 && s1 == s2);
            r.rate = d->rate_index[roff + j];
            r.mult = r.homodimer ? 0.5f : 1.0f;
            const int beg = (int)csr.size();
            std::vector<uint32_t> packed(nd.wpr, 0u);
            for (int q = 0; q < N; ++q) {
                const int v = d->stoich[soff + (int64_t)j * N + q];
                if (v != 0) {
                    csr.push_back((int32_t)((uint32_t)q | ((uint32_t)(v & 0xFFFF) << 16)));
                    if (q < nmax) packed[q / 8] |= (uint32_t)(v & 0xF) << (4 * (q % 8));
                }
            }
            r.csr = beg | (((int)csr.size() - beg) << 24);
            rd.push_back(r);
            rows.insert(rows.end(), packed.begin(), packed.end());
            // channel j contributes coef*A2 to dlambda[s1] (role 1) and coef*A1 to dlambda[s2] (role 2)
            if (s1 >= 0) incid[s1].push_back(j | (1 << 16));
            if (s2 >= 0) incid[s2].push_back(j | (2 << 16));
            max_ve = std::max(max_ve, (int)csr.size() - beg);
        }
        // incidence slots grouped by species; each channel keeps its two slots
        std::vector<int32_t> pos(2 * (size_t)M, 0xFFFF);
        int slot = 0;
        for (int q = 0; q < N; ++q) {
            inc_ptr.push_back(slot);
            for (int32_t ent : incid[q]) pos[2 * (ent & 0xFFFF) + ((ent >> 16) - 1)] = slot++;
        }
        inc_ptr.push_back(slot);
        for (int j = 0; j < M; ++j) chan_inc.push_back(pos[2 * j] | (pos[2 * j + 1] << 16));
        net_nnz.push_back((int)(csr.size() - (rd[nd.react_off].csr & 0xFFFFFF)));
        net_ve.push_back(max_ve);
        for (int o = 0; o < nob; ++o) obs_sp.push_back(d->obs_species[ooff + o]);
        // parameter -> channels map for the gradient reduction
        for (int pp = 0; pp < P; ++pp) {
            pmap_off.push_back((int32_t)pmap_ch.size());
            for (int j = 0; j < M; ++j)
                if (d->rate_index[roff + j] == pp) pmap_ch.push_back(j);
            param_net.push_back(n);
        }
        if (mode == kWave) {
            const int wc = wave_split ? wave_class_for(M, wave_lanes) : wave_cls;
            for (int i = 0; i < B; ++i) {
                LaneItem it;
                it.net = n; it.first = i; it.count = 1; it.pad = M;
                wave_items[wc].push_back(it);
            }
        } else {
            for (int first = 0; first < B; first += 64) {
                LaneItem it;
                it.net = n; it.first = first; it.count = std::min(64, B - first); it.pad = M;
                if (mode == kSpec) spec_items[srcs[n]].push_back(it);
                else items[cls].push_back(it);
            }
        }
        net->traj_total += B;
        net->state_total += (int64_t)N * B;
        net->param_total += P;
        net->obsb_total += (int64_t)nob * B;
        net->obsw_total += nob;
        net->tobs_total += (int64_t)((B + 63) / 64) * nob;
        net->obst_total += (int64_t)(nob + 1) * B;
        net->obstw_total += nob + 1;
        net->tanw_total += (int64_t)nob * M * B;
        net->part_total += (int64_t)M * B;
        net->ppt_total += (int64_t)P * B;
        net->max_M = std::max(net->max_M, M);
        net->max_B = std::max<int64_t>(net->max_B, B);
        net->nets_h.push_back(nd);
        roff += M;
        soff += (int64_t)M * N;
        ooff += nob;
    }
    pmap_off.push_back((int32_t)pmap_ch.size());
    if (net->traj_total > 0x7FFFFFFFll) return bail(SSA_ESHAPE, "too many trajectories");
    // longest work first (channels are the per-step cost)
    auto by_cost = [](const LaneItem &a, const LaneItem &b) { return a.pad > b.pad; };
    for (auto &kv : spec_items) std::stable_sort(kv.second.begin(), kv.second.end(), by_cost);
    for (auto &v : items) std::stable_sort(v.begin(), v.end(), by_cost);
    for (auto &kv : wave_items) std::stable_sort(kv.second.begin(), kv.second.end(), by_cost);

    hipError_t e = hipGetDevice(&net->device);
    if (e == hipSuccess) e = static_scratch(net->device, &net->scratch);
    if (e == hipSuccess) e = upload(&net->nets_d, net->nets_h);
    if (e == hipSuccess) e = upload(&net->rd_d, rd);
    if (e == hipSuccess) e = upload(&net->rows_d, rows);
    if (e == hipSuccess) e = upload(&net->csr_d, csr.empty() ? std::vector<int32_t>{0} : csr);
    if (e == hipSuccess) e = upload(&net->obs_sp_d, obs_sp.empty() ? std::vector<int32_t>{0} : obs_sp);
    if (e == hipSuccess) e = upload(&net->pmap_off_d, pmap_off);
    if (e == hipSuccess) e = upload(&net->pmap_ch_d, pmap_ch.empty() ? std::vector<int32_t>{0} : pmap_ch);
    if (e == hipSuccess) e = upload(&net->param_net_d, param_net);
    if (e == hipSuccess) e = upload(&net->inc_ptr_d, inc_ptr);
    if (e == hipSuccess) e = upload(&net->chan_inc_d, chan_inc.empty() ? std::vector<int32_t>{0} : chan_inc);
    for (auto &kv : spec_items) {
        if (e != hipSuccess) break;
        ssa_net::Group gr;
        gr.spec = true;
        gr.kernels = spec_kernels[kv.first];
        gr.spec_nobs = kv.second.empty() ? 0 : d->n_obs[kv.second.front().net];
        gr.n_items = (int)kv.second.size();
        e = upload(&gr.items_d, kv.second);
        net->groups.push_back(gr);
    }
    for (int c = 0; c < kLaneClassCount && e == hipSuccess; ++c) {
        if (items[c].empty()) continue;
        ssa_net::Group gr;
        gr.lane_class = c;
        gr.n_items = (int)items[c].size();
        e = upload(&gr.items_d, items[c]);
        net->groups.push_back(gr);
    }
    for (auto &kv : wave_items) {
        if (e != hipSuccess) break;
        ssa_net::Group gr;
        gr.wave_class = kv.first;
        gr.n_items = (int)kv.second.size();
        for (const LaneItem &it : kv.second) {
            gr.tab_m = std::max(gr.tab_m, d->n_reactions[it.net]);
            gr.tab_nnz = std::max(gr.tab_nnz, net_nnz[it.net]);
            if (net_ve[it.net] > kVecSlots) gr.wide_ve = 1;
        }
        const int per_wave = 64 / wave_class_lanes(gr.wave_class);
        const size_t tab_bytes = sizeof(int32_t) * (size_t)(gr.tab_m + gr.tab_nnz + kWaveMaxSpecies + 1);
        const size_t lds = std::max(wave_static_lds(gr.wave_class, true), wave_static_lds(gr.wave_class, false)) +
                           tab_bytes * 4 * per_wave;
        if (lds > kLdsPerBlock)
            return bail(SSA_ESHAPE, "network tables do not fit the LDS of a wave-mode block");
        const int64_t blocks_needed = ((int64_t)gr.n_items + 4 * per_wave - 1) / (4 * per_wave);
        gr.wave_blocks = (int)std::min<int64_t>(blocks_needed, 2048);
        e = upload(&gr.items_d, kv.second);
        net->groups.push_back(gr);
    }
    if (e == hipSuccess) e = hipMalloc((void **)&net->flags_d, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(net->flags_d, 0, sizeof(uint32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        ssa_status st = hip_fail(e, "ssa_net_create");
        std::string m = g_last_error;
        ssa_net_destroy(net);
        return fail(st, m);
    }
    *out = net;
    return SSA_OK;
}

void ssa_net_destroy(ssa_net *net)
{
    if (!net) return;
    (void)hipFree(net->nets_d);
    (void)hipFree(net->rd_d);
    (void)hipFree(net->rows_d);
    (void)hipFree(net->csr_d);
    (void)hipFree(net->obs_sp_d);
    (void)hipFree(net->pmap_off_d);
    (void)hipFree(net->pmap_ch_d);
    (void)hipFree(net->param_net_d);
    (void)hipFree(net->inc_ptr_d);
    (void)hipFree(net->chan_inc_d);
    for (auto &gr : net->groups) (void)hipFree(gr.items_d);
    (void)hipFree(net->flags_d);
    delete net;
}

ssa_status ssa_net_sizes(const ssa_net *net, int64_t *n_traj_total, int64_t *state_total,
                         int64_t *param_total, int64_t *n_networks)
{
    if (!net) return fail(SSA_EINVAL, "network handle is NULL");
    if (n_traj_total) *n_traj_total = net->traj_total;
    if (state_total) *state_total = net->state_total;
    if (param_total) *param_total = net->param_total;
    if (n_networks) *n_networks = net->n_networks;
    return SSA_OK;
}

ssa_status ssa_net_layout(const ssa_net *net, int32_t obs_kind, int32_t n_bins, int32_t network,
                          ssa_net_layout_t *out)
{
    if (!net || !out) return fail(SSA_EINVAL, "NULL argument");
    if (network < 0 || network >= net->n_networks) return fail(SSA_EINVAL, "network index out of range");
    const NetDev &nd = net->nets_h[network];
    out->traj_offset = nd.traj_off;
    out->state_offset = nd.state_off;
    out->param_offset = nd.param_off;
    out->obs_offset = obs_block_offset(nd, obs_kind, n_bins);
    out->ppt_offset = nd.ppt_off;
    out->mean_offset = mean_block_offset(nd, obs_kind, n_bins);
    return SSA_OK;
}

ssa_status ssa_buffer_sizes(const ssa_net *net, const ssa_config *cfg, size_t *ckpt_bytes,
                            size_t *work_bytes)
{
    ssa_status s = check_config(net, cfg);
    if (s != SSA_OK) return s;
    if (ckpt_bytes) *ckpt_bytes = ckpt_layout(net, cfg).bytes;
    if (work_bytes) *work_bytes = work_bytes_for(net, cfg);
    return SSA_OK;
}

ssa_status ssa_forward(const ssa_net *net, const ssa_config *cfg, const float *theta, const int32_t *x0,
                       int32_t *x_final, double *t_final, int32_t *steps_done, double *obs, void *ckpt,
                       size_t ckpt_bytes, ssa_tie *ties, uint32_t *n_ties, void *work, size_t work_bytes,
                       hipStream_t stream)
{
    g_last_error.clear();
    ssa_status s = check_config(net, cfg);
    if (s != SSA_OK) return s;
    if (!theta || !x0 || !x_final || !t_final || !steps_done)
        return fail(SSA_EINVAL, "theta, x0, x_final, t_final and steps_done are required");
    if (obs_total(net, cfg) > 0 && !obs) return fail(SSA_EINVAL, "obs is NULL but species are observed");
    if (!work || work_bytes < work_bytes_for(net, cfg)) return fail(SSA_EWORKSPACE, "work buffer too small");
    if ((ties == nullptr) != (n_ties == nullptr)) return fail(SSA_EINVAL, "ties and n_ties go together");
    const CkptLayout L = ckpt_layout(net, cfg);
    if (ckpt && ckpt_bytes < L.bytes) return fail(SSA_EWORKSPACE, "checkpoint buffer too small");
    if (ckpt && L.bytes == 0) return fail(SSA_EINVAL, "checkpoints need a bounded n_steps");

    RunParams p = base_params(net, cfg);
    p.theta = theta;
    p.x0 = x0;
    p.x_final = x_final;
    p.t_final = t_final;
    p.steps_done = steps_done;
    p.obs = obs;
    if (ckpt && cfg->bwd_mode == SSA_BWD_TANGENT) {
        p.tangent = (double *)ckpt;
    } else if (ckpt) {
        char *base = (char *)ckpt;
        p.ck_t = (double *)(base + L.off_t);
        p.ck_x = (int32_t *)(base + L.off_x);
        p.tape = L.tape_words ? (uint32_t *)(base + L.off_tape) : nullptr;
        p.n_ckpt = L.n_ckpt;
        p.tape_bits = L.tape_words ? L.tape_bits : 0;
        p.tape_words = L.tape_words;
    }
    p.work_counter = (uint32_t *)((char *)work + 64);
    p.ties = reinterpret_cast<TieRec *>(ties);
    p.n_ties = n_ties;
    p.tie_cap = (uint32_t)cfg->tie_capacity;
    if (n_ties) {
        hipError_t e = launch_fill_u32(n_ties, 1, 0u, stream);
        if (e != hipSuccess) return hip_fail(e, "clearing the tie counter");
    }
    if (cfg->obs_layout != SSA_OBS_ENSEMBLE_MEAN) return launch_all_classes(net, p, false, stream);
    // ensemble means: the tiles' rows of sums, then each network's rows in order
    p.tile_sums = tile_sums_of(net, cfg, work);
    s = launch_all_classes(net, p, false, stream);
    if (s != SSA_OK) return s;
    double *sums = (double *)((char *)work + grad_work_bytes(net));
    for (const NetDev &nd : net->nets_h) {
        const int64_t W = obs_width(nd, cfg);
        if (W == 0) continue;
        hipError_t e = launch_obs_mean(p.tile_sums + nd.tobs_off * cfg->n_bins, (nd.B + 63) / 64, W, true, sums,
                                       obs + nd.obsw_off * cfg->n_bins, nd.B, stream);
        if (e != hipSuccess) return hip_fail(e, "ensemble mean of the tiles");
    }
    return SSA_OK;
}

static ssa_status backward_impl(const ssa_net *net, const ssa_config *cfg, const float *theta, const int32_t *x0,
                        const int32_t *x_final, const double *t_final, const int32_t *steps_done,
                        const void *ckpt, size_t ckpt_bytes, const double *d_obs, float *d_params,
                        float *d_params_per_traj, void *work, size_t work_bytes, hipStream_t stream)
{
    ssa_status s = check_config(net, cfg);
    if (s == SSA_OK && cfg->selection != SSA_SELECT_GUMBEL_MAX)
        return fail(SSA_ENOTSUP, "the straight-through backward needs the Gumbel-max selection");
    if (s != SSA_OK) return s;
    if (cfg->obs_layout == SSA_OBS_ENSEMBLE_MEAN && !cfg->dobs_shared)
        return fail(SSA_ENOTSUP, "after an ensemble-mean forward the backward needs a shared d_obs");
    if (!theta || !x0 || !x_final || !t_final || !steps_done || !d_params)
        return fail(SSA_EINVAL, "theta, x0, x_final, t_final, steps_done and d_params are required");
    if (obs_total(net, cfg) > 0 && !d_obs) return fail(SSA_EINVAL, "d_obs is NULL but species are observed");
    const CkptLayout L = ckpt_layout(net, cfg);
    if (L.bytes == 0) return fail(SSA_EINVAL, "the backward needs a bounded n_steps");
    if (!ckpt || ckpt_bytes < L.bytes) return fail(SSA_EWORKSPACE, "checkpoint buffer too small");
    if (!work || work_bytes < work_bytes_for(net, cfg)) return fail(SSA_EWORKSPACE, "work buffer too small");

    RunParams p = base_params(net, cfg);
    p.theta = theta;
    p.x0 = x0;
    p.x_final = const_cast<int32_t *>(x_final);
    p.t_final = const_cast<double *>(t_final);
    p.steps_done = const_cast<int32_t *>(steps_done);
    p.d_obs = d_obs;
    p.partials = (double *)((char *)work + kWorkHeader);
    p.work_counter = (uint32_t *)((char *)work + 64);
    double *chunk_sums = (double *)((char *)work + kWorkHeader + partials_bytes(net));
    if (cfg->bwd_mode == SSA_BWD_TANGENT) {
        // the forward's tangents contracted with dL/dobs: no reverse sweep
        const int npts = cfg->obs_kind == SSA_OBS_BINS ? cfg->n_bins : 1;
        hipError_t e = launch_tangent_contract(net->nets_d, net->n_networks, net->traj_total, npts, d_obs,
                                               (const double *)ckpt, p.partials, stream);
        if (e == hipSuccess)
            e = launch_reduce_params(net->nets_d, net->pmap_off_d, net->pmap_ch_d, net->param_net_d, net->param_total,
                                     net->max_B, p.partials, chunk_sums, d_params, d_params_per_traj, stream);
        if (e != hipSuccess) return hip_fail(e, "tangent contraction");
        return SSA_OK;
    }
    const char *base = (const char *)ckpt;
    p.ck_t = (double *)(base + L.off_t);
    p.ck_x = (int32_t *)(base + L.off_x);
    p.tape = L.tape_words ? (uint32_t *)(base + L.off_tape) : nullptr;
    p.n_ckpt = L.n_ckpt;
    p.tape_bits = L.tape_words ? L.tape_bits : 0;
    p.tape_words = L.tape_words;
    if (prefix_work_bytes(net, cfg) > 0) {
        double *pre = (double *)((char *)work + grad_work_bytes(net) + mean_work_bytes(net, cfg));
        hipError_t e = launch_dobs_prefix(net->nets_d, net->n_networks, cfg->n_bins, d_obs, pre, stream);
        if (e != hipSuccess) return hip_fail(e, "dL/dobs prefix sums");
        p.dobs_prefix = pre;
    }
    s = launch_all_classes(net, p, true, stream);
    if (s != SSA_OK) return s;
    hipError_t e = launch_reduce_params(net->nets_d, net->pmap_off_d, net->pmap_ch_d, net->param_net_d,
                                        net->param_total, net->max_B, p.partials, chunk_sums, d_params,
                                        d_params_per_traj, stream);
    if (e != hipSuccess) return hip_fail(e, "gradient reduction");
    return SSA_OK;
}

ssa_status ssa_backward(const ssa_net *net, const ssa_config *cfg, const float *theta, const int32_t *x0,
                        const int32_t *x_final, const double *t_final, const int32_t *steps_done,
                        const void *ckpt, size_t ckpt_bytes, const double *d_obs, float *d_params,
                        float *d_params_per_traj, void *work, size_t work_bytes, hipStream_t stream)
{
    g_last_error.clear();
    return backward_impl(net, cfg, theta, x0, x_final, t_final, steps_done, ckpt, ckpt_bytes, d_obs, d_params,
                         d_params_per_traj, work, work_bytes, stream);
}

ssa_status ssa_backward_static(const ssa_net *net, const ssa_config *cfg, const float *theta, const int32_t *x0,
                               const int32_t *x_final, const double *t_final, const int32_t *steps_done,
                               const void *ckpt, size_t ckpt_bytes, const double *d_obs, float *d_params,
                               float *d_params_per_traj, hipStream_t stream)
{
    g_last_error.clear();
    ssa_status s = check_config(net, cfg);
    if (s != SSA_OK) return s;
    if (!net->scratch) return fail(SSA_EHIP, "the static scratch of this device was not resolved");
    const size_t need = work_bytes_for(net, cfg);
    if (need > kStaticScratchBytes)
        return fail(SSA_EWORKSPACE, "this backward needs " + std::to_string(need) +
                                        " bytes of scratch; the static array holds " +
                                        std::to_string(kStaticScratchBytes));
    return backward_impl(net, cfg, theta, x0, x_final, t_final, steps_done, ckpt, ckpt_bytes, d_obs, d_params,
                         d_params_per_traj, net->scratch, kStaticScratchBytes, stream);
}

ssa_status ssa_obs_mean(const ssa_net *net, const ssa_config *cfg, const double *obs, double *mean,
                        void *work, size_t work_bytes, hipStream_t stream)
{
    g_last_error.clear();
    ssa_status s = check_config(net, cfg);
    if (s != SSA_OK) return s;
    if (cfg->obs_layout == SSA_OBS_ENSEMBLE_MEAN)
        return fail(SSA_EINVAL, "ensemble-mean observations are means already");
    if (obs_total(net, cfg) > 0 && (!obs || !mean)) return fail(SSA_EINVAL, "obs and mean are required");
    if (!work || work_bytes < work_bytes_for(net, cfg)) return fail(SSA_EWORKSPACE, "work buffer too small");
    double *sums = (double *)((char *)work + grad_work_bytes(net));
    for (const NetDev &nd : net->nets_h) {
        const int64_t W = obs_width(nd, cfg);
        if (W == 0) continue;
        hipError_t e = launch_obs_mean(obs + obs_block_offset(nd, cfg->obs_kind, cfg->n_bins), nd.B, W,
                                       cfg->obs_layout == SSA_OBS_TRAJ_MAJOR, sums,
                                       mean + mean_block_offset(nd, cfg->obs_kind, cfg->n_bins), nd.B, stream);
        if (e != hipSuccess) return hip_fail(e, "ensemble mean");
    }
    return SSA_OK;
}

ssa_status ssa_step_batch(const ssa_net *net, const ssa_config *cfg, const float *theta, int32_t *x,
                          double *t, uint32_t step, int32_t *chosen, float *tau, float *a, hipStream_t stream)
{
    g_last_error.clear();
    ssa_status s = check_config(net, cfg);
    if (s != SSA_OK) return s;
    if (cfg->selection != SSA_SELECT_GUMBEL_MAX) return fail(SSA_ENOTSUP, "ssa_step_batch runs the Gumbel-max selection");
    if (!theta || !x || !t || !chosen || !tau) return fail(SSA_EINVAL, "theta, x, t, chosen, tau are required");
    RunParams p = base_params(net, cfg);
    p.theta = theta;
    hipError_t e = launch_step_batch(p, net->n_networks, step, x, t, chosen, tau, a, stream);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    return SSA_OK;
}

ssa_status ssa_device_status(const ssa_net *net, hipStream_t stream, uint32_t *flags)
{
    if (!net || !flags) return fail(SSA_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(flags, net->flags_d, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "reading device flags");
    if (*flags & kFlagOverflow) return fail(SSA_EOVERFLOW, "copy number overflow on the device");
    if (*flags & kFlagNonFinite) return fail(SSA_ENONFINITE, "non-finite propensity or clock on the device");
    return SSA_OK;
}

ssa_status ssa_selftest_philox(const uint32_t *ctr_key, uint32_t *out, int64_t n, hipStream_t stream)
{
    if (n < 0 || (n > 0 && (!ctr_key || !out))) return fail(SSA_EINVAL, "bad arguments");
    hipError_t e = launch_selftest_philox(ctr_key, out, n, stream);
    return e == hipSuccess ? SSA_OK : hip_fail(e, "philox self-test");
}

ssa_status ssa_selftest_neglog(uint32_t first, int64_t count, float *out, hipStream_t stream)
{
    if (count < 0 || (count > 0 && !out) || (int64_t)first + count > (1ll << 23))
        return fail(SSA_EINVAL, "lattice range is [0, 2^23)");
    hipError_t e = launch_selftest_neglog(first, count, out, stream);
    return e == hipSuccess ? SSA_OK : hip_fail(e, "-ln self-test");
}

}  // extern "C"
