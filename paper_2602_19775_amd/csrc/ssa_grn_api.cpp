// C ABI of the gene-regulatory network classifier (declared in include/ssa.h):
// argument checks, buffer layout and kernel launches.  ssa_grn_forward and
// ssa_grn_backward never allocate, free or synchronise.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "ssa.h"
#include "ssa_grn.hpp"
#include "ssa_host.hpp"
#include "ssa_misc.hpp"

using namespace ssa;

struct ssa_grn {
    ssa_grn_desc d;
    int64_t B = 0;
    int64_t P = 0;
    int32_t C = 0;
    uint32_t *flags_d = nullptr;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x)
{
    return (x + kAlign - 1) / kAlign * kAlign;
}

ssa_status check_cfg(const ssa_grn *g, const ssa_config *cfg)
{
    if (!g) return fail(SSA_EINVAL, "GRN handle is NULL");
    if (!cfg) return fail(SSA_EINVAL, "config is NULL");
    if (cfg->n_steps < 0) return fail(SSA_EINVAL, "n_steps must be >= 0");
    if (!(cfg->t_end > 0.0)) return fail(SSA_EINVAL, "t_end must be > 0");
    if (cfg->t_end != INFINITY) return fail(SSA_ENOTSUP, "GRN runs stop after n_steps only (t_end must be INFINITY)");
    if (cfg->obs_kind != SSA_OBS_FINAL) return fail(SSA_ENOTSUP, "GRN runs observe the final output counts only");
    if (cfg->obs_layout != SSA_OBS_POINT_MAJOR || cfg->dobs_shared)
        return fail(SSA_ENOTSUP, "GRN runs use the point-major observation layout");
    if (!(cfg->temperature > 0.f) || !std::isfinite(cfg->temperature))
        return fail(SSA_EINVAL, "temperature must be finite and > 0");
    if (cfg->tie_capacity < 0) return fail(SSA_EINVAL, "tie_capacity must be >= 0");
    if (cfg->relaxed != 0 && cfg->relaxed != 1) return fail(SSA_EINVAL, "relaxed must be 0 or 1");
    if (cfg->relaxed && cfg->selection != SSA_SELECT_GUMBEL_MAX)
        return fail(SSA_ENOTSUP, "the relaxed forward takes the Gumbel-Softmax sample (selection must be Gumbel-max)");
    return SSA_OK;
}

size_t tape_words(const ssa_config *cfg)
{
    return (size_t)64 * (size_t)(((int64_t)cfg->n_steps + 127) / 128);
}

// Relaxed runs store the starting point of every step instead of the fired
// channels: (n_steps + 1) rows of kHid + 2 kMaxOut floats per trajectory.
constexpr size_t kSoftRowFloats = grn::kHid + 2 * grn::kMaxOut;

size_t tape_bytes_for(const ssa_grn *g, const ssa_config *cfg)
{
    if (cfg->relaxed)
        return align_up(sizeof(float) * kSoftRowFloats * ((size_t)cfg->n_steps + 1) * (size_t)g->B);
    return align_up(sizeof(uint32_t) * tape_words(cfg) * (size_t)g->B);
}

// Backward scratch: per-trajectory partials [B][C], per-image sums
// [n_images][C] (FP64), and dL/dv_o of every step [B][n_steps][n_out] (FP32).
size_t work_bytes_for(const ssa_grn *g, const ssa_config *cfg)
{
    return align_up(sizeof(double) * (size_t)g->B * g->C) +
           align_up(sizeof(double) * (size_t)g->d.n_images * g->C) +
           align_up(sizeof(float) * (size_t)g->B * (size_t)cfg->n_steps * g->d.n_out);
}

grn::GrnParams base_params(const ssa_grn *g, const ssa_config *cfg, const float *theta, const float *x_img)
{
    grn::GrnParams p{};
    const int64_t I = g->d.n_in, H = grn::kHid, O = g->d.n_out;
    p.n_in = g->d.n_in;
    p.n_out = g->d.n_out;
    p.n_images = g->d.n_images;
    p.n_rep = g->d.n_rep;
    p.B = g->B;
    p.beta = g->d.beta;
    p.delta_min = g->d.delta_min;
    p.theta = theta;
    p.off_b = H * I;
    p.off_U = p.off_b + H;
    p.off_c = p.off_U + O * H;
    p.off_psi = p.off_c + O;
    p.x_img = x_img;
    p.tape_words = (int32_t)tape_words(cfg);
    p.relaxed = cfg->relaxed;
    p.flags = g->flags_d;
    p.seed_lo = (uint32_t)cfg->seed;
    p.seed_hi = (uint32_t)(cfg->seed >> 32);
    p.purpose = cfg->purpose;
    p.epoch = cfg->epoch;
    p.d_epoch = cfg->d_epoch;
    p.traj_ids = cfg->traj_ids;
    p.n_steps = cfg->n_steps;
    p.temperature = cfg->temperature;
    p.d_temperature = cfg->d_temperature;
    p.C = g->C;
    return p;
}

}  // namespace

extern "C" {

ssa_status ssa_grn_create(const ssa_grn_desc *d, ssa_grn **out)
{
    g_last_error.clear();
    if (!d || !out) return fail(SSA_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->n_hid != grn::kHid) return fail(SSA_ESHAPE, "this build runs networks with 256 hidden genes");
    if (d->n_out < 1 || d->n_out > grn::kMaxOut) return fail(SSA_ESHAPE, "n_out must be in [1, 16]");
    if (d->n_in < 1) return fail(SSA_EINVAL, "n_in must be >= 1");
    if (d->n_images < 1 || d->n_rep < 1) return fail(SSA_EINVAL, "n_images and n_rep must be >= 1");
    if ((int64_t)d->n_images * d->n_rep > (int64_t)INT32_MAX)
        return fail(SSA_ESHAPE, "too many trajectories");
    if (!(d->beta > 0.f) || !std::isfinite(d->beta)) return fail(SSA_EINVAL, "beta must be finite and > 0");
    if (!(d->delta_min >= 0.f) || !std::isfinite(d->delta_min)) return fail(SSA_EINVAL, "delta_min must be finite and >= 0");
    ssa_grn *g = new ssa_grn;
    g->d = *d;
    g->B = (int64_t)d->n_images * d->n_rep;
    const int64_t I = d->n_in, H = grn::kHid, O = d->n_out;
    g->P = H * I + H + O * H + O + H + O;
    g->C = (int32_t)(H + O * H + O + H + O);
    hipError_t e = hipMalloc((void **)&g->flags_d, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(g->flags_d, 0, sizeof(uint32_t));
    if (e != hipSuccess) {
        if (g->flags_d) (void)hipFree(g->flags_d);
        delete g;
        return hip_fail(e, "ssa_grn_create");
    }
    *out = g;
    return SSA_OK;
}

void ssa_grn_destroy(ssa_grn *g)
{
    if (!g) return;
    if (g->flags_d) (void)hipFree(g->flags_d);
    delete g;
}

ssa_status ssa_grn_buffer_sizes(const ssa_grn *g, const ssa_config *cfg, size_t *tape_bytes, size_t *work_bytes)
{
    g_last_error.clear();
    ssa_status s = check_cfg(g, cfg);
    if (s != SSA_OK) return s;
    if (tape_bytes) *tape_bytes = tape_bytes_for(g, cfg);
    if (work_bytes) *work_bytes = work_bytes_for(g, cfg);
    return SSA_OK;
}

ssa_status ssa_grn_forward(const ssa_grn *g, const ssa_config *cfg, const float *theta, const float *x_img,
                           const int32_t *x0, float *u_hid, int32_t *x_final, double *t_final,
                           int32_t *steps_done, double *obs, void *tape, size_t tape_bytes, ssa_tie *ties,
                           uint32_t *n_ties, hipStream_t stream)
{
    g_last_error.clear();
    ssa_status s = check_cfg(g, cfg);
    if (s != SSA_OK) return s;
    if (!theta || !x_img || !x0 || !u_hid || !x_final || !t_final || !steps_done || !obs)
        return fail(SSA_EINVAL, "theta, x_img, x0, u_hid, x_final, t_final, steps_done and obs are required");
    if ((ties == nullptr) != (n_ties == nullptr)) return fail(SSA_EINVAL, "ties and n_ties go together");
    if (tape && tape_bytes < tape_bytes_for(g, cfg)) return fail(SSA_EWORKSPACE, "tape buffer too small");
    grn::GrnParams p = base_params(g, cfg, theta, x_img);
    p.u_hid = u_hid;
    p.x0 = x0;
    p.x_final = x_final;
    p.t_final = t_final;
    p.steps_done = steps_done;
    p.obs = obs;
    p.tape = cfg->relaxed ? nullptr : (uint32_t *)tape;
    p.soft = cfg->relaxed ? (float *)tape : nullptr;
    p.ties = cfg->relaxed ? nullptr : reinterpret_cast<TieRec *>(ties);
    p.n_ties = n_ties;
    p.tie_cap = (uint32_t)cfg->tie_capacity;
    hipError_t e = hipSuccess;
    if (n_ties) {
        e = launch_fill_u32(n_ties, 1, 0u, stream);
        if (e != hipSuccess) return hip_fail(e, "clearing the tie counter");
    }
    e = grn::launch_hidden_input(p, stream);
    if (e != hipSuccess) return hip_fail(e, "hidden-input launch");
    e = grn::launch_forward(p, stream);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return SSA_OK;
}

ssa_status ssa_grn_backward(const ssa_grn *g, const ssa_config *cfg, const float *theta, const float *x_img,
                            const int32_t *x0, const float *u_hid, const int32_t *x_final,
                            const int32_t *steps_done,
                            const void *tape, size_t tape_bytes, const double *d_obs, float *d_params,
                            double *d_compact, void *work, size_t work_bytes, hipStream_t stream)
{
    g_last_error.clear();
    ssa_status s = check_cfg(g, cfg);
    if (s != SSA_OK) return s;
    if (!theta || !x_img || !x0 || !u_hid || !x_final || !steps_done || !d_obs || !d_params)
        return fail(SSA_EINVAL, "theta, x_img, x0, u_hid, x_final, steps_done, d_obs and d_params are required");
    if (!tape || tape_bytes < tape_bytes_for(g, cfg)) return fail(SSA_EWORKSPACE, "tape buffer too small");
    if (!work || work_bytes < work_bytes_for(g, cfg)) return fail(SSA_EWORKSPACE, "work buffer too small");
    grn::GrnParams p = base_params(g, cfg, theta, x_img);
    p.u_hid = const_cast<float *>(u_hid);
    p.x0 = x0;
    p.x_final = const_cast<int32_t *>(x_final);
    p.steps_done = const_cast<int32_t *>(steps_done);
    p.tape = cfg->relaxed ? nullptr : (uint32_t *)const_cast<void *>(tape);
    p.soft = cfg->relaxed ? (float *)const_cast<void *>(tape) : nullptr;
    p.d_obs = d_obs;
    char *w = (char *)work;
    p.part = d_compact ? d_compact : (double *)w;
    p.g_img = (double *)(w + align_up(sizeof(double) * (size_t)g->B * g->C));
    p.e_hist = (float *)((char *)p.g_img + align_up(sizeof(double) * (size_t)g->d.n_images * g->C));
    p.d_params = d_params;
    hipError_t e = grn::launch_backward(p, stream);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    e = grn::launch_reduce(p, stream);
    if (e != hipSuccess) return hip_fail(e, "gradient reduction");
    return SSA_OK;
}

ssa_status ssa_grn_device_status(const ssa_grn *g, hipStream_t stream, uint32_t *flags)
{
    if (!g || !flags) return fail(SSA_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(flags, g->flags_d, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "reading device flags");
    if (*flags & kFlagOverflow) return fail(SSA_EOVERFLOW, "copy number overflow on the device");
    if (*flags & kFlagNonFinite) return fail(SSA_ENONFINITE, "non-finite propensity on the device");
    return SSA_OK;
}

}  // extern "C"
