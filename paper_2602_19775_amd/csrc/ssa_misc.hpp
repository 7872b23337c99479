// Launchers of the auxiliary kernels (ssa_misc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "ssa_plan.hpp"

namespace ssa {

hipError_t launch_step_batch(const RunParams &p, int n_networks, uint32_t step, int32_t *x, double *t,
                             int32_t *chosen, float *tau, float *a, hipStream_t stream);
// Deterministic gradient reduction in two passes (chunks of trajectories in a
// fixed tree order, then the chunks in order); chunk_sums holds
// param_total * reduce_chunks(max_traj) doubles.
int reduce_chunks(int64_t max_traj);
hipError_t launch_reduce_params(const NetDev *nets, const int32_t *pmap_off, const int32_t *pmap_ch,
                                const int32_t *param_net, int64_t param_total, int64_t max_traj,
                                const double *partials, double *chunk_sums, float *d_params, float *d_ppt,
                                hipStream_t stream);
// Ensemble mean of one network's observation block (B rows, W values each;
// traj_major: [B][W], else [W][B]): FP64 sums over chunks of rows, then over
// the chunks in index order, divided by `divisor` into mean[W].  sums holds
// obs_mean_chunks(B) * W doubles.
int obs_mean_chunks(int64_t B);
hipError_t launch_obs_mean(const double *obs, int64_t B, int64_t W, bool traj_major, double *sums,
                           double *mean, int64_t divisor, hipStream_t stream);
// Prefix sums [obs][n_bins + 1] per network of a shared bin dL/dobs block
// (networks at obsw_off * n_bins in d_obs, at obsw_off * (n_bins + 1) in pre).
hipError_t launch_dobs_prefix(const NetDev *nets, int n_networks, int n_bins, const double *d_obs, double *pre,
                              hipStream_t stream);
// Per-channel FP64 gradient partials [M][B] per network from forward-mode
// tangents ([point][obs][channel][B] at tanw_off * npts) and a per-trajectory
// dL/dobs (point-major).
hipError_t launch_tangent_contract(const NetDev *nets, int n_networks, int64_t traj_total, int npts,
                                   const double *d_obs, const double *tangent, double *partials, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_selftest_philox(const uint32_t *ck, uint32_t *out, int64_t n, hipStream_t stream);
hipError_t launch_selftest_neglog(uint32_t first, int64_t count, float *out, hipStream_t stream);

}  // namespace ssa
