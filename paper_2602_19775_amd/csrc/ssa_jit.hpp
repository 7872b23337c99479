// Plan-time compiled lane kernels specialised to one network topology.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "ssa_plan.hpp"

namespace ssa {

constexpr int spec_waves_per_block = 4;   // matches spec::kWaves

struct SpecKernels {
    hipModule_t module = nullptr;
    hipFunction_t fwd = nullptr;        // final and bin observations
    hipFunction_t bwd = nullptr;
    hipFunction_t fwd_grid = nullptr;   // grid observation
    hipFunction_t bwd_grid = nullptr;
    hipFunction_t fwd_cdf = nullptr;    // inverse-CDF selection (forward only)
    hipFunction_t fwd_tm = nullptr;     // bin observation, trajectory-major layout
    hipFunction_t bwd_sh = nullptr;     // bin observation, shared dL/dobs (prefix sums)
    hipFunction_t fwd_ens = nullptr;    // bin observation, ensemble means only (LDS tile sums)
    hipFunction_t fwd_grid_ens = nullptr;   // grid observation, ensemble means only
    hipFunction_t fwd_tan = nullptr;    // final and bin observations with forward-mode tangents
};

// Source of the specialised kernel pair for one network (host tables).
std::string spec_source(int N, int M, const int32_t *reactant, const int32_t *rate_index,
                        const int8_t *stoich, int n_obs, const int32_t *obs_species);
// Compiles (or fetches from the in-process cache) the module for `src`.
bool spec_compile(const std::string &src, SpecKernels *out, std::string *log);
hipError_t spec_launch(const SpecKernels &k, const RunParams &p, bool backward, size_t dyn_lds,
                       hipStream_t stream);

}  // namespace ssa
