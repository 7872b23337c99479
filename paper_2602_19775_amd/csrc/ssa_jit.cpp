// Plan-time specialisation of the lane-mode kernels to a network topology:
// the channel tables become compile-time constants of a small type that the
// kernel bodies in ssa_spec_body.hpp are instantiated with, compiled for the
// current device with hipRTC.  Identical topologies share one module.
#include "ssa_jit.hpp"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace ssa {

// Header texts compiled into the library (generated at build time).
extern const int kEmbeddedCount;
extern const char *const kEmbeddedNames[];
extern const char *const kEmbeddedSources[];

namespace {

std::mutex g_mu;
std::map<std::string, SpecKernels> g_cache;

std::string hex_float(float f)
{
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%a", (double)f);
    return std::string(buf) + "f";
}

}  // namespace

std::string spec_source(int N, int M, const int32_t *reactant, const int32_t *rate_index,
                        const int8_t *stoich, int n_obs, const int32_t *obs_species)
{
    std::ostringstream s;
    s << "#include \"ssa_spec_body.hpp\"\n";
    s << "struct Net {\n";
    s << "  static constexpr int N = " << N << ", M = " << M << ", NOBS = " << n_obs << ";\n";
    auto arr = [&](const char *name, auto get) {
        s << "  static constexpr int " << name << "[" << M << "] = {";
        for (int j = 0; j < M; ++j) s << (j ? ", " : "") << get(j);
        s << "};\n";
    };
    arr("S1", [&](int j) { return reactant[2 * j] < 0 ? N : reactant[2 * j]; });
    arr("S2", [&](int j) { return reactant[2 * j + 1] < 0 ? N : reactant[2 * j + 1]; });
    arr("HOMO", [&](int j) { return (reactant[2 * j] >= 0 && reactant[2 * j] == reactant[2 * j + 1]) ? 1 : 0; });
    arr("RATE", [&](int j) { return rate_index[j]; });
    s << "  static constexpr float MULT[" << M << "] = {";
    for (int j = 0; j < M; ++j) {
        const bool homo = reactant[2 * j] >= 0 && reactant[2 * j] == reactant[2 * j + 1];
        s << (j ? ", " : "") << hex_float(homo ? 0.5f : 1.0f);
    }
    s << "};\n";
    s << "  static constexpr int V[" << M << "][" << N << "] = {";
    for (int j = 0; j < M; ++j) {
        s << (j ? ", " : "") << "{";
        for (int q = 0; q < N; ++q) s << (q ? ", " : "") << (int)stoich[(size_t)j * N + q];
        s << "}";
    }
    s << "};\n";
    s << "  static constexpr int OBS[" << (n_obs > 0 ? n_obs : 1) << "] = {";
    if (n_obs == 0) s << "0";
    for (int o = 0; o < n_obs; ++o) s << (o ? ", " : "") << obs_species[o];
    s << "};\n};\n";
    // one kernel pair for the final and bin observations, one for the grid
    for (const char *g : {"false", "true"}) {
        const std::string sfx = std::string(g) == "true" ? "_grid" : "";
        s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_fwd" << sfx
          << "(ssa::RunParams p) { ssa::spec::forward<Net, " << g << ">(p); }\n";
        s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_bwd" << sfx
          << "(ssa::RunParams p) { ssa::spec::backward<Net, " << g << ">(p); }\n";
    }
    // the forward with the inverse-CDF selection (final and bin observations)
    // the backward of bin observations with a shared dL/dobs block
    s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_bwd_sh"
         "(ssa::RunParams p) { ssa::spec::backward<Net, false, true>(p); }\n";
    // the forwards of bin and grid observations that keep only the ensemble means
    s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_fwd_ens"
         "(ssa::RunParams p) { ssa::spec::forward<Net, false, false, true, true>(p); }\n";
    s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_fwd_grid_ens"
         "(ssa::RunParams p) { ssa::spec::forward<Net, true, false, false, true>(p); }\n";
    // the forward of bin observations in the trajectory-major layout
    s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_fwd_tm"
         "(ssa::RunParams p) { ssa::spec::forward<Net, false, false, true>(p); }\n";
    s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_fwd_cdf"
         "(ssa::RunParams p) { ssa::spec::forward<Net, false, true>(p); }\n";
    // the forward with forward-mode tangents (an empty kernel for a network
    // with more channels than the tangents carry)
    s << "extern \"C\" __global__ void __launch_bounds__(ssa::spec::kBlock) ssa_spec_fwd_tan"
         "(ssa::RunParams p) { ssa::spec::forward_tangent<Net>(p); }\n";
    return s.str();
}

bool spec_compile(const std::string &src, SpecKernels *out, std::string *log)
{
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(src);
    if (it != g_cache.end()) {
        *out = it->second;
        return true;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        *log = "no HIP device for runtime compilation";
        return false;
    }
    std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
    const std::string::size_type colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "ssa_spec.hip", kEmbeddedCount, kEmbeddedSources,
                            kEmbeddedNames) != HIPRTC_SUCCESS) {
        *log = "hiprtcCreateProgram failed";
        return false;
    }
    const char *opts[] = {arch.c_str(), "-O3", "-std=c++17",
                          // no packed FP32 instructions
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    size_t log_size = 0;
    hiprtcGetProgramLogSize(prog, &log_size);
    std::string lg(log_size, '\0');
    if (log_size) hiprtcGetProgramLog(prog, &lg[0]);
    if (rc != HIPRTC_SUCCESS) {
        *log = "runtime compilation failed: " + lg;
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t code_size = 0;
    hiprtcGetCodeSize(prog, &code_size);
    std::vector<char> code(code_size);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    SpecKernels k;
    if (hipModuleLoadData(&k.module, code.data()) != hipSuccess ||
        hipModuleGetFunction(&k.fwd, k.module, "ssa_spec_fwd") != hipSuccess ||
        hipModuleGetFunction(&k.bwd, k.module, "ssa_spec_bwd") != hipSuccess ||
        hipModuleGetFunction(&k.fwd_grid, k.module, "ssa_spec_fwd_grid") != hipSuccess ||
        hipModuleGetFunction(&k.bwd_grid, k.module, "ssa_spec_bwd_grid") != hipSuccess ||
        hipModuleGetFunction(&k.fwd_cdf, k.module, "ssa_spec_fwd_cdf") != hipSuccess ||
        hipModuleGetFunction(&k.fwd_tm, k.module, "ssa_spec_fwd_tm") != hipSuccess ||
        hipModuleGetFunction(&k.bwd_sh, k.module, "ssa_spec_bwd_sh") != hipSuccess ||
        hipModuleGetFunction(&k.fwd_ens, k.module, "ssa_spec_fwd_ens") != hipSuccess ||
        hipModuleGetFunction(&k.fwd_grid_ens, k.module, "ssa_spec_fwd_grid_ens") != hipSuccess ||
        hipModuleGetFunction(&k.fwd_tan, k.module, "ssa_spec_fwd_tan") != hipSuccess) {
        *log = "loading the compiled module failed";
        return false;
    }
    g_cache[src] = k;
    *out = k;
    return true;
}

hipError_t spec_launch(const SpecKernels &k, const RunParams &p, bool backward, size_t dyn_lds,
                       hipStream_t stream)
{
    const unsigned blocks = (unsigned)((p.n_items + spec_waves_per_block - 1) / spec_waves_per_block);
    if (blocks == 0) return hipSuccess;
    RunParams copy = p;
    void *args[] = {&copy};
    const bool grid = p.obs_kind == 2;
    hipFunction_t f = backward ? (grid ? k.bwd_grid : p.dobs_prefix ? k.bwd_sh : k.bwd)
                               : (p.tangent ? k.fwd_tan
                                  : p.selection == 1 ? k.fwd_cdf
                                  : grid           ? (p.obs_ens ? k.fwd_grid_ens : k.fwd_grid)
                                  : p.obs_ens      ? k.fwd_ens
                                  : p.obs_tm && p.obs_kind == 1 ? k.fwd_tm
                                                   : k.fwd);
    return hipModuleLaunchKernel(f, blocks, 1, 1, 64 * spec_waves_per_block, 1, 1, (unsigned)dyn_lds, stream, args,
                                 nullptr);
}

}  // namespace ssa
