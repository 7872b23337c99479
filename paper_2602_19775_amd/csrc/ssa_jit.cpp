// Plan-time specialisation of the lane-mode kernels to a network topology:
// the channel tables become compile-time constants of a small type that the
// kernel bodies in ssa_spec_body.hpp are instantiated with, compiled for the
// current device with hipRTC.  Identical topologies share one module, and
// code objects are kept on disk for later processes.
#include "ssa_jit.hpp"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
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

namespace {

uint64_t fnv1a(uint64_t h, const std::string &s)
{
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

// Directory of compiled code objects: SSA_JIT_CACHE_DIR if set (empty: no
// cache), else $XDG_CACHE_HOME/ssa_mi355x/jit or $HOME/.cache/ssa_mi355x/jit.
std::string cache_dir()
{
    if (const char *d = std::getenv("SSA_JIT_CACHE_DIR")) return std::string(d);
    std::string base;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) base = x;
    else if (const char *h = std::getenv("HOME")) base = std::string(h) + "/.cache";
    else return "";
    return base + "/ssa_mi355x/jit";
}

bool make_dirs(const std::string &path)
{
    for (size_t i = 1; i <= path.size(); ++i) {
        if (i == path.size() || path[i] == '/') {
            const std::string part = path.substr(0, i);
            if (mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) return false;
        }
    }
    return true;
}

bool read_file(const std::string &path, std::vector<char> *out)
{
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    bool ok = n > 0;
    if (ok) {
        out->resize((size_t)n);
        ok = std::fread(out->data(), 1, (size_t)n, f) == (size_t)n;
    }
    std::fclose(f);
    return ok;
}

void write_file_atomic(const std::string &path, const std::vector<char> &data)
{
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    if (std::fclose(f) == 0 && ok) std::rename(tmp.c_str(), path.c_str());
    else std::remove(tmp.c_str());
}

// The code object of `src`, compiled by hipRTC (which compiles one program at
// a time within a process, so the kernels of a topology share one program).
bool compile_program(const std::string &src, const std::string &arch, std::vector<char> *code, std::string *log)
{
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
    code->resize(code_size);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    if (code_size == 0) {
        *log = "runtime compilation produced no code";
        return false;
    }
    return true;
}

}  // namespace

bool spec_code_object(const std::string &src, const std::string &arch, std::vector<char> *code, std::string *log,
                      bool *from_cache)
{
    if (from_cache) *from_cache = false;
    std::string path, dir = from_cache ? cache_dir() : std::string();
    if (!dir.empty() && make_dirs(dir)) {
        int major = 0, minor = 0;
        hiprtcVersion(&major, &minor);
        uint64_t h = fnv1a(1469598103934665603ull, arch + "|-O3|c++17|no-packed-fp32|hiprtc " +
                                                       std::to_string(major) + "." + std::to_string(minor) + "|");
        for (int e = 0; e < kEmbeddedCount; ++e) h = fnv1a(fnv1a(h, kEmbeddedNames[e]), kEmbeddedSources[e]);
        char name[64];
        std::snprintf(name, sizeof(name), "/%016llx.co", (unsigned long long)fnv1a(h, src));
        path = dir + name;
        if (read_file(path, code)) {
            *from_cache = true;
            return true;
        }
    }
    if (!compile_program(src, arch, code, log)) return false;
    if (!path.empty()) write_file_atomic(path, *code);
    return true;
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
    std::vector<char> code;
    bool from_cache = false;
    if (!spec_code_object(src, arch, &code, log, &from_cache)) return false;

    SpecKernels kn;
    hipError_t e = hipModuleLoadData(&kn.module, code.data());
    if (e != hipSuccess && from_cache) {
        // an unreadable cached object: compile again (and do not store it)
        if (!spec_code_object(src, arch, &code, log, nullptr)) return false;
        e = hipModuleLoadData(&kn.module, code.data());
    }
    if (e != hipSuccess) {
        *log = "loading the compiled module failed";
        return false;
    }
    const char *names[] = {"ssa_spec_fwd", "ssa_spec_bwd", "ssa_spec_fwd_grid", "ssa_spec_bwd_grid",
                           "ssa_spec_fwd_cdf", "ssa_spec_fwd_tm", "ssa_spec_bwd_sh", "ssa_spec_fwd_ens",
                           "ssa_spec_fwd_grid_ens", "ssa_spec_fwd_tan"};
    hipFunction_t *fn[] = {&kn.fwd, &kn.bwd, &kn.fwd_grid, &kn.bwd_grid, &kn.fwd_cdf,
                           &kn.fwd_tm, &kn.bwd_sh, &kn.fwd_ens, &kn.fwd_grid_ens, &kn.fwd_tan};
    for (int k = 0; k < (int)(sizeof(names) / sizeof(names[0])); ++k) {
        if (hipModuleGetFunction(fn[k], kn.module, names[k]) != hipSuccess) {
            *log = std::string("kernel ") + names[k] + " missing from the compiled module";
            (void)hipModuleUnload(kn.module);
            return false;
        }
    }
    g_cache[src] = kn;
    *out = kn;
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
