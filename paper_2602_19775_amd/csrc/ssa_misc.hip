// Small kernels around the simulation: the single-step kernel used for
// step-wise inspection, the deterministic FP64 gradient reduction, counter
// clearing and the self-test entry points of the device primitives.
#include "ssa_device.hpp"
#include "ssa_misc.hpp"

#include <algorithm>

#include <math.h>

namespace ssa {

namespace {

__device__ int find_network(const NetDev *nets, int n_networks, int64_t g)
{
    int lo = 0, hi = n_networks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (nets[mid].traj_off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One direct-method step for every trajectory (one thread each).  Same
// arithmetic as the simulation kernels: a_j = (k_j mult X[s1]) (X[s2] - h),
// tau = E_0 rcp(a0), j = argmin E_j rcp(a_j).
__global__ void step_batch_kernel(RunParams p, int n_networks, uint32_t step, int32_t *x, double *t,
                                  int32_t *chosen, float *tau_out, float *a_out)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= p.traj_total) return;
    const int n = find_network(p.nets, n_networks, g);
    const NetDev nd = p.nets[n];
    const int64_t B = nd.B;
    const int64_t i = g - nd.traj_off;
    const ReactDesc *rd = p.rd + nd.react_off;
    const uint32_t tid = p.traj_ids ? p.traj_ids[g] : (uint32_t)g;
    const uint32_t epoch = p.d_epoch ? *p.d_epoch : p.epoch;
    const uint32_t pe = (p.purpose << 24) | (epoch & 0xFFFFFFu);
    int32_t *xs = x + nd.state_off + i;

    auto xval = [&](int s) -> int { return s == kNoSpecies ? 1 : xs[(int64_t)s * B]; };
    float a0 = 0.f;
    for (int j = 0; j < nd.M; ++j) {
        const ReactDesc r = rd[j];
        const float c = expf(p.theta[nd.param_off + r.rate]) * r.mult;
        const float aj = (c * (float)xval(r.s1)) * (float)(xval(r.s2) - (int)r.homodimer);
        if (a_out) a_out[nd.part_off + (int64_t)j * B + i] = aj;
        a0 += aj;
    }
    if (!(a0 > 0.f)) {
        chosen[g] = -1;
        tau_out[g] = 0.f;
        return;
    }
    Philox::Out blk = Philox::block(0u, step, tid, pe, p.seed_lo, p.seed_hi);
    const float tau = neglog_u(blk.x) * fast_rcp(a0);
    tau_out[g] = tau;
    const double tn = t[g] + (double)tau;
    if (p.t_end < INFINITY && !(tn <= p.t_end)) {
        chosen[g] = -2;
        return;
    }
    float r1 = INFINITY;
    int j1 = 0;
    for (int j = 0; j < nd.M; ++j) {
        const int w = 1 + j;
        if ((w & 3) == 0) blk = Philox::block((uint32_t)(w >> 2), step, tid, pe, p.seed_lo, p.seed_hi);
        const uint32_t word = (w & 3) == 0 ? blk.x : (w & 3) == 1 ? blk.y : (w & 3) == 2 ? blk.z : blk.w;
        const ReactDesc r = rd[j];
        const float c = expf(p.theta[nd.param_off + r.rate]) * r.mult;
        const float aj = (c * (float)xval(r.s1)) * (float)(xval(r.s2) - (int)r.homodimer);
        const float rj = aj > 0.f ? neglog_u(word) * fast_rcp(aj) : INFINITY;
        j1 = rj < r1 ? j : j1;
        r1 = fminf(r1, rj);
    }
    chosen[g] = j1;
    const int beg = rd[j1].csr & 0xFFFFFF, cnt = (int)((uint32_t)rd[j1].csr >> 24);
    for (int e = 0; e < cnt; ++e) {
        const int32_t ent = p.csr[beg + e];
        xs[(int64_t)csr_species(ent) * B] += csr_delta(ent);
    }
    t[g] = tn;
}

// d_params[p] = sum over channels j with rate(j) = p and over trajectories i
// of partials[j][i], summed in a fixed order (thread-strided FP64 sums, then
// a fixed LDS tree), so repeated runs give identical bits.
constexpr int kRedThreads = 256;
constexpr int64_t kRedChunk = 4096;   // trajectories per block of the first reduction pass

// Pass 1: the sum of each parameter's per-trajectory partials over one chunk
// of kRedChunk trajectories (channels sharing a parameter are added first),
// in a fixed tree order; also the per-trajectory gradient if asked for.
__global__ __launch_bounds__(kRedThreads) void reduce_chunks_kernel(
    const NetDev *nets, const int32_t *pmap_off, const int32_t *pmap_ch, const int32_t *param_net,
    const double *partials, int n_chunks, double *chunk_sums, float *d_ppt)
{
    __shared__ double s[kRedThreads];
    const int pg = blockIdx.x;                   // global parameter index
    const int chunk = blockIdx.y;
    const int n = param_net[pg];
    const NetDev nd = nets[n];
    const int pl = (int)(pg - nd.param_off);
    const int64_t B = nd.B;
    const int64_t lo = (int64_t)chunk * kRedChunk, hi = min(B, lo + kRedChunk);
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kRedThreads) {
        double v = 0.0;
        for (int e = pmap_off[pg]; e < pmap_off[pg + 1]; ++e)
            v += partials[nd.part_off + (int64_t)pmap_ch[e] * B + i];
        if (d_ppt) d_ppt[nd.ppt_off + (int64_t)pl * B + i] = (float)v;
        acc += v;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) chunk_sums[(int64_t)pg * n_chunks + chunk] = s[0];
}

// Pass 2: the chunk sums of each parameter, in chunk order.
__global__ __launch_bounds__(256) void reduce_total_kernel(const NetDev *nets, const int32_t *param_net,
                                                           int64_t param_total, int n_chunks,
                                                           const double *chunk_sums, float *d_params)
{
    const int64_t pg = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pg >= param_total) return;
    const int64_t B = nets[param_net[pg]].B;
    const int used = (int)((B + kRedChunk - 1) / kRedChunk);
    double acc = 0.0;
    for (int c = 0; c < used && c < n_chunks; ++c) acc += chunk_sums[pg * n_chunks + c];
    d_params[pg] = (float)acc;
}

// Ensemble means.  Pass 1, trajectory-major blocks [B][W]: thread w of a
// block walks the trajectories of one chunk in order (eight interleaved
// accumulators, combined in a fixed tree), so a wave reads contiguous values.
__global__ __launch_bounds__(64) void mean_sums_tm_kernel(const double *obs, int64_t B, int64_t W, int64_t len,
                                                          double *sums)
{
    const int64_t c = blockIdx.x;
    const int64_t lo = c * len, hi = min(B, lo + len);
    for (int64_t w = (int64_t)blockIdx.y * 64 + threadIdx.x; w < W; w += (int64_t)gridDim.y * 64) {
        const double *q = obs + lo * W + w;
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int64_t i = lo;
        for (; i + 8 <= hi; i += 8, q += 8 * W)
#pragma unroll
            for (int r = 0; r < 8; ++r) a[r] += q[r * W];
        for (int r = 0; i < hi; ++i, ++r, q += W) a[r] += q[0];
        sums[c * W + w] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
}

// Pass 1, point-major blocks [W][B]: one row w per block iteration, the
// threads stride over the chunk's trajectories, then a fixed LDS tree.
__global__ __launch_bounds__(256) void mean_sums_pm_kernel(const double *obs, int64_t B, int64_t W, int64_t len,
                                                           double *sums)
{
    __shared__ double red[256];
    const int64_t c = blockIdx.x;
    const int64_t lo = c * len, hi = min(B, lo + len);
    for (int64_t w = blockIdx.y; w < W; w += gridDim.y) {
        const double *q = obs + w * B;
        double a = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) a += q[i];
        red[threadIdx.x] = a;
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) sums[c * W + w] = red[0];
        __syncthreads();
    }
}

// Pass 2: the chunk sums of each value, divided by B.  Thread (part, w) of a
// block of 64 values sums the chunks c = part (mod 4) with eight interleaved
// accumulators; the four parts are then added in order in LDS.  The loads of
// a thread are independent, so the pass is not a chain of memory latencies.
__global__ __launch_bounds__(256) void mean_total_kernel(const double *sums, int nc, int64_t W, int64_t B,
                                                         double *mean)
{
    __shared__ double part_sum[4][64];
    const int wl = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * 64 + wl;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (w < W) {
        int c = part;
        for (; c + 28 < nc; c += 32)
#pragma unroll
            for (int r = 0; r < 8; ++r) a[r] += sums[(int64_t)(c + 4 * r) * W + w];
        for (int r = 0; c < nc; c += 4, ++r) a[r] += sums[(int64_t)c * W + w];
    }
    part_sum[part][wl] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    if (part == 0 && w < W) {
        const double s = ((part_sum[0][wl] + part_sum[1][wl]) + part_sum[2][wl]) + part_sum[3][wl];
        mean[w] = B > 0 ? s / (double)B : 0.0;
    }
}

// Prefix sums over the bins of a shared dL/dobs block, one block per network:
// pre[o][b] = the sum of d_obs[b'][o] over b' < b, for b <= n_bins.  Each
// chunk of 256 bins is scanned in LDS (a fixed sequence of additions, so the
// result is the same on every call) and carried into the next.
__global__ __launch_bounds__(256) void dobs_prefix_kernel(const NetDev *nets, int n_bins, const double *d_obs,
                                                          double *pre)
{
    __shared__ double buf[256];
    const NetDev nd = nets[blockIdx.x];
    for (int o = 0; o < nd.n_obs; ++o) {
        const double *d = d_obs + nd.obsw_off * n_bins + o;
        double *q = pre + nd.obsw_off * (int64_t)(n_bins + 1) + (int64_t)o * (n_bins + 1);
        double carry = 0.0;
        for (int b0 = 0; b0 < n_bins; b0 += 256) {
            const int b = b0 + (int)threadIdx.x;
            buf[threadIdx.x] = b < n_bins ? d[(int64_t)b * nd.n_obs] : 0.0;
            __syncthreads();
            for (int off = 1; off < 256; off <<= 1) {
                const double a = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0.0;
                __syncthreads();
                buf[threadIdx.x] += a;
                __syncthreads();
            }
            if (b < n_bins) q[b + 1] = carry + buf[threadIdx.x];
            carry += buf[255];
            __syncthreads();
        }
        if (threadIdx.x == 0) q[0] = 0.0;
    }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void selftest_philox_kernel(const uint32_t *ck, uint32_t *out, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const uint32_t *c = ck + 6 * q;
    const Philox::Out o = Philox::block(c[0], c[1], c[2], c[3], c[4], c[5]);
    out[4 * q] = o.x;
    out[4 * q + 1] = o.y;
    out[4 * q + 2] = o.z;
    out[4 * q + 3] = o.w;
}

__global__ void selftest_neglog_kernel(uint32_t first, int64_t count, float *out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const uint32_t m = first + (uint32_t)q;
    out[q] = neglog_u(m << 9);
}

unsigned grid_for(int64_t n, int threads)
{
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

hipError_t launch_step_batch(const RunParams &p, int n_networks, uint32_t step, int32_t *x, double *t,
                             int32_t *chosen, float *tau, float *a, hipStream_t stream)
{
    if (p.traj_total == 0) return hipSuccess;
    hipLaunchKernelGGL(step_batch_kernel, dim3(grid_for(p.traj_total, 256)), dim3(256), 0, stream, p,
                       n_networks, step, x, t, chosen, tau, a);
    return hipGetLastError();
}

int reduce_chunks(int64_t max_traj)
{
    return (int)std::max<int64_t>(1, (max_traj + kRedChunk - 1) / kRedChunk);
}

hipError_t launch_reduce_params(const NetDev *nets, const int32_t *pmap_off, const int32_t *pmap_ch,
                                const int32_t *param_net, int64_t param_total, int64_t max_traj,
                                const double *partials, double *chunk_sums, float *d_params, float *d_ppt,
                                hipStream_t stream)
{
    if (param_total == 0) return hipSuccess;
    const int nc = reduce_chunks(max_traj);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)param_total, (unsigned)nc), dim3(kRedThreads), 0,
                       stream, nets, pmap_off, pmap_ch, param_net, partials, nc, chunk_sums, d_ppt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_total_kernel, dim3((unsigned)((param_total + 255) / 256)), dim3(256), 0, stream,
                       nets, param_net, param_total, nc, chunk_sums, d_params);
    return hipGetLastError();
}

// Trajectories per chunk: a multiple of 64, about 256 chunks for large B.
static int64_t obs_mean_chunk_len(int64_t B)
{
    constexpr int64_t kMeanSplit = 256;
    const int64_t c = (B + kMeanSplit - 1) / kMeanSplit;
    return std::max<int64_t>(64, (c + 63) / 64 * 64);
}

int obs_mean_chunks(int64_t B)
{
    if (B <= 0) return 0;
    const int64_t len = obs_mean_chunk_len(B);
    return (int)((B + len - 1) / len);
}

hipError_t launch_obs_mean(const double *obs, int64_t B, int64_t W, bool traj_major, double *sums,
                           double *mean, int64_t divisor, hipStream_t stream)
{
    if (W <= 0) return hipSuccess;
    const int nc = obs_mean_chunks(B);
    const int64_t len = obs_mean_chunk_len(B);
    if (nc > 0) {
        if (traj_major) {
            const unsigned gy = (unsigned)std::min<int64_t>((W + 63) / 64, 65535);
            hipLaunchKernelGGL(mean_sums_tm_kernel, dim3((unsigned)nc, gy), dim3(64), 0, stream, obs, B, W, len,
                               sums);
        } else {
            const unsigned gy = (unsigned)std::min<int64_t>(W, 65535);
            hipLaunchKernelGGL(mean_sums_pm_kernel, dim3((unsigned)nc, gy), dim3(256), 0, stream, obs, B, W, len,
                               sums);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mean_total_kernel, dim3(grid_for(W, 64)), dim3(256), 0, stream, sums, nc, W, divisor, mean);
    return hipGetLastError();
}

// Per-channel gradient partials of forward-mode tangents: for global
// trajectory g of network n (found by bisection over traj_off),
//   partials[part_off + q B + i] = sum over points pt and observed species o of
//     d_obs[(obsb_off npts) + (pt n_obs + o) B + i] * tangent[(tanw_off npts) + ((pt n_obs + o) M + q) B + i]
// in FP64, in (pt, o) order.
__global__ __launch_bounds__(256) void tangent_contract_kernel(const NetDev *nets, int n_networks, int64_t traj_total,
                                                               int npts, const double *d_obs, const double *tangent,
                                                               double *partials)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= traj_total) return;
    int lo = 0, hi = n_networks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (nets[mid].traj_off <= g) lo = mid;
        else hi = mid - 1;
    }
    const NetDev nd = nets[lo];
    const int64_t B = nd.B, i = g - nd.traj_off;
    const double *dob = d_obs + nd.obsb_off * npts + i;
    const double *tan = tangent + nd.tanw_off * npts + i;
    for (int q = 0; q < nd.M; ++q) {
        double acc = 0.0;
        for (int pt = 0; pt < npts; ++pt)
            for (int o = 0; o < nd.n_obs; ++o) {
                const int64_t r = (int64_t)pt * nd.n_obs + o;
                acc += dob[r * B] * tan[(r * nd.M + q) * B];
            }
        partials[nd.part_off + (int64_t)q * B + i] = acc;
    }
}

hipError_t launch_tangent_contract(const NetDev *nets, int n_networks, int64_t traj_total, int npts,
                                   const double *d_obs, const double *tangent, double *partials, hipStream_t stream)
{
    if (traj_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(tangent_contract_kernel, dim3((unsigned)((traj_total + 255) / 256)), dim3(256), 0, stream, nets,
                       n_networks, traj_total, npts, d_obs, tangent, partials);
    return hipGetLastError();
}

hipError_t launch_dobs_prefix(const NetDev *nets, int n_networks, int n_bins, const double *d_obs, double *pre,
                              hipStream_t stream)
{
    if (n_networks <= 0 || n_bins <= 0) return hipSuccess;
    hipLaunchKernelGGL(dobs_prefix_kernel, dim3((unsigned)n_networks), dim3(256), 0, stream, nets, n_bins, d_obs,
                       pre);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_selftest_philox(const uint32_t *ck, uint32_t *out, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(selftest_philox_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, ck, out, n);
    return hipGetLastError();
}

hipError_t launch_selftest_neglog(uint32_t first, int64_t count, float *out, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(selftest_neglog_kernel, dim3(grid_for(count, 256)), dim3(256), 0, stream, first,
                       count, out);
    return hipGetLastError();
}

}  // namespace ssa
