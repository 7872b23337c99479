// Tables and launch parameters shared by the host side of libssa and its
// kernels.  Everything here is plain data with a fixed layout.
#pragma once

#ifdef __HIPCC_RTC__
// runtime compilation: the fixed-width integer types come with the builtin headers
using __hip_internal::int8_t;
using __hip_internal::uint8_t;
using __hip_internal::int32_t;
using __hip_internal::uint32_t;
using __hip_internal::int64_t;
using __hip_internal::uint64_t;
#else
#include <stdint.h>
#endif

namespace ssa {

// Species slot meaning "no reactant": the kernels map it to a register that
// always holds the value 1, so order-0 and order-1 channels use the same
// two-factor propensity formula as order-2 channels.
constexpr int kNoSpecies = 0xFF;

// One channel (16 bytes).  a_j = k_j * mult * X[s1] * (X[s2] - homodimer).
struct ReactDesc {
    uint8_t s1, s2;
    uint8_t homodimer;   // 1 for 2S -> ..., so the second factor is X - 1
    uint8_t pad;
    int32_t rate;        // local parameter slot
    float mult;          // 0.5 for homodimers (number of distinct pairs), else 1
    int32_t csr;         // first change-vector entry (low 24 bits) | entry count << 24
};

// Sparse change-vector entry: species | delta << 16 (delta signed 16 bit).
__host__ __device__ inline int csr_species(int32_t e) { return e & 0xFFFF; }
__host__ __device__ inline int csr_delta(int32_t e) { return e >> 16; }

// Per-network header.
struct NetDev {
    int32_t N, M, P, n_obs;
    int32_t B;           // trajectories of this network
    int32_t wpr;         // 32-bit words of one packed change vector (8 species a word)
    int32_t react_off;   // first ReactDesc / parameter-map entry of the network
    int32_t rows_off;    // first packed change-vector word
    int32_t obs_sp_off;  // first observed-species entry
    int32_t mode;        // execution class chosen at plan time
    int32_t inc_off;     // first species-incidence offset (wave mode: N+1 entries)
    int32_t pad0;
    int64_t traj_off;    // sum of B over earlier networks
    int64_t state_off;   // sum of N*B
    int64_t param_off;   // sum of P
    int64_t obsb_off;    // sum of n_obs*B (times n_bins for bin observations)
    int64_t part_off;    // sum of M*B (per-channel gradient partials)
    int64_t ppt_off;     // sum of P*B (per-trajectory parameter gradients)
    int64_t obsw_off;    // sum of n_obs (times n_bins for bin and grid observations):
                         // ensemble means and a shared dL/dobs
    int64_t tobs_off;    // sum of ceil(B / 64) * n_obs (times n_bins): per-tile sums of the
                         // ensemble-mean forward, [tile][n_bins][n_obs] per network
    int64_t obst_off;    // sum of (n_obs + 1) * B: tail observations [n_obs + 1][B] per network
    int64_t obstw_off;   // sum of (n_obs + 1): their ensemble means
    int64_t tanw_off;    // sum of n_obs * M * B: forward-mode tangents d obs / d ln k_q per
                         // observation point, [point][obs][channel][B] per network
    double t_obs;
};

// A tile of up to 64 trajectories of one network (one wavefront in lane mode).
struct LaneItem {
    int32_t net;
    int32_t first;
    int32_t count;
    int32_t pad;
};

// Layout-identical to ssa_tie of the public header.
struct TieRec {
    uint32_t traj;
    uint32_t step;
    int32_t chosen;
    int32_t second;
    float margin;
    int32_t kind;
};

enum : uint32_t { kFlagOverflow = 1u, kFlagNonFinite = 2u };

// Selection near-tie window of the FP32 path: the relative gap of the two
// smallest E_j/a_j is logged when at most this (twice the analytic FP32 error
// bound of the ratios, so every true gap <= 1e-6 is caught).
constexpr float kTieLog = 2e-6f;
// Stop-decision window at t_end (relative to t_end).
constexpr double kClockTieLog = 1e-5;
// Bin-edge window of the bin observation (relative to the edge's time): an
// event time this close to a bin edge is logged with the side of the edge the
// FP32-accumulated clock put it on.  The derivative of a bin average with
// respect to an event time jumps at an edge, so that side decides which bin's
// dL/dobs enters the clock adjoint; a checker whose clock differs by less than
// half this window can take the same side.
constexpr double kEdgeLog = 4e-7;

// Forward-mode tangents (SSA_BWD_TANGENT) carry dX/d ln k_q for every channel
// rate q: networks with at most this many channels and species x channels.
constexpr int kTanMaxChannels = 4;
constexpr int kTanMaxStateTangents = 32;

struct RunParams {
    const NetDev *nets;
    const ReactDesc *rd;
    const uint32_t *rows;
    const int32_t *csr;
    const int32_t *obs_sp;
    const LaneItem *items;
    int32_t n_items;

    const float *theta;
    const int32_t *x0;
    int32_t *x_final;       // forward out / backward in
    double *t_final;
    int32_t *steps_done;
    double *obs;            // forward out
    const double *d_obs;    // backward in
    double *partials;       // backward out: per-channel FP64 partials [M][B] per network

    int32_t *ck_x;          // [n_ckpt][state_total]
    double *ck_t;           // [n_ckpt][traj_total]
    uint32_t *tape;         // [tape_words][traj_total]

    TieRec *ties;
    uint32_t *n_ties;
    uint32_t tie_cap;
    uint32_t *flags;

    uint32_t seed_lo, seed_hi;
    uint32_t purpose;
    uint32_t epoch;
    const uint32_t *d_epoch;
    const uint32_t *traj_ids;

    int32_t n_steps;
    double t_end;
    int32_t obs_kind;
    int32_t n_bins;
    int32_t K;              // checkpoint interval
    int32_t n_ckpt;
    int32_t tape_bits;      // bits per step in the choice tape (0: no tape)
    int32_t tape_words;
    int64_t state_total;
    int64_t traj_total;
    float temperature;
    const float *d_temperature;   // when set, the temperature is read here on the device
    int32_t selection;            // 0 Gumbel-max race, 1 inverse CDF (forward only)
    int32_t recompute;      // backward: recover choices by re-running segments
    int32_t obs_tm;         // obs / d_obs blocks are [trajectory][point][obs]
    int32_t dobs_shared;    // d_obs is one [point][obs] block per network
    const double *dobs_prefix;   // bins, shared d_obs: [obs][n_bins + 1] prefix sums per network
    double *tile_sums;           // ensemble-mean forward: per-tile sums (NetDev::tobs_off)
    int32_t obs_ens;             // the forward writes ensemble means (tile sums) only
    double *tangent;             // forward-mode tangents (SSA_BWD_TANGENT): forward out, backward in

    // wave mode: species -> range of incidence slots, and per channel the
    // slots of its (role 1, role 2) contributions: pos1 | pos2 << 16 with
    // 0xFFFF for none (incidence slots are grouped by species, channels in
    // increasing order, role 1 before role 2)
    const int32_t *inc_ptr;
    const int32_t *chan_inc;
    uint32_t *work_counter;
    // wave mode: per-group LDS copy of a network's change vectors and
    // incidence ranges (capacities in 32-bit words); wide_ve is set when a
    // channel of the group changes more than kVecSlots species
    int32_t tab_m, tab_nnz, tab_words;
    int32_t wide_ve;
};

}  // namespace ssa
