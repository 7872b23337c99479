// Gene-regulatory network classifier kernels (Sec. 4.3, Fig. 4A): the dense
// input contraction on bf16 MFMA, the direct-method forward and the
// straight-through backward with one trajectory per wavefront, and the
// deterministic gradient reductions (the weight gradient on FP64 MFMA).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ssa_plan.hpp"

namespace ssa {
namespace grn {

constexpr int kHid = 256;      // hidden genes (the kernels' lane/slot layout assumes it)
constexpr int kMaxOut = 16;    // output genes

struct GrnParams {
    int32_t n_in, n_out, n_images, n_rep;
    int64_t B;                  // trajectories = n_images * n_rep; trajectory q runs image q / n_rep
    float beta, delta_min;
    const float *theta;         // [W | b | U | c | psi]
    int64_t off_b, off_U, off_c, off_psi;
    const float *x_img;         // [n_images][n_in]
    float *u_hid;               // [n_images][kHid]
    const int32_t *x0;          // [kHid + n_out][B]
    int32_t *x_final;           // [kHid + n_out][B]
    double *t_final;            // [B]
    int32_t *steps_done;        // [B]
    double *obs;                // [n_out][B]
    uint32_t *tape;             // [B][tape_words]: the fired channel of step k is the 16-bit
                                // half (k & 1) of word 64 * (k >> 7) + ((k >> 1) & 63)
    int32_t tape_words;
    int32_t relaxed;            // nonzero: the relaxed forward of Eq. 4 and its exact backward
    float *soft;                // relaxed runs: [B][n_steps + 1][kHid + 2 kMaxOut] starting
                                // point of every step (hidden levels, output levels, output
                                // pre-activations), in place of the tape
    TieRec *ties;
    uint32_t *n_ties;
    uint32_t tie_cap;
    uint32_t *flags;
    uint32_t seed_lo, seed_hi, purpose, epoch;
    const uint32_t *d_epoch;
    const uint32_t *traj_ids;
    int32_t n_steps;
    float temperature;
    const float *d_temperature;   // when set, the temperature is read here on the device
    const double *d_obs;        // [n_out][B]
    double *part;               // [B][C] compact per-trajectory gradient
    float *e_hist;              // [B][n_steps][n_out] dL/dv_o of every step (backward scratch)
    int32_t C;                  // kHid + n_out*kHid + n_out + kHid + n_out
    double *g_img;              // [n_images][C]
    float *d_params;            // [P]
};

hipError_t launch_hidden_input(const GrnParams &p, hipStream_t stream);
hipError_t launch_forward(const GrnParams &p, hipStream_t stream);
// backward sweep, then the dL/dU and dL/dc pass
hipError_t launch_backward(const GrnParams &p, hipStream_t stream);
hipError_t launch_reduce(const GrnParams &p, hipStream_t stream);

}  // namespace grn
}  // namespace ssa
