// Wave-mode kernel classes: lanes per trajectory and Philox blocks per lane.
#pragma once

#include <hip/hip_runtime.h>

#include "ssa_plan.hpp"

namespace ssa {

enum WaveClass : int {
    kWave_L8 = 0,      // up to 31 channels
    kWave_L16 = 1,     // up to 63
    kWave_L32 = 2,     // up to 127
    kWave_L64 = 3,     // up to 255
    kWave_L64x2 = 4,   // up to 511
    kWaveClassCount = 5,
};

constexpr int kWaveMaxSpecies = 64;
// Change-vector entries a channel slot keeps in registers for the backward's
// w = v_j . lambda (channels with more use the table in LDS).
constexpr int kVecSlots = 4;

// Smallest class whose group covers every Philox block of a network with
// max_M channels, or -1.
int wave_class_for(int max_M);
int wave_class_lanes(int cls);
// Persistent launch over p.items (one trajectory each); p.work_counter must be 0.
hipError_t wave_launch(int cls, const RunParams &p, bool backward, int n_blocks, hipStream_t stream);
// LDS bytes of a block besides the per-group network tables.
size_t wave_static_lds(int cls, bool backward);
constexpr size_t kLdsPerBlock = 160 * 1024;

}  // namespace ssa
