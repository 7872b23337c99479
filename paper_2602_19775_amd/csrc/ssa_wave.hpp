// Wave-mode kernel classes: lanes per trajectory and Philox blocks per lane.
#pragma once

#include <hip/hip_runtime.h>

#include "ssa_plan.hpp"

namespace ssa {

// A class is a group width (lanes per trajectory) and the Philox blocks of
// four channel words each lane draws (channel j uses word j + 1, so a group of
// L lanes with BPL blocks each covers up to 4 L BPL - 1 channels).
enum WaveClass : int {
    kWave_L8 = 0,      // up to 31 channels
    kWave_L16 = 1,     // up to 63
    kWave_L32 = 2,     // up to 127
    kWave_L64 = 3,     // up to 255
    kWave_L64x2 = 4,   // up to 511
    kWave_L8x2 = 5,    // up to 63 on 8 lanes
    kWave_L16x2 = 6,   // up to 127 on 16 lanes
    kWave_L32x2 = 7,   // up to 255 on 32 lanes
    kWaveClassCount = 8,
};

constexpr int kWaveMaxSpecies = 64;
// Change-vector entries a channel slot keeps in registers for the backward's
// w = v_j . lambda (channels with more use the table in LDS).
constexpr int kVecSlots = 4;

// Class of a network with max_M channels for a width cap of max_lanes lanes
// (8, 16, 32 or 64): the narrowest group of at most max_lanes lanes with one
// Philox block per lane that covers it, else the max_lanes-wide group with two
// blocks per lane, else (too large for the cap) the narrowest class without
// the cap; -1 if nothing covers it.
int wave_class_for(int max_M, int max_lanes = 64);
int wave_class_lanes(int cls);
int wave_class_bpl(int cls);
// Persistent launch over p.items (one trajectory each); p.work_counter must be 0.
hipError_t wave_launch(int cls, const RunParams &p, bool backward, int n_blocks, hipStream_t stream);
// LDS bytes of a block besides the per-group network tables.
size_t wave_static_lds(int cls, bool backward);
constexpr size_t kLdsPerBlock = 160 * 1024;

}  // namespace ssa
