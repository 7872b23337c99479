// Lane-mode kernel classes (compile-time bounds on species and channels).
#pragma once

#include <hip/hip_runtime.h>

#include "ssa_plan.hpp"

namespace ssa {

enum LaneClass : int {
    kLane_N4_M4 = 0,
    kLane_N8_M8 = 1,
    kLane_N8_M16 = 2,
    kLane_N16_M16 = 3,
    kLane_N16_M32 = 4,
    kLaneClassCount = 5,
};

// Class able to run a network with N species and M channels, or -1.
int lane_class_for(int N, int M);
int lane_class_nmax(int cls);
// Enqueues the forward (or backward) kernel of one class over p.items.
hipError_t lane_launch(int lane_class, const RunParams &p, bool backward, hipStream_t stream);

}  // namespace ssa
