// Host-side helpers shared by the C ABI translation units: the thread-local
// detail message behind ssa_last_error().
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "ssa.h"

namespace ssa {

extern thread_local std::string g_last_error;

// Records msg as the detail of the failing call and returns s.
ssa_status fail(ssa_status s, const std::string &msg);
ssa_status hip_fail(hipError_t e, const char *what);

}  // namespace ssa
