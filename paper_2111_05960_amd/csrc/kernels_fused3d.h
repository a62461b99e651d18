// Fused schedule for D3Q19 (one kernel per step): not yet available.
#pragma once

#include "kernels_fused2d.h"

namespace gplbm {

inline bool fused3d_supported(int, int, int, const int*) { return false; }

}  // namespace gplbm
