// Fused schedule for D2Q9 (one kernel per step): not yet available.
#pragma once

#include "kernels_split.h"

namespace gplbm {

inline bool fused2d_supported(int, int) { return false; }

template <class L, class S, class C>
struct FusedLaunch {
  static int launch(const Geo&, const Coef<C>&, const StepBufs<S>&, hipStream_t) { return -1; }
};

}  // namespace gplbm
