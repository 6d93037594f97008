// The paper's own start (Algorithm 1 as printed): random memberships U^0,
// centroids first.  Host-side launcher of the two passes that differ from the
// centroid-first iteration (fcm_random.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcm_internal.h"

namespace fcm {

// Pass `phase` (0 or 1) of a solve that starts from random memberships drawn
// from the SplitMix64 stream `seed`; the state's pass counter must equal
// `phase`.  Phase 0 computes v^1 from U^0 (Eq.3); phase 1 evaluates U^1 from
// v^1 (Eq.4), its change against the regenerated U^0, J^1 and v^2.  One launch
// of `grid` blocks; the last block to finish reduces and commits, as in the
// per-pass driver.
hipError_t launch_random_pass(const PassArgs& a, int C, int phase, uint64_t seed, int grid, hipStream_t s);

}  // namespace fcm
