// Kernel selection and launch of the fused pass (both drivers).
#include <hip/hip_runtime.h>

#include "fcm_internal.h"

namespace fcm {

PassFn pick_c2(int mclass, int unroll, bool persistent);
PassFn pick_c3(int mclass, int unroll, bool persistent);
PassFn pick_c4(int mclass, int unroll, bool persistent);
PassFn pick_c5(int mclass, int unroll, bool persistent);
PassFn pick_c6(int mclass, int unroll, bool persistent);
PassFn pick_c7(int mclass, int unroll, bool persistent);
PassFn pick_c8(int mclass, int unroll, bool persistent);

static PassFn pick(int C, int mclass, int unroll, bool persistent) {
    if ((mclass != kM2 && mclass != kM15 && mclass != kMGeneric) || (unroll != 1 && unroll != 2)) return nullptr;
    switch (C) {
        case 2: return pick_c2(mclass, unroll, persistent);
        case 3: return pick_c3(mclass, unroll, persistent);
        case 4: return pick_c4(mclass, unroll, persistent);
        case 5: return pick_c5(mclass, unroll, persistent);
        case 6: return pick_c6(mclass, unroll, persistent);
        case 7: return pick_c7(mclass, unroll, persistent);
        case 8: return pick_c8(mclass, unroll, persistent);
        default: return nullptr;
    }
}
bool pass_supported(int C, int mclass, int unroll) { return pick(C, mclass, unroll, false) != nullptr; }

hipError_t launch_pass(const PassArgs& a, int C, int mclass, int unroll, int grid, hipStream_t s) {
    PassFn f = pick(C, mclass, unroll, false);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t persist_max_grid(int C, int mclass, int unroll, int ncu, int* max_grid) {
    PassFn f = pick(C, mclass, unroll, true);
    if (!f) return hipErrorInvalidValue;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f), kBlock, 0);
    if (e != hipSuccess) return e;
    *max_grid = per_cu * ncu;
    return hipSuccess;
}

hipError_t launch_persist(const PassArgs& a, int C, int mclass, int unroll, int grid, bool cooperative,
                          hipStream_t s) {
    PassFn f = pick(C, mclass, unroll, true);
    if (!f) return hipErrorInvalidValue;
    PassArgs copy = a;
    void* args[] = {&copy};
    if (cooperative)
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(f), dim3(grid), dim3(kBlock), args, 0, s);
    return hipLaunchKernel(reinterpret_cast<const void*>(f), dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace fcm
