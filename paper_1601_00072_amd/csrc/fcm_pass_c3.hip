// Pass and persistent kernels instantiated for C = 3 clusters.
#include "fcm_device.h"

namespace fcm {

template <int MK>
static PassFn pick_u(int unroll, bool persistent) {
    if (persistent) return unroll == 2 ? fcm_persist_kernel<3, MK, 2> : fcm_persist_kernel<3, MK, 1>;
    return unroll == 2 ? fcm_pass_kernel<3, MK, 2> : fcm_pass_kernel<3, MK, 1>;
}

PassFn pick_c3(int mclass, int unroll, bool persistent) {
    if (mclass == kM2) return pick_u<kM2>(unroll, persistent);
    if (mclass == kM15) return pick_u<kM15>(unroll, persistent);
    return pick_u<kMGeneric>(unroll, persistent);
}

}  // namespace fcm
