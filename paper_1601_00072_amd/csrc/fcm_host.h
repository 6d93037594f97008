// Host-side helpers shared by the runtime translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace fcm {

// Text returned by fcm_last_error (per thread).
std::string& last_error();

// Record a failed HIP call and return FCM_EDEVICE.
int dev_err(hipError_t e, const char* what);

}  // namespace fcm

#define FCM_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return ::fcm::dev_err(e_, #call); \
    } while (0)
