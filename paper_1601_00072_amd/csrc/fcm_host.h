// Host-side helpers shared by the runtime translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string>

struct fcm_handle;
struct fcm_batch;

namespace fcm {

// What the autotuner needs to know about a handle or a batch.
struct HandleShape {
    int64_t n, nbody;   // voxels, aligned 16-voxel chunks
    int C, mclass, kahan, device, ncu, coop;
};
struct BatchShape {
    int64_t voxels;     // all instances
    int count, max_C, device, max_grid, chunks_per_thread, grid, block;
};
int handle_shape(const fcm_handle* h, HandleShape* s);
int batch_shape(const fcm_batch* b, BatchShape* s);

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
