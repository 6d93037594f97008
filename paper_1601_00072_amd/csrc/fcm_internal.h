// Internal layout shared by the gfx950 kernels and the host runtime (not part of the ABI).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace fcm {

constexpr int kMaxC = 8;
constexpr int kBlock = 256;          // threads per block of every streaming kernel
constexpr int kMaxGrid = 8192;       // capacity of the partial-sum table
constexpr int kMaxPersistGrid = 2048; // blocks of a cooperative launch

// Cross-block exchange of the cooperative driver.  Zeroed when the handle is
// created (and after an aborted solve), never by a reset: the round count only
// grows, so tagged words of earlier rounds never match a later one.
// Two-level exchange: the blocks are dealt to the XCDs in turn (from some
// starting XCD), so blocks b and b + kXcds share an XCD; block x < kXcds
// reduces the rows of blocks x, x + kXcds, ... and publishes one row of the
// 2C + 1 FP64 sums (two tagged halves each) and the max.
constexpr int kXcds = 8;
constexpr int kXcdRowWords = 64;  // >= 2 (2 kMaxC + 1) + 1

struct SyncState {
    uint32_t gen;             // last round of the previous cooperative launch
    uint32_t abort;           // set when a wait hit its time limit; every block then exits
    uint64_t bcw[kMaxC + 1];  // block 0's decision: tagged centroids, then
                              // (next pass << 2 | two-level exchange usable << 1 | done)
    uint64_t passes_total;    // fused passes committed since the handle was created (every driver)
    uint64_t fin[2 * kMaxC];  // block 0's final centroids in FP64, two tagged halves each (fused labels)
    alignas(128) uint64_t xrow[2][kXcds][kXcdRowWords];  // two-level exchange: XCD rows, by round parity
};
static_assert(2 * (2 * kMaxC + 1) + 1 <= kXcdRowWords, "XCD row too small");

// Device-resident solver state.  Written only by the last block of a pass (or
// of the data-range pass), or by block 0 of a cooperative launch; read by every
// block at the start of the next launch.
struct DevState {
    int32_t pass;        // index p of the next fused pass (pass p computes U^p)
    int32_t done;        // nonzero once converged, out of iterations, or non-finite
    int32_t iters;       // last completed iteration t (-1 before the first pass)
    int32_t status;      // FCM_* status of the solve
    uint32_t ticket;     // arrival counter of the running pass; 0 between passes
    int32_t passes;      // fused passes executed
    int32_t lo, hi;      // grey-level range of the data
    double delta;        // max |dU| of iteration `iters` (NaN for iteration 0)
    double J;            // J_m(U^iters, v^iters)
    double vres[kMaxC];  // v^iters in FP64: the current result
    float v32[2][kMaxC]; // FP32 centroids used by the passes: v32[p & 1] = fl32(v^p)
    SyncState sync;      // cooperative driver handshake (not cleared by a reset)
};

// Per-block partial row of a fused pass, stored column-major in a
// [rows][grid] float table so that the final reduction reads it coalesced.
// Rows: for each k < C: num (sum, comp), den (sum, comp); then J (sum, comp);
// then delta (max).  Row count 4C + 3.
__host__ __device__ constexpr int partial_rows(int C) { return 4 * C + 3; }

// Row stride (64-bit words) of a persistent launch's tagged row of K words:
// rows start on 128-byte boundaries, so a row of up to 16 words is one cache
// line.  Buffer: [2][kMaxPersistGrid][kTaggedStrideMax] words.
__host__ __device__ constexpr int tagged_stride(int K) { return K <= 16 ? 16 : 32; }
constexpr int kTaggedStrideMax = 32;
static_assert(tagged_stride(2 * kMaxC + 2) <= kTaggedStrideMax, "tagged row buffer too small");

enum MClass : int { kM2 = 0, kM15 = 1, kMGeneric = 2 };

struct PassArgs {
    const uint8_t* x;      // voxel grey levels
    int64_t n;             // voxel count
    int64_t head;          // voxels before the first 16-byte aligned address
    int64_t nbody;         // 16-voxel chunks of the aligned body
    DevState* st;
    float* partials;       // [partial_rows(C)][grid]
    double* hist_v;        // [(max_iter + 2) * C]
    double* hist_d;        // [max_iter + 2]
    double* hist_J;        // [max_iter + 2]
    double eps;
    float alpha;           // 1 / (m - 1)
    float mexp;            // m
    int32_t max_iter;
    int32_t kahan_only;    // cross-block reduction in compensated FP32
    // cooperative driver only
    uint64_t* rows;        // [2][grid][16 or 32] tagged partial rows, by round parity
    uint64_t* mm_rows;     // [2][grid][2] tagged per-block grey-level range, by round parity
    int32_t allgather;     // every block reduces all rows (else block 0 reduces and broadcasts)
    int32_t xcd;           // two-level exchange through the XCDs when the dealing allows it
    int32_t do_init;       // run the data-range pass and set v^0 first
    int32_t given;         // start mode: 0 evenly spaced, 1 v0 below, 2 dv0 (device),
                           // 3 learned (persistent launch only; mlp_w, ghist below)
    double v0[kMaxC];
    const double* dv0;     // C start centroids in device memory (mode 2)
    int32_t max_passes;    // passes this launch may run
    int32_t pad;
    uint64_t spin_ticks;   // wall-clock limit of one wait
    const uint16_t* mlp_w; // mode 3: BF16 parameters of the histogram -> centroid network (C outputs)
    uint32_t* ghist;       // mode 3: [kHistCopies][256] grey-level counters, zero at entry
    uint32_t* ghist_next;  // mode 3: the counters of the next learned launch, zeroed by this one
    uint8_t* labels;       // persistent launch: labels of the result, written when the solve ends (or null)
    int32_t labels_bytewise;  // x and labels differ in 16-byte alignment
    int32_t pad3;
};

constexpr int kHistCopies = 16;  // copies of the in-kernel histogram (blocks spread their atomics)

struct InitArgs {
    const uint8_t* x;
    int64_t n, head, nbody;
    DevState* st;
    uint32_t* partials;    // [2][grid]
    double* hist_v;
    int32_t C;
    int32_t given;         // start mode: 0 evenly spaced, 1 v0 below, 2 dv0 (device)
    double v0[kMaxC];
    const double* dv0;
};

struct LabelArgs {
    const uint8_t* x;
    uint8_t* labels;
    int64_t n, head, nbody;
    const DevState* st;
    const double* hist_v;
    int32_t C;
    int32_t bytewise;      // x and labels differ in 16-byte alignment
};

// ---- batched solver: many instances of uneven size in one persistent launch ----

constexpr int kBatchRowWords = 32;  // stride of a tile row (2C + 2 tagged words used), 256-byte aligned
// Tagged decision words per instance: v^p (FP32) [kMaxC], v^(p-1) (FP32)
// [kMaxC], p, then v^p in FP64 as two halves each [2 kMaxC].  The block that
// completes the next pass takes v^p from here, not from the history: it may
// run on another XCD, whose L2 need not hold the history's latest contents.
constexpr int kBatchDecWords = 4 * kMaxC + 1;
constexpr int kBatchDecF64 = 2 * kMaxC + 1;  // offset of the FP64 halves

// Control word of an instance (64 bits, changed only by agent-scope atomics):
//   bits 63..32  tag of the instance's current phase (phase 0: data range,
//                phase p + 1: fused pass p), round0 + 1 + phase
//   bits 31..16  tiles of the phase whose rows are written (arrivals)
//   bits 15..0   tiles of the phase handed out (claims)
// A finished instance keeps claims at kBatchDoneClaims, above any tile count.
constexpr uint64_t kBatchClaim = 1ull;
constexpr uint64_t kBatchArrive = 1ull << 16;
constexpr uint32_t kBatchDoneClaims = 0x8000u;
constexpr int32_t kBatchFineFrom = 96;      // default first pass on the fine tiles
constexpr int32_t kBatchFineChunks = 2;     // default chunks per thread of a fine tile
constexpr int32_t kBatchChunks = 4;         // default chunks per thread of a coarse tile
constexpr int32_t kBatchBlock = 512;        // default threads per block of the batched kernel
constexpr int32_t kBatchMaxTiles = 0x6000;  // tiles per instance: a phase's claims stay below 2^16 (every
                                            // arrival also claims, so at most twice the tiles plus one
                                            // per concurrent claimer, kMaxPersistGrid)

struct BatchInst {
    int64_t base;        // byte offset of the instance's first voxel in the input
    int64_t n, head, nbody;
    int64_t hist;        // offset (doubles) of its history: v (max_iter + 2) * C, then delta, J and the
                         // commit times (max_iter + 2 each)
    int32_t C, mclass, max_iter, kahan_only;
    int32_t given;       // start mode (0 spaced, 1 v0, 2 dv0)
    int32_t tile0, ntiles;    // coarse tiles: phase 0 and passes below BatchArgs::fine_from
    int32_t tile0f, ntilesf;  // fine tiles: the passes from BatchArgs::fine_from on
    int32_t pad;
    float alpha, mexp;
    double eps;
    double v0[kMaxC];
    const double* dv0;   // C start centroids in device memory (mode 2)
};

struct BatchTile {
    int64_t c0, c1;      // 16-voxel chunks [c0, c1) of the instance's aligned body
    int32_t inst;
    int32_t ragged;      // this tile also takes the instance's unaligned head and tail voxels
};

struct BatchRec {        // per-instance result, written by the block that completes each phase
    int32_t pass, done, iters, status, passes, lo, hi, pad;
    double delta, J;
    double vres[kMaxC];
};

struct BatchSync {
    uint32_t abort;      // set when a wait hit its time limit; every block then exits
    uint32_t active;     // instances not yet finished
    uint32_t tiles_left; // tiles of the instances not yet finished
    uint32_t epoch;      // phases opened so far: blocks without work rescan only when it changes
    uint64_t t_start;    // wall clock at the start of the launch (block 0)
};

struct BatchArgs {
    const uint8_t* x;
    const BatchInst* inst;
    const int32_t* ntiles;  // [I][2] coarse and fine tiles per instance (dense copy for the scan)
    const BatchTile* tiles;
    BatchRec* recs;
    double* hist;
    uint64_t* rows;      // [ntiles][kBatchRowWords] tagged tile rows (phase 0: grey-level range)
    uint64_t* dec;       // [I][kBatchDecWords] tagged decisions (see kBatchDecWords)
    uint64_t* ctl;       // [I] control words, round0 + 1 << 32 at launch
    BatchSync* sync;
    int32_t I;
    int32_t fine_from;   // passes from this one on run on the fine tiles
    uint32_t round0;     // tags of this launch are above round0
    uint32_t pad2;
    uint64_t spin_ticks;
};

struct BatchLabelArgs {
    const uint8_t* x;
    uint8_t* labels;
    const BatchInst* inst;
    const BatchTile* tiles;
    const BatchRec* recs;
    const double* hist;
    int32_t ntiles, bytewise;
};

// the batched kernel is built for 128-, 256- and 512-thread blocks
hipError_t batch_max_grid(int block, int ncu, int* max_grid);
hipError_t launch_batch(const BatchArgs& a, int block, int grid, hipStream_t s);
hipError_t launch_batch_labels(const BatchLabelArgs& a, int grid, hipStream_t s);
hipError_t launch_batch_targets(const BatchRec* recs, int32_t I, int32_t C, float* out, hipStream_t s);

// Histogram-domain solve (one block; fcm_levels.hip).
struct LevelArgs {
    const uint32_t* counts;  // [256] grey-level counts of the input
    DevState* st;
    double* hist_v;
    double* hist_d;
    double* hist_J;
    double eps, m;
    int32_t max_iter;
    int32_t do_init;         // compute the data range and v^0 first
    int32_t given;           // start mode: 0 evenly spaced, 1 v0 below, 2 dv0 (device)
    int32_t max_passes;      // passes this launch may run
    double v0[kMaxC];
    const double* dv0;
};
hipError_t launch_levels(const LevelArgs& a, int C, hipStream_t s);

using PassFn = void (*)(PassArgs);

// Launchers (fcm_common.hip, fcm_dispatch.hip).  Return hipSuccess or the launch error.
hipError_t launch_init(const InitArgs& a, int grid, hipStream_t s);
hipError_t launch_pass(const PassArgs& a, int C, int mclass, int unroll, int grid, hipStream_t s);
hipError_t launch_labels(const LabelArgs& a, int grid, hipStream_t s);
bool pass_supported(int C, int mclass, int unroll);
hipError_t persist_max_grid(int C, int mclass, int unroll, int ncu, int* max_grid);
hipError_t launch_persist(const PassArgs& a, int C, int mclass, int unroll, int grid, bool cooperative,
                          hipStream_t s);

}  // namespace fcm
