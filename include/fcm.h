/*
 * fcm.h -- C ABI of the gfx950 Fuzzy C-Means segmentation library.
 *
 * The library clusters 8-bit images or volumes by grey level with Fuzzy
 * C-Means (FCM): objective J_m = sum_i sum_j u_ij^m (x_i - v_j)^2 (Eq.1) under
 * sum_j u_ij = 1 (Eq.2), alternating the centroid update
 * v_j = sum_i u_ij^m x_i / sum_i u_ij^m (Eq.3) and the membership update
 * u_ij = 1 / sum_k (d_ij / d_ik)^(2/(m-1)) (Eq.4) until the largest change of
 * any membership between two iterations falls below eps (Algorithm 1), then
 * assigning each voxel to its cluster of largest membership (defuzzification,
 * Sec. 2.1 and Sec. 4.3).  The problem statement -- pixel array in, cluster
 * count c, fuzziness m and eps as parameters, cluster centres and the
 * segmented image out -- is that of Algorithm 1 and Sec. 4.1-4.3.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HIP device memory); all other
 *     pointers are host pointers.  Device buffers passed in are borrowed: the
 *     caller owns them and keeps them valid while the handle uses them.
 *   - All GPU work is enqueued on the stream given to fcm_init (a hipStream_t
 *     passed as void*; NULL means the null stream).  Only fcm_iterate,
 *     fcm_solve, fcm_centroids and fcm_trajectory wait for that stream.
 *   - Functions return an int status: FCM_OK (0), FCM_NOT_CONVERGED (1),
 *     FCM_RUNNING (2), or a negative error.  Arguments are validated before any
 *     HIP call; on error nothing is enqueued and outputs are left untouched.
 *     No C++ exception crosses this boundary.
 *   - A handle is not re-entrant; distinct handles may be used concurrently on
 *     distinct streams.
 */
#ifndef FCM_H
#define FCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FCM_OK              0   /* converged: max |dU| < eps at iteration T */
#define FCM_NOT_CONVERGED   1   /* max_iter iterations ran; result is v^max_iter */
#define FCM_RUNNING         2   /* neither converged nor out of iterations yet */
#define FCM_EINVAL        (-1)  /* invalid argument */
#define FCM_ENOMEM        (-2)  /* device or host allocation failed */
#define FCM_EDEVICE       (-3)  /* a HIP call failed (message: fcm_last_error) */
#define FCM_ESTATE        (-4)  /* call out of order (e.g. labels before init) */
#define FCM_ENUMERIC      (-5)  /* a non-finite centroid or objective appeared */
#define FCM_EUNSUPPORTED  (-6)  /* configuration not built into this library */
#define FCM_EIO           (-7)  /* a file could not be read or written, or does not hold
                                   a network of the expected layout */

#define FCM_MAX_CLUSTERS 8

/* initialisation of the centroids v^0 */
#define FCM_INIT_LINSPACE 0     /* v_j = lo + j (hi - lo) / (C - 1) over the data range,
                                   evaluated in FP64, rounded to FP32 */
#define FCM_INIT_GIVEN    1     /* v^0 = init_centroids, rounded to FP32 */
#define FCM_INIT_DEVICE   2     /* v^0 read at the start of every solve from the DEVICE
                                   array init_centroids (C doubles, borrowed), rounded
                                   to FP32; any non-finite value selects LINSPACE.
                                   Used by the learned warm start. */
#define FCM_INIT_RANDOM_U 3     /* the paper's start (Sec. 2.1, Algorithm 1): random
                                   memberships U^0, u_ij = r_ij / sum_k r_ik with r_ij
                                   = (top 24 bits of draw i C + j of the SplitMix64
                                   stream `seed`, plus 1) / 2^24, then the centroids
                                   first: pass 0 computes v^1 from U^0, pass 1 tests
                                   U^1 against U^0.  v^0, J^0 and delta^0 are NaN.
                                   Not for batches or the histogram driver (U^0 is not
                                   a function of the grey level). */

/* flags */
#define FCM_F_KAHAN_ONLY  (1u << 0)  /* cross-block reduction in compensated FP32
                                        instead of FP64 */
#define FCM_F_TIMING      (1u << 1)  /* time every fused pass with HIP events */

/* iteration drivers */
#define FCM_DRIVER_LOOP   0     /* one launch per pass from the host */
#define FCM_DRIVER_GRAPH  1     /* a hipGraph of graph_k passes, replayed */
#define FCM_DRIVER_PERSISTENT 2 /* one persistent launch runs the data-range pass
                                   and every pass of a solve (default where
                                   supported) */
#define FCM_DRIVER_HISTOGRAM  3 /* histogram domain: one pass counts the grey levels,
                                   then Algorithm 1 runs over the (at most 256)
                                   levels present in FP64 in one block; every voxel
                                   sum regroups exactly by level, so the result is the
                                   same iteration (up to rounding order), and the data
                                   are read once per solve */

/* how the blocks of a persistent launch combine their partial sums each pass */
#define FCM_EXCHANGE_AUTO      0  /* all-gather on small grids, else leader */
#define FCM_EXCHANGE_LEADER    1  /* block 0 reduces and broadcasts the decision */
#define FCM_EXCHANGE_ALLGATHER 2  /* every block reduces every partial row itself */
#define FCM_EXCHANGE_XCD       3  /* two levels: the blocks sharing an XCD (blocks are dealt to
                                     the 8 XCDs in turn) combine their rows in one block of that
                                     XCD, which publishes an FP64 row; every block adds the 8
                                     XCD rows itself (no broadcast).  Every exchange word is
                                     stored and read with agent scope.  The dealing is checked in
                                     the data-range pass of each solve; where it differs, and for
                                     launches that continue a solve, the leader exchange is used.
                                     Not with FCM_F_KAHAN_ONLY */

/* how the persistent driver launches its kernel */
#define FCM_LAUNCH_COOPERATIVE 0  /* hipLaunchCooperativeKernel: the runtime guarantees
                                     that every block is resident at once (about 15 us
                                     more dispatch time per solve on MI355X) */
#define FCM_LAUNCH_RESIDENT    1  /* default: ordinary launch of a grid no larger than the
                                     device holds at once.  Another kernel occupying the
                                     device can delay some blocks; a wait that exceeds the
                                     time limit (5 s, fcm_set_wait_limit) ends the launch:
                                     fcm_solve then solves again from the start in a
                                     cooperative launch (fcm_solve_async reports
                                     FCM_EDEVICE through fcm_solve_wait) */

typedef struct fcm_params {
    int32_t n_clusters;           /* C, 2..FCM_MAX_CLUSTERS */
    double  m;                    /* fuzziness, finite and > 1 */
    double  eps;                  /* stop when max_ij |u_ij^t - u_ij^(t-1)| < eps; finite, > 0 */
    int32_t max_iter;             /* >= 1 */
    int32_t init;                 /* FCM_INIT_* */
    const double* init_centroids; /* FCM_INIT_GIVEN: host, C finite values (copied);
                                     FCM_INIT_DEVICE: device, C values (borrowed) */
    uint32_t flags;               /* FCM_F_* */
    uint64_t seed;                /* FCM_INIT_RANDOM_U: the generator stream (else ignored) */
} fcm_params;

typedef struct fcm_tuning {
    int32_t block;      /* threads per block of the fused pass: 256 (the only size built) */
    int32_t grid;       /* blocks of the fused pass; 0 picks from the device and n.
                           The persistent driver caps it at the number of blocks
                           that fit on the device at once. */
    int32_t unroll;     /* 16-voxel chunks in flight per thread: 1 or 2 */
    int32_t driver;     /* FCM_DRIVER_* */
    int32_t graph_k;    /* loop/graph drivers: passes per host synchronisation
                           (and per graph), 1..64 */
    int32_t exchange;   /* persistent driver: FCM_EXCHANGE_* */
    int32_t launch;     /* persistent driver: FCM_LAUNCH_* */
} fcm_tuning;

typedef struct fcm_result {
    int32_t iters;      /* T: iterations completed (0 after the first pass) */
    int32_t passes;     /* fused passes executed (T + 1 once finished) */
    int32_t status;     /* FCM_OK, FCM_NOT_CONVERGED, FCM_RUNNING or FCM_ENUMERIC */
    int32_t n_clusters;
    double  delta;      /* max |dU| of iteration T (NaN for T = 0) */
    double  J;          /* J_m(U^T, v^T) */
    double  centroids[FCM_MAX_CLUSTERS]; /* v^T, the centroids that produced U^T */
    double  kernel_ms;  /* with FCM_F_TIMING: summed event time of the passes run */
    int32_t lo, hi;     /* smallest and largest grey level of the data */
} fcm_result;

typedef struct fcm_handle fcm_handle;

/* Create a solver for d_x[0..n) (uint8 grey levels, any alignment, borrowed,
 * never written).  Validates, allocates the handle's workspace (O(grid * C)
 * partial sums plus O(max_iter * C) history), and enqueues the data-range pass
 * that computes lo, hi and v^0.  n >= 1; n < C is allowed.
 * Errors: FCM_EINVAL (null pointers, n < 1, C outside 2..8, m <= 1 or not
 * finite, eps <= 0 or not finite, max_iter < 1, bad init mode, non-finite
 * given centroids, unknown flags), FCM_ENOMEM, FCM_EDEVICE. */
int fcm_init(fcm_handle** h, const uint8_t* d_x, int64_t n, const fcm_params* p, void* stream);

/* Restart the solve from v^0 on the same input: enqueues the data-range pass
 * again (the input may have new contents of the same size) and clears the
 * iteration history and the FCM_F_TIMING total.  No allocation. */
int fcm_reset(fcm_handle* h);

/* Override the launch configuration (before the first pass, or between
 * calls).  FCM_EINVAL for values outside the documented ranges. */
int fcm_set_tuning(fcm_handle* h, const fcm_tuning* t);
int fcm_get_tuning(const fcm_handle* h, fcm_tuning* t);

/* Run up to k more fused passes (stopping early once finished), wait for the
 * stream, and report the state.  Returns the result status (FCM_RUNNING if
 * more iterations remain) or a negative error. */
int fcm_iterate(fcm_handle* h, int32_t k, fcm_result* out);

/* Iterate to convergence or max_iter and report (Algorithm 1). */
int fcm_solve(fcm_handle* h, fcm_result* out);

/* Defuzzify (Sec. 2.1, Sec. 4.3): d_labels[i] = argmin_j |x_i - v_j^T| in FP64,
 * ties to the lowest j, which is the cluster of largest membership for m > 1.
 * d_labels: caller-owned device buffer of n bytes.  Enqueued, not waited for. */
int fcm_labels(fcm_handle* h, uint8_t* d_labels);

/* Enqueue a whole solve (reset, start, Algorithm 1 to its end) on the
 * handle's stream and return without waiting: with the persistent driver this
 * is one kernel launch and no host synchronisation, so that solves and other
 * work can follow back to back (serving loops, pipelines).  d_labels (device,
 * n bytes, may be NULL): the labels of the result (as fcm_labels writes
 * them), computed by the same launch once the solve ends.  With the other
 * drivers, or the random-membership start, whose passes are driven from the
 * host, it runs the synchronous solve (and fcm_labels).  The result is read
 * with fcm_solve_wait; trajectories may be requested meanwhile (they are
 * ordered on the same stream).  A wait that hits its time limit in any
 * pending solve is reported by the next fcm_solve_wait (the labels of that
 * solve are then not written). */
int fcm_solve_async(fcm_handle* h, uint8_t* d_labels);

/* Wait for the handle's stream and report the last solve (as fcm_solve
 * does).  out->kernel_ms: with FCM_F_TIMING, the summed launch time of every
 * solve since the previous fcm_solve_wait.  total_passes (may be NULL): fused
 * passes committed on this handle since it was created (all drivers; restarts
 * from 0 after a recovered time-out), to count the work of pending solves. */
int fcm_solve_wait(fcm_handle* h, fcm_result* out, int64_t* total_passes);

/* Wall-clock limit of one cross-block wait of the persistent driver, in
 * seconds (0 < seconds <= 60; default 5; 0 keeps the current limit), and
 * recoveries (may be NULL): how many solves on this handle were run again in a
 * cooperative launch.  A wait that reaches the limit ends the launch in every
 * block (each wait also watches a shared abort word), and the solve reports
 * FCM_EDEVICE -- except that fcm_solve (also inside fcm_solve_warm) runs a
 * solve that began from its start, with the default resident launch
 * (FCM_LAUNCH_RESIDENT), once more from the start in a cooperative launch,
 * which the runtime makes co-resident, waiting at least the default limit;
 * that result is then returned and counted here.  A limit far below the
 * duration of a pass makes every wait give up: that is how the tests drive the
 * failure path from the host.  FCM_EINVAL for a limit outside the range. */
int fcm_set_wait_limit(fcm_handle* h, double seconds, int32_t* recoveries);

/* Copy v^T (C doubles) to the host buffer out. */
int fcm_centroids(fcm_handle* h, double* out);

/* Iteration history: v^t (C doubles into v_out, may be NULL), delta^t and J^t
 * (may be NULL) for 0 <= t <= T.  FCM_EINVAL for t outside that range. */
int fcm_trajectory(fcm_handle* h, int32_t t, double* v_out, double* delta, double* J);

/* Release the handle's workspace (waits for the stream).  NULL is ignored. */
void fcm_destroy(fcm_handle* h);

/* ---- batched solver ------------------------------------------------------
 * Many independent instances (2-D slices, 3-D volumes; each with its own C,
 * m, eps, max_iter, init and flags) solved together in one persistent launch:
 * every instance follows Algorithm 1 exactly as fcm_solve would, and the
 * launch ends when every instance has converged or run out of iterations.
 * Instance i is d_x[offsets[i] .. offsets[i+1]) of one concatenated uint8
 * device buffer (borrowed); offsets (count + 1 values, host) must start at 0,
 * be non-decreasing with every instance non-empty.  params: count host
 * records (init_centroids, if used, are copied). */
typedef struct fcm_batch fcm_batch;

/* Validates everything before any HIP call (FCM_EINVAL), allocates the
 * workspace (tile table, per-instance state and history), enqueues nothing.
 * The solve is one ordinary launch: its blocks take tiles of whichever
 * instance has work ready and never wait for one another's work in
 * progress, so the grid need not be resident at once. */
int fcm_batch_init(fcm_batch** b, const uint8_t* d_x, const int64_t* offsets, int32_t count,
                   const fcm_params* params, void* stream);

/* Tile size: chunks_per_thread 16-voxel chunks per thread and tile (1..64,
 * default 4; a tile is one block wide, fcm_batch_set_block; an instance that
 * would need more than 24,576 tiles gets larger ones), and the launch grid
 * (0 = as many blocks as fit on the device).  Rebuilds the tile table.  The tiling fixes the
 * order in which an instance's partial sums are added, so results are
 * reproducible for a given tiling (and differ between tilings by FP32
 * rounding only). */
int fcm_batch_set_tiling(fcm_batch* b, int32_t chunks_per_thread, int32_t grid);

/* Threads per block of the batched kernel: 512 (default; one block per CU,
 * so a tile, and a whole single-tile phase, runs on a whole CU), 256 (two
 * blocks per CU) or 128 (four).  A tile holds threads x chunks_per_thread chunks, so tile
 * sizes scale with the block size.  Results are reproducible for a given
 * block size and tiling.  Rebuilds the tile table; FCM_EINVAL for other
 * sizes. */
int fcm_batch_set_block(fcm_batch* b, int32_t threads);

/* Tiles of the later passes: from pass from_pass on (>= 0; default 96) every
 * instance runs on a second, finer tile set of chunks_per_thread chunks per
 * thread (1..64; default 2).  Few instances remain by then, and each pass of
 * the longest solves lies on the launch's critical path, so more, smaller
 * tiles let more blocks share it; the early passes keep the coarse tiles and
 * their lower per-tile cost.  The switch depends on the pass index only, so
 * results stay reproducible.  Rebuilds the tile table. */
int fcm_batch_set_tail_tiling(fcm_batch* b, int32_t from_pass, int32_t chunks_per_thread);

/* Solve every instance from its v^0; waits for the stream; out[i] (count
 * records) receives instance i's result.  Returns FCM_OK if every instance
 * converged, FCM_NOT_CONVERGED if any ran out of iterations, FCM_ENUMERIC if
 * any hit a non-finite value (see each out[i].status), or an error. */
int fcm_batch_solve(fcm_batch* b, fcm_result* out);

/* Labels of every instance into d_labels (offsets[count] bytes, the same
 * layout as the input), after fcm_batch_solve.  Enqueued, not waited for. */
int fcm_batch_labels(fcm_batch* b, uint8_t* d_labels);

/* History of instance inst (as fcm_trajectory). */
int fcm_batch_trajectory(fcm_batch* b, int32_t inst, int32_t t, double* v_out, double* delta, double* J);

/* Timeline of instance inst in the last solve: us[0] = microseconds from the
 * start of the launch until the instance's data range and v^0 were
 * committed, us[1 + p] = until pass p was committed (device wall clock), for
 * the first min(cap, passes + 1) phases; count (may be NULL) receives
 * passes + 1.  FCM_ESTATE before a solve. */
int fcm_batch_timeline(fcm_batch* b, int32_t inst, double* us, int32_t cap, int32_t* count);

void fcm_batch_destroy(fcm_batch* b);

/* ---- autotuner ------------------------------------------------------------
 * Both calls time whole solves on the object's own data (host wall clock
 * around reset + solve, the median of `reps` runs, 1..100) for a set of
 * candidate launch configurations, keep the fastest candidate whose result
 * agrees with the configuration in place at entry (same iteration count and
 * centroids within 1e-5 relative, or one iteration apart and within 1e-4),
 * apply it, and return it.  cache_path (may be NULL): a text file of earlier
 * choices, one line each, keyed by device, HIP runtime version and problem
 * class; a matching entry is applied without timing, and a new choice is
 * appended.  Choices are also cached per process.  The data must not change
 * during the call. */

/* Single instance: persistent driver (ordinary launch) over grids from half
 * the CU count up to one 16-voxel chunk per thread, leader, all-gather and two-level
 * exchange, unroll 1 and 2; graph driver with 4 and 16 passes per graph.
 * Key: C, the m class (2, 1.5, other), the precision flag and floor(log2 n).
 * The handle is left reset with the chosen tuning (chosen may be NULL; ms:
 * the chosen configuration's median solve time, may be NULL). */
int fcm_autotune(fcm_handle* h, const char* cache_path, int32_t reps, fcm_tuning* chosen, double* ms);

/* Batch: blocks of 512, 256 and 128 threads x tiles of 1, 2, 3, 4, 5, 6, 8, 12
 * or 16 chunks per thread, on the largest grid the device holds and on half
 * of it (the tail tiling stays as set).  Key: instance count, largest C and
 * floor(log2 of the total voxels).  The chosen block size and tiling are
 * applied (fcm_batch_set_block, fcm_batch_set_tiling); outputs may be NULL. */
int fcm_batch_autotune(fcm_batch* b, const char* cache_path, int32_t reps, int32_t* block,
                       int32_t* chunks_per_thread, int32_t* grid, double* ms);

/* ---- learned warm start -------------------------------------------------
 * A small network maps the normalised 256-bin grey-level histogram of an
 * instance to start centroids: 256 -> 128 (ReLU) -> 64 (ReLU) -> C (linear),
 * output = centroids / 255.  The fuzzy objective J_m (Eq.1) is what FCM
 * minimises; the network only proposes v^0, and Algorithm 1 is then run from
 * there exactly as from any other start.  Parameters are one flat FP32
 * vector: W1 [256][128], b1 [128], W2 [128][64], b2 [64], W3 [64][C], b3 [C]
 * (row-major, [in][out]).  Training: FP32 forward and backward on the GPU,
 * mean squared error over the batch and the C outputs, Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected).  Inference for warm starts: BF16
 * weights and activations (round to nearest even), FP32 accumulation.  All
 * reductions run in a fixed order: the same calls give the same bits.
 * A network belongs to the stream given at creation; its parameters must not
 * change while inference that reads them runs on another stream. */
typedef struct fcm_mlp fcm_mlp;

#define FCM_MLP_FP32 0
#define FCM_MLP_BF16 1

typedef struct fcm_train_cfg {
    int32_t  epochs;   /* passes over the training set, >= 1 */
    int32_t  batch;    /* minibatch size, 1..4096 (the last batch of an epoch may be smaller) */
    float    lr;       /* Adam step size, finite and > 0 */
    uint32_t pad;
    uint64_t seed;     /* order of the samples: a Fisher-Yates shuffle per epoch
                          drawn from a SplitMix64 counter generator */
} fcm_train_cfg;

/* Number of parameters of the network with C outputs (41,412 for C = 4), or
 * FCM_EINVAL for C outside 2..8. */
int32_t fcm_mlp_param_count(int32_t C);

/* Create a network with C outputs, He-initialised (weights N(0, 2 / fan_in)
 * from a SplitMix64 counter generator and Box-Muller keyed by seed; biases
 * 0), Adam state zero.  Allocates its parameters, optimiser state and
 * workspace on the current device. */
int fcm_mlp_create(fcm_mlp** net, int32_t C, uint64_t seed, void* stream);

/* Copy the flat parameter vector to / from host memory (fcm_mlp_param_count
 * floats).  Setting parameters also clears the Adam state.  Both wait for
 * the stream. */
int fcm_mlp_get_params(fcm_mlp* net, float* out);
int fcm_mlp_set_params(fcm_mlp* net, const float* in);

/* Inference: d_out[count][C] = network(d_hist[count][256]) in FP32
 * (FCM_MLP_FP32) or BF16 (FCM_MLP_BF16) arithmetic.  Device buffers,
 * caller-owned; count >= 1.  Enqueued, not waited for. */
int fcm_mlp_forward(fcm_mlp* net, const float* d_hist, int32_t count, float* d_out, int32_t precision);

/* Loss and gradient at the current parameters on one batch (no update):
 * *loss = sum (y - t)^2 / (count C); grad (host, may be NULL) receives the
 * flat gradient.  d_target[count][C] holds centroids / 255.  Grows the
 * workspace if count exceeds it; waits for the stream. */
int fcm_mlp_loss_grad(fcm_mlp* net, const float* d_hist, const float* d_target, int32_t count, double* loss,
                      float* grad);

/* Train on d_hist[count][256], d_target[count][C] (device): cfg->epochs
 * epochs of shuffled minibatches, one Adam step each.  epoch_loss (host,
 * cfg->epochs doubles, may be NULL) receives the mean training loss of every
 * epoch.  Waits for the stream. */
int fcm_mlp_train(fcm_mlp* net, const float* d_hist, const float* d_target, int32_t count, const fcm_train_cfg* cfg,
                  double* epoch_loss);

void fcm_mlp_destroy(fcm_mlp* net);

/* Persistence of a trained network (the warm start's only learned state).
 * File layout, little-endian: a 64-byte header
 *   char     magic[8]   "FCMMLP01"
 *   uint32_t version    1
 *   uint32_t dtype      0 (FP32 parameters)
 *   int32_t  n_in, h1, h2, C   256, 128, 64, C
 *   int64_t  n_params   fcm_mlp_param_count(C)
 *   uint64_t seed       the seed the network was created with
 *   uint64_t layout     FNV-1a 64 hash of the eight 32-bit words version, dtype,
 *                       n_in, h1, h2, C, low and high half of n_params
 *   uint64_t checksum   FNV-1a 64 hash of the parameter bytes
 * followed by the n_params FP32 values of the flat vector (the order of
 * fcm_mlp_get_params).  The Adam state is not saved.
 * fcm_mlp_save writes the file (through a temporary file renamed over path,
 * so a reader never sees half a file) and waits for the network's stream.
 * Errors: FCM_EINVAL (null arguments), FCM_EIO (the file cannot be written).
 * fcm_mlp_load replaces the parameters of a network with the same C (and, as
 * fcm_mlp_set_params, clears its Adam state); it takes the file's seed.
 * Errors: FCM_EINVAL (null arguments, or the file's C differs from the
 * network's), FCM_EIO (unreadable or truncated file, wrong magic, version,
 * dtype, layer sizes, layout hash or checksum); the network is unchanged on
 * error. */
int fcm_mlp_save(fcm_mlp* net, const char* path);
int fcm_mlp_load(fcm_mlp* net, const char* path);

/* Normalised 256-bin histograms (each row sums to 1) of the instances
 * d_x[offsets[i] .. offsets[i+1]) (offsets: count + 1 host values, starting
 * at 0, non-decreasing, every instance non-empty) into d_hist[count][256].
 * Allocates and frees temporaries; waits for the stream. */
int fcm_histogram(const uint8_t* d_x, const int64_t* offsets, int32_t count, float* d_hist, void* stream);

/* fcm_histogram for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * arguments, results and wait, but its workspace (the instance offsets and the
 * counters) lives in a fixed array of about 1 MiB in the library's device
 * memory, one per device for the life of the process, so the call allocates
 * nothing.  At most 1,024 instances per call: FCM_EINVAL beyond that (see
 * fcm_last_error).  The counters are cleared by a kernel at every call.  Calls
 * on one device share the array, so two calls that overlap in time on one
 * device (other threads, other streams) race: serialise them. */
int fcm_histogram_noalloc(const uint8_t* d_x, const int64_t* offsets, int32_t count, float* d_hist, void* stream);

/* Start centroids from histograms: BF16 inference, then v = 255 y sorted
 * ascending, clamped to the instance's grey-level range [lo, hi] (read off
 * its histogram), consecutive gaps of at least 1.  d_v0[count][C] doubles
 * (device); a row is NaN where no such set exists (non-finite output, or
 * fewer than C grey levels in the range), which FCM_INIT_DEVICE reads as
 * "use the evenly spaced start".  Grows a scratch buffer if needed; enqueued
 * on the stream, not waited for. */
int fcm_warm_centroids(fcm_mlp* net, const float* d_hist, int32_t count, double* d_v0, void* stream);

/* Warm-started solve on a handle (whose C must equal the network's): the
 * histogram of the handle's input, the network's start centroids, then
 * Algorithm 1 from them, all on the handle's stream; the handle afterwards
 * holds that solve (labels, trajectory).  check != 0: also solve from the
 * handle's own start (the plain result, copied to *plain if non-NULL) and
 * keep the warm result only if J_warm <= J_plain (1 + 1e-6); otherwise the
 * plain solve is run again so that the handle holds it, and *used = 0.
 * used (may be NULL): 1 if the returned result is the warm-started one.
 * The first call allocates a small workspace (histogram, start). */
int fcm_solve_warm(fcm_handle* h, fcm_mlp* net, int32_t check, fcm_result* out, fcm_result* plain, int32_t* used);

/* Start of each batch instance for the following fcm_batch_solve calls:
 * instance i takes the network's start centroids if net != NULL, its C
 * equals the network's, and use_learned (count host flags, NULL = all) is
 * nonzero for it; every other instance takes its own init from
 * fcm_batch_init.  Computes the histograms and runs the network on the
 * batch's stream (allocating their buffers on the first call). */
int fcm_batch_set_start(fcm_batch* b, fcm_mlp* net, const uint8_t* use_learned);

/* Warm-started batch solve with the fall-back rule of fcm_solve_warm, per
 * instance.  check != 0: every instance is first solved from its own start
 * (the plain results, copied to plain[count] if non-NULL); then the instances
 * whose C equals the network's are solved from the network's start; warm
 * instance i is kept only if its status is not FCM_ENUMERIC and J_warm <=
 * J_plain (1 + 1e-6), and every instance that falls back is solved again from
 * its own start in one final launch, so that labels and trajectories match the
 * returned results.  check == 0: one launch from the learned starts.  out
 * (count records) receives the returned results, used (count host bytes, may
 * be NULL) 1 where the warm-started result is returned.  The batch keeps the
 * starts of the returned results for later fcm_batch_solve calls
 * (fcm_batch_set_start(b, NULL, NULL) restores the instances' own starts).
 * Returns as fcm_batch_solve.  The plain start is the judge (Algorithm 1 from
 * the instance's own v^0); the network only proposes v^0. */
int fcm_batch_solve_warm(fcm_batch* b, fcm_mlp* net, int32_t check, fcm_result* out, fcm_result* plain,
                         uint8_t* used);

/* Training targets of the network from the last fcm_batch_solve:
 * d_target[i * C + k] = the k-th smallest centroid of instance i's v^T,
 * divided by 255 in FP64 and rounded to FP32 (the network's output scale).
 * d_target: device, count * C floats, caller-owned.  Every instance must
 * have C clusters (FCM_EINVAL otherwise); FCM_ESTATE before a solve.
 * Enqueued on the batch's stream, not waited for. */
int fcm_batch_targets(fcm_batch* b, int32_t C, float* d_target);

/* ---- segmentation quality (Sec. 5.2.2, Eq.5) ----------------------------- */

/* Confusion counts of two label images over n voxels (device, any alignment):
 * d_counts[j * n_truth + k] = number of voxels with d_pred == j and
 * d_truth == k, and d_counts[n_pred * n_truth] = number of voxels whose pred
 * or truth value lies outside [0, n_pred) or [0, n_truth).  d_counts is a
 * device array of n_pred * n_truth + 1 counters, cleared by the call.
 * 1 <= n_pred, n_truth <= 16; n >= 0 (n = 0 leaves all counts zero).
 * Enqueued on the stream, not waited for. */
int fcm_confusion(const uint8_t* d_pred, const uint8_t* d_truth, int64_t n, int32_t n_pred, int32_t n_truth,
                  uint64_t* d_counts, void* stream);

/* Dice similarity coefficient per ground-truth class (Eq.5) from confusion
 * counts made by fcm_confusion: cluster j is counted as class class_of[j]
 * (host, n_pred values in [-1, n_truth), -1 = no class; NULL maps cluster j
 * to class j where j < n_truth).  d_dsc (device, n_truth doubles) receives
 * 2 |PR_k and GT_k| / (|PR_k| + |GT_k|), rounded once from the exact counts,
 * or NaN where both sets are empty.  Enqueued on the stream, not waited for. */
int fcm_dice(const uint64_t* d_counts, int32_t n_pred, int32_t n_truth, const int32_t* class_of, double* d_dsc,
             void* stream);

/* ---- the paper's GPU design, as a baseline (Sec. 4) -------------------------- */

typedef struct fcm_paper_stats {
    double  total_ms;    /* the iteration loop, host wall clock */
    double  kernels_ms;  /* device time of the per-cluster kernels (HIP events) */
    double  copy_ms;     /* device-to-host copies of U and v after each iteration */
    double  host_ms;     /* the host's stopping tests */
    int64_t launches;    /* kernel launches in the loop (5 C per iteration) */
} fcm_paper_stats;

/* Solve with the structure the paper gives its GPU implementation (Sec. 4):
 * U (C x n, FP32) in device memory; per iteration and cluster a per-pixel
 * kernel for the Eq.3 terms, two Algorithm 2 reductions (128 threads per
 * block, n / 256 partial sums), a one-thread kernel for the final sums (FP64)
 * and the centroid; per cluster a per-pixel Eq.4 kernel; then U is copied to
 * the host, which tests max |U^t - U^(t-1)| < eps.  Defuzzification on the
 * host.  Starts: FCM_INIT_RANDOM_U (the paper's: U^0 drawn on the host from
 * the same SplitMix64 stream as the fused solver's), FCM_INIT_LINSPACE or
 * FCM_INIT_GIVEN (U^0 = Eq.4 at v^0).  d_x: n device bytes.  Host outputs, each
 * may be NULL: v_hist[(max_iter + 1) * C] (v^t for t = 0..T; v^0 NaN for the
 * random start), delta_hist[max_iter + 1] (delta^t, delta^0 NaN), labels[n].
 * out->J is NaN (the design computes no objective).  Allocates and frees its
 * own buffers (U on the device, two pinned host copies of U); synchronous.
 * A baseline for measurement, not a fast path. */
int fcm_paper_solve(const uint8_t* d_x, int64_t n, const fcm_params* p, void* stream, fcm_result* out,
                    double* v_hist, double* delta_hist, uint8_t* labels, fcm_paper_stats* stats);

/* Static description of a status code, and the last HIP error text of this thread. */
const char* fcm_strerror(int status);
const char* fcm_last_error(void);

/* Library version, as major * 10000 + minor * 100 + patch. */
int fcm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FCM_H */
