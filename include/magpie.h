/*
 * magpie.h -- C ABI of the MI355X (gfx950) MAGPIE ptychography hot path.
 *
 * MAGPIE (arXiv 2504.10118) reconstructs a complex object z (n_rows x n_cols)
 * from far-field intensities d_k = |F(Q * P_k z)|^2 measured at N scan
 * positions (Section 2.1, problem statement), by minimising the exit-wave
 * misfit of eq. (2.1) with the stochastic multigrid surrogate solver of
 * Alg 4 (MAGPIE), whose per-position step is the V-cycle of Alg 3 (MAGPS).
 * This library runs that solver with minibatches of positions on one GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status: MAGPIE_OK (0) or a negative
 *   MAGPIE_ERR_* code.  magpie_last_error() returns a message describing
 *   the last failure on the calling thread (valid until the next failing
 *   call on that thread).  On error no output argument is written unless
 *   stated otherwise.
 * - Complex arrays are interleaved (re, im), row-major, i.e. the memory
 *   layout of torch.complex64 (MAGPIE_C64) or torch.complex128 (MAGPIE_C128).
 * - The 2-D DFT F is unnormalised with kernel exp(-2 pi i (a y + b x) / m)
 *   and zero frequency at index [0][0] (no fftshift); F^{-1} = F^* / m^2.
 * - Host pointers (on_device = 0) are read or written before the call
 *   returns.  Device pointers (on_device = 1, e.g. torch's data_ptr() on the
 *   same device) are used in stream order on the context's stream: inputs
 *   must stay valid and unmodified until the next call that synchronises the
 *   stream (any get_* into host memory, magpie_objective, magpie_sync,
 *   magpie_destroy).  The library never frees caller memory.
 * - A context owns all device memory it allocates and releases it in
 *   magpie_destroy.  A context is not thread-safe; distinct contexts are
 *   independent.
 * - Call order: magpie_create -> magpie_set_probe -> magpie_set_positions ->
 *   magpie_load_intensities -> [magpie_set_object] -> magpie_run_epochs ...
 *   Out-of-order calls return MAGPIE_ERR_BAD_STATE.  The initial object is
 *   all ones.
 */
#ifndef MAGPIE_H
#define MAGPIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MAGPIE_OK               0
#define MAGPIE_ERR_INVALID_ARG (-1)  /* null/out-of-range argument, bad offsets */
#define MAGPIE_ERR_BAD_STATE   (-2)  /* call made before its prerequisites */
#define MAGPIE_ERR_OOM         (-3)  /* device or pinned-host allocation failed */
#define MAGPIE_ERR_HIP         (-4)  /* a HIP runtime call failed */
#define MAGPIE_ERR_NUMERIC     (-5)  /* non-finite value found in inputs or objective */
#define MAGPIE_ERR_UNSUPPORTED (-6)  /* m not in {8,16,32,64,128}, bad level count */

/* complex element types */
#define MAGPIE_C64  0   /* float  (re, im) */
#define MAGPIE_C128 1   /* double (re, im) */

/* flags for magpie_set_flags */
#define MAGPIE_UPDATE_PROBE 0x1u  /* also update the probe each minibatch (beyond the paper) */
#define MAGPIE_GRAPH        0x2u  /* replay a captured per-epoch hipGraph instead of
                                     launching each kernel directly (same results) */
#define MAGPIE_PHASE_RECYCLE 0x4u /* eq. (3.2): where F(Q z_k) vanishes exactly, take the
                                     phase of position k's previous visit instead of 0 */
#define MAGPIE_PROBE_ALTERNATE 0x8u /* with MAGPIE_UPDATE_PROBE: take the probe step at the
                                     minibatch's updated object (alternating half steps)
                                     instead of at the object the step started from */
#define MAGPIE_PERSISTENT   0x10u /* run epochs as one work-queue launch per plan
                                     partition and chunk of epochs (see
                                     magpie_run_epochs_multi); same results bit for bit */

typedef struct magpie_ctx magpie_ctx;

/* Message for the last failing call on this thread ("" if none). */
const char* magpie_last_error(void);

/*
 * Create a reconstruction context on HIP device `device`.
 *   n_rows, n_cols : object size (>= m each); the object's n_rows * n_cols
 *                    complex64 values must take fewer than 2^32 bytes (the
 *                    kernels address it through 32-bit buffer ranges), else
 *                    MAGPIE_ERR_UNSUPPORTED.
 *   m              : probe / patch side; one of 8, 16, 32, 64, 128.
 *   n_levels       : number of grids of the MAGPS V-cycle (Alg 3): the fine
 *                    grid plus n_levels-1 coarse grids, 1 <= n_levels <=
 *                    log2(m)+1.  n_levels = 1 is rPIE (Alg 1, eq. 2.3).
 *   alpha          : rPIE constant of u = alpha (max|Q|^2 - |Q|^2)
 *                    (Section 2.1, the u^rPIE definition; Section 5), >= 0.
 *   hip_stream     : hipStream_t to run on, or NULL to create a private one.
 * Errors: INVALID_ARG, UNSUPPORTED, HIP, OOM.
 */
int magpie_create(magpie_ctx** out, int n_rows, int n_cols, int m, int n_levels,
                  double alpha, int device, void* hip_stream);

/* Synchronise the stream and release every device allocation.  NULL is a no-op. */
int magpie_destroy(magpie_ctx* ctx);

/*
 * Set the probe Q (m x m complex, dtype MAGPIE_C64 or MAGPIE_C128) and build
 * the level hierarchy of Alg 3 in FP64 on the device: Q_{l+1} = I_h^H Q_l,
 * the weights of eq. (4.4), u_{l+1} = W_u^H (I_h^H u_l), and the per-level
 * coefficients of the gradient form of the coarse step (eq. 4.6).  The
 * regularisation is reset to u^rPIE with the context's alpha.
 * Errors: INVALID_ARG (null, Q identically zero), NUMERIC (non-finite), HIP.
 */
int magpie_set_probe(magpie_ctx* ctx, const void* probe, int dtype, int on_device);

/*
 * Replace the fine-grid regularisation vector (Section 2.1, eq. 2.4).
 * u == NULL: u = alpha (max|Q|^2 - |Q|^2) (u^rPIE).  Otherwise u is a host
 * array of m*m doubles >= 0.  Coarse-level vectors follow automatically
 * (Prop 4.4).  Requires a probe.  Errors: INVALID_ARG, BAD_STATE, HIP.
 */
int magpie_set_regularization(magpie_ctx* ctx, double alpha, const double* u);

/*
 * Scan positions: offsets is a host array [n_pos][2] of int32 (row, col)
 * top-left corners of the m x m windows P_k (Section 2.1), with
 * 0 <= row <= n_rows - m and 0 <= col <= n_cols - m.  Resets loaded
 * intensities.  Errors: INVALID_ARG (bounds, n_pos < 1), OOM, HIP.
 */
int magpie_set_positions(magpie_ctx* ctx, int n_pos, const int32_t* offsets);

/*
 * Measured data d_k of the problem statement (Section 2.1: the far-field
 * intensities |F(Q * P_k z)|^2 recorded at scan position k), float32
 * [n_pos][m][m], zero frequency at [0][0], in the order of the positions.
 * Host data are copied before the call returns; device data are read in
 * stream order (see the conventions above).
 * is_sqrt = 0: intensities d_k (>= 0), the library takes square roots;
 * is_sqrt = 1: amplitudes sqrt(d_k).  Stored internally in the order the
 * kernels consume.  Errors: BAD_STATE (no positions), INVALID_ARG, HIP.
 */
int magpie_load_intensities(magpie_ctx* ctx, const float* d, int is_sqrt, int on_device);

/*
 * Set the object z (n_rows x n_cols complex, dtype MAGPIE_C64 or MAGPIE_C128):
 * the initial guess z^(0) that Alg 4 (MAGPIE) takes as input, or any later
 * iterate to resume from.  Stored as complex64.  Errors: INVALID_ARG (null,
 * bad dtype), NUMERIC (non-finite values), HIP.
 */
int magpie_set_object(magpie_ctx* ctx, const void* z, int dtype, int on_device);

/*
 * Run n_epochs epochs of minibatch MAGPIE (Alg 4 with the minibatch
 * combination): each epoch draws a uniformly random permutation of the
 * positions and cuts it into consecutive minibatches of `batch` positions
 * (the last one shorter).  In a minibatch every position reads the same z,
 * computes its revised exit wave (Definition 2.1) and its MAGPS update
 * dz_k (Alg 3), and the object becomes
 *     z <- z + sum_k P_k^T (w0 dz_k) / sum_k P_k^T w0,   w0 = u + |Q|^2,
 * on pixels covered by the minibatch.  batch = 1 is Alg 4 exactly.
 *   order : NULL -> permutations from splitmix64-driven Fisher-Yates seeded
 *           with seed XOR epoch_index (epoch_index counts epochs run on this
 *           context); otherwise a host array [n_epochs][n_pos] of
 *           permutations of 0..n_pos-1, used as given.
 * Asynchronous: returns after enqueuing.  Errors: BAD_STATE, INVALID_ARG
 * (batch < 1, order not a permutation), HIP.
 */
int magpie_run_epochs(magpie_ctx* ctx, int n_epochs, int batch, uint64_t seed,
                      const int32_t* order);

/*
 * One minibatch step (the inner step of magpie_run_epochs) over exactly the
 * `count` distinct positions listed in `positions` (host int32 array of indices
 * in [0, n_pos)): every listed position reads the same z and
 *     z <- z + sum_k P_k^T (w0 dz_k) / sum_k P_k^T w0
 * on the pixels they cover.  With one position this is one update of Alg 4.
 * The epoch counter is not advanced and no graph is used.  Asynchronous.
 * Errors: BAD_STATE, INVALID_ARG (count out of range, repeated or invalid
 * index), OOM, HIP.
 */
int magpie_run_minibatch(magpie_ctx* ctx, int count, const int32_t* positions);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the epochs of
 * magpie_run_epochs with order = NULL (the library's seeded permutations, seed
 * XOR epoch counter), with the same results bit for bit, without any device or
 * pinned-host allocation.  The per-call buffers (the minibatch staging, 8 m^2
 * bytes per position of a minibatch, and each epoch's position records and
 * inverse permutation, 20 bytes per position) live in a 16 MiB device array of
 * the library, one per GPU, held until the process ends; its address is resolved
 * when a context is created on that GPU.  Epochs are processed in chunks whose
 * records fit beside the staging; their permutations are drawn on the device.
 * Nothing in the array needs to start cleared, and it keeps the last call's
 * contents: calls that overlap on one GPU (contexts on different streams) race
 * and must be serialised by the caller.  MAGPIE_GRAPH is ignored (kernels are
 * launched directly) and timing is not recorded.  Asynchronous.
 * Errors: INVALID_ARG, BAD_STATE, UNSUPPORTED (MAGPIE_UPDATE_PROBE set; more
 * than 16384 positions; staging plus one epoch's records above 16 MiB), HIP.
 */
int magpie_run_epochs_noalloc(magpie_ctx* ctx, int n_epochs, int batch, uint64_t seed);

/*
 * Objective pass over all positions at the current object (eq. 2.1, reported
 * in exit-wave form (1 / (2 m^2)) sum_k || |F(Q z_k)| - sqrt(d_k) ||^2),
 * reduced in FP64 in a fixed order.  grad_stat (nullable) receives the
 * stopping statistic (1 / (N m)) sum_k ||conj(Q)(Q z_k - R_k(z_k))||_2
 * (Section 5, "Stopping criterion").  Synchronises.
 * Errors: BAD_STATE, NUMERIC (non-finite objective), HIP.
 */
int magpie_objective(magpie_ctx* ctx, double* phi, double* grad_stat);

/*
 * Per-position objective terms Phi_k (eq. 2.1's term of position k; [n_pos],
 * returned as FP64) at the object as it was when each position was last visited
 * by magpie_run_epochs (NaN if never).  Summed by the step itself: per thread in
 * FP32 over at most 16 spectrum values, then in FP64 (about 1e-6 relative; use
 * magpie_objective for the FP64 objective).  Host output; synchronises.
 */
int magpie_get_step_phi(magpie_ctx* ctx, double* phi_k);

/*
 * Copy out the current iterate z^(j) of Alg 4 (magpie_get_object; n_rows x
 * n_cols) or the probe Q (magpie_get_probe; m x m: the one set, or the
 * updated one with MAGPIE_UPDATE_PROBE), as dtype C64 or C128, into caller
 * memory (host, or device with on_device = 1, written in stream order).
 * Host outputs synchronise the stream.  Errors: INVALID_ARG, HIP.
 */
int magpie_get_object(magpie_ctx* ctx, void* out, int dtype, int on_device);
int magpie_get_probe(magpie_ctx* ctx, void* out, int dtype, int on_device);

/* Wait for all work enqueued on the context's stream. */
int magpie_sync(magpie_ctx* ctx);

/* Set behaviour flags (MAGPIE_UPDATE_PROBE, MAGPIE_GRAPH, MAGPIE_PHASE_RECYCLE).
 * beta: probe-step proximal weight.  With MAGPIE_GRAPH (and timing off) an epoch
 * is one replay of a hipGraph captured on first use for the current minibatch
 * size; the graph reads the epoch's permutation through a device counter.
 * MAGPIE_PHASE_RECYCLE (Section 3.1, eq. 3.2) keeps the phase of F(Q z_k) of
 * every position's last visit in device memory the context owns (n_pos * m * m
 * complex64, natural order) and uses it wherever F(Q z_k) is exactly zero
 * (theta = 0 before a position's first visit).  The store starts over (theta =
 * 0 everywhere) when the flag is switched on, on magpie_set_positions and on
 * magpie_load_intensities; magpie_set_object keeps it.  Only object steps use
 * it (the objective and its stopping statistic keep theta(0) = 0); the
 * autotuner's trial epochs leave it untouched, and magpie_run_epochs_multi
 * rejects contexts with this flag (MAGPIE_ERR_UNSUPPORTED).
 * MAGPIE_PROBE_ALTERNATE (only together with MAGPIE_UPDATE_PROBE, else
 * MAGPIE_ERR_INVALID_ARG): the probe step of each minibatch is taken after its
 * object update, at the new object, by a second pass of the step kernel over the
 * minibatch; each half step then minimises its proximal surrogate in its own
 * variable (Lemma C.1 in z, then in Q), so with one grid the minibatch's partial
 * objective does not increase.  Costs one more step-kernel launch per minibatch. */
int magpie_set_flags(magpie_ctx* ctx, uint32_t flags, double beta);

/*
 * Forward model (Section 2.1): d_k = |F(Q * P_k z)|^2 for every position, at
 * the given object z (n_rows x n_cols, dtype C64, host or device) with the
 * context's probe and positions, written to d_out float32 [n_pos][m][m]
 * (zero frequency at [0][0]).  Errors: BAD_STATE, INVALID_ARG, HIP.
 */
int magpie_forward_model(magpie_ctx* ctx, const void* z, int z_on_device,
                         float* d_out, int out_on_device);

/*
 * The library's epoch permutation: Fisher-Yates over 0..n-1, for
 * i = n-1 .. 1 swapping entries i and (next mod (i+1)), where next are the
 * outputs of splitmix64 (Steele, Lea & Flood 2014) started from state
 * seed XOR epoch.  Host output [n].  Errors: INVALID_ARG.
 */
int magpie_permutation(uint64_t seed, uint64_t epoch, int n, int32_t* out);

/* Number of epochs run so far on this context (drives the seeded permutations). */
int magpie_get_epoch_index(magpie_ctx* ctx, uint64_t* epoch_index);
int magpie_set_epoch_index(magpie_ctx* ctx, uint64_t epoch_index);

/*
 * Kernel timing for measurement.  While enabled, magpie_run_epochs brackets
 * every launch of the per-position step kernel and of the accumulation
 * kernel with HIP events on the context's stream.  magpie_get_timing
 * synchronises, returns the summed event times (milliseconds), the number
 * of launches of each kernel and the number of positions processed by the
 * step kernel since timing was last read or enabled, and resets the sums.
 * Errors: INVALID_ARG, HIP.
 */
int magpie_set_timing(magpie_ctx* ctx, int enable);
int magpie_get_timing(magpie_ctx* ctx, double* step_ms, double* accum_ms, int64_t* step_launches,
                      int64_t* accum_launches, int64_t* positions);

/*
 * The recorded launches of one kernel (kind 0: step kernel, 1: accumulation
 * kernel) since timing was last read or enabled, without resetting them:
 * per-launch durations in microseconds (us) and the positions of each step
 * launch (positions; 0 for the accumulation), at most cap entries each, in launch
 * order.  Synchronises.  Returns the number of recorded launches of that kind
 * (which may exceed cap) or a negative error code.  Errors: INVALID_ARG, HIP.
 */
int magpie_get_launch_times(magpie_ctx* ctx, int kind, double* us, int32_t* positions, int cap);

/*
 * Kernel variants (no effect on the mathematics; results agree to FP32
 * rounding).  The step kernel's FFT plan is the number of threads per 1-D
 * transform (each thread then holds m / threads points); the accumulation
 * kernel works on object tiles of 32 columns x tile_rows rows (8, 16 or
 * 32).
 * magpie_list_plans writes the compiled plans of m (default first) and
 * returns their count.  magpie_set_tuning (0 = keep) changes them, moving the
 * loaded sqrt(d) to the new plan's order.  Errors: UNSUPPORTED, INVALID_ARG.
 */
int magpie_list_plans(int m, int32_t* threads_per_transform, int cap);
int magpie_set_tuning(magpie_ctx* ctx, int threads_per_transform, int tile_rows);
int magpie_get_tuning(magpie_ctx* ctx, int* threads_per_transform, int* tile_rows);

/*
 * Autotuner: times trial_epochs epochs of minibatch size `batch` with every
 * compiled FFT plan (step kernel) and then every tile height (accumulation
 * kernel), each after one untimed epoch of the same variant, keeps the fastest
 * of each, and restores the object and the epoch counter (the trials' updates
 * are discarded).  Outputs (nullable): mean
 * per-launch times in microseconds of the chosen variants.
 * Errors: BAD_STATE, INVALID_ARG, HIP.
 */
int magpie_autotune(magpie_ctx* ctx, int batch, int trial_epochs, double* step_us, double* accum_us);

/*
 * Minibatch autotuner.  The minibatch size B is a parameter of the method (the
 * paper's Alg 4 visits positions one at a time; a minibatch combines B surrogate
 * minimisations, and its Conclusion leaves the minibatch variant open): a larger
 * B makes an epoch cheaper on the GPU but each epoch reduces the objective less.
 * For each of the n_candidates sizes, from the object and epoch counter the call
 * started with, runs trial_epochs epochs of minibatch MAGPIE (the library's
 * permutations for a fixed seed and the context's epoch counter, the same for
 * every candidate) and measures the wall time of those epochs
 * (records drawn on the host included, objective passes excluded) and the
 * objective (eq. 2.1) before and after; a candidate's rate is the objective's
 * decrease per second.  Keeps the candidate with the largest rate in *best_batch,
 * restores the object and the epoch counter, and writes the rates (nullable,
 * n_candidates doubles, objective units per second; negative where the objective
 * rose).  Positions beyond N count as N.  Synchronises.
 * Errors: BAD_STATE, INVALID_ARG (no candidates, a candidate < 1, trial_epochs < 1,
 * NULL best_batch), NUMERIC (non-finite objective), OOM, HIP.
 */
int magpie_autotune_batch(magpie_ctx* ctx, const int32_t* candidates, int n_candidates, int trial_epochs,
                          int32_t* best_batch, double* rates);

/*
 * Many independent reconstructions (contexts of any sizes on one device)
 * advanced together: each context runs n_epochs epochs of minibatch MAGPIE
 * with its own minibatch size batch[i] and its own seeded permutations
 * (seed XOR its epoch counter), exactly as magpie_run_epochs would.  The
 * contexts are partitioned by FFT plan (a plan of 1024-thread workgroups, one
 * per compute unit, into two partitions of about equal work), each partition
 * on a stream of its own.  Within a partition, rounds pair the t-th minibatches
 * of its contexts still running: one step-kernel launch and one accumulation
 * launch per tile height cover every context of the round.  Runs on the first
 * context's stream (the other streams fork from it and join it, and the other
 * contexts' streams are joined with events) and synchronises it.  The probe step is not available
 * here.  Errors: INVALID_ARG, BAD_STATE, UNSUPPORTED, OOM, HIP.
 */
int magpie_run_epochs_multi(magpie_ctx* const* ctxs, int count, int n_epochs, const int* batch, uint64_t seed);
/*
 * With MAGPIE_PERSISTENT set on every context of the call (or on none: mixing
 * is INVALID_ARG), the rounds of each chunk of up to 8 epochs run as one
 * work-queue launch per plan partition instead of two or more launches per round
 * (the batched, persistent execution of many reconstructions; the paper leaves
 * the minibatch/GPU variant of Alg 4 to future work).  Workgroups, as many as
 * are resident, take items in queue order: for each round, one per position of
 * every context's minibatch (the step), then one per accumulation tile of every
 * context (tile height m * threads_per_transform / 32, which gives the same
 * sums: the summation order does not depend on the tile).  A step waits for its
 * context's tiles of earlier rounds, a tile for its context's steps so far;
 * data handed between workgroups is read and written at device scope.  Results
 * are identical to those without the flag.  magpie_run_epochs with the flag set
 * runs its context this way (caller orders: UNSUPPORTED).  A wait that exceeds
 * its bound (2 s of the device clock; the environment variable
 * MAGPIE_QUEUE_WAIT_US overrides it, in microseconds) stops the queue: the call
 * returns MAGPIE_ERR_HIP and the objects are left part-way.  UNSUPPORTED: a
 * context's FFT plan with fewer than 64 threads (m = 8, and m = 16 at 2
 * threads per transform) or a minibatch of more than 256 positions.
 */

#ifdef __cplusplus
}
#endif

#endif /* MAGPIE_H */
