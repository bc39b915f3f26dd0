/*
 * perm_est.h -- C ABI of the MI355X sparse-permanent estimator.
 *
 * The library runs many independent sequential-importance-sampling
 * trajectories of the generic adaptive estimator of "The Quick and the
 * Dead: Estimating Sparse-Matrix Permanents with Adaptive Work Filtering"
 * (Alg. 2; Alg. 1 with the row-order rule and no scaling) on one AMD
 * Instinct MI355X (gfx950) and returns the estimate of per(A), Eq. (per1),
 * together with the per-trajectory log-weights and the statistics of
 * Sec. 2 and Sec. 4 "Metrics".
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status: PE_OK (0) or a negative PE_E*
 *     code; none throws or aborts.  perm_est_last_error() gives a message
 *     for the most recent failure in the calling thread.
 *   - Matrix input arrays are HOST pointers owned by the caller; they are
 *     validated and copied to the device by perm_est_create and may be
 *     freed afterwards.
 *   - Per-trajectory output arrays are DEVICE pointers (for example the
 *     data_ptr() of torch tensors on the handle's device) owned by the
 *     caller; any of them may be NULL.  The result struct is a host pointer.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it and the call returns after the stream has finished
 *     the work it enqueued, so outputs are ready on return.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Results are a pure function of (matrix, schedule, seed, trajectory
 *     index): trajectory k always draws its random numbers from
 *     Philox4x32-10 with key = seed and counter = (k, b, t, d) where b is
 *     the matrix index (0 for a single matrix), t the step and d the draw.
 *   - "No perfect matching" is not an error: the run returns PE_OK with
 *     p_match = 0, log_estimate = -inf and every trajectory dead.
 */
#ifndef PERM_EST_H
#define PERM_EST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PE_OK 0
#define PE_EINVAL (-1)   /* bad argument: n <= 0, index out of range,
                            unsorted or duplicate entries, CSR/CSC mismatch,
                            non-positive value, unknown preset, bad schedule */
#define PE_ENOMEM (-2)   /* device or host allocation failed               */
#define PE_EDEVICE (-3)  /* a HIP call failed (message has the HIP error)  */
#define PE_ENOTSUP (-4)  /* valid request this build does not implement,
                            e.g. a degree above 65534                        */
#define PE_EIO (-5)      /* a file could not be opened, read or written     */

/* vertex selection rule R_V (Alg. 2 input; Sec. 3.2) */
#define PE_VR_MD 0        /* two-sided minimum degree over rows and columns,
                             ties to the smallest vertex id (rows 0..n-1
                             before columns n..2n-1)                        */
#define PE_VR_ROW_ORDER 1 /* rows in index order (Alg. 1)                   */

/* scaling policy P_SK (Sec. 3.3) */
#define PE_SK_NONE 0      /* outer scaling only (or none if K0 = 0)         */
#define PE_SK_FIXED 1     /* K full SK iterations on every child            */
#define PE_SK_ADAPTIVE 2  /* ceil((1 - z) K) full iterations, clamped [0,K] */
#define PE_SK_LOCAL 3     /* one local Jacobi repair per step, Eq. (local)  */
#define PE_SK_LEARNED 4   /* learned per-edge proposal in place of the
                             scaling scores of Eq. (q); no inner SK.  Needs
                             perm_est_set_model on the handle first         */

/* support-filtering policy P_DM (Sec. 3.3) */
#define PE_DM_NONE 0
#define PE_DM_ALL 1       /* DM on every child                              */
#define PE_DM_THRS 2      /* DM when z < theta_th                           */
#define PE_DM_TRCK 3      /* track *= z; DM when track < theta_tr, then 1   */

typedef struct perm_est perm_est_t; /* opaque; owns all device state */

/* option flags */
#define PE_FLAG_FORCE_HBM 1u  /* keep per-trajectory state in HBM scratch even
                                 when it would fit in LDS (results are
                                 identical; used to cross-check the tiers) */
#define PE_FLAG_WAVE_PER_TRAJECTORY 2u
                              /* run every trajectory on a whole wave; by
                                 default a single matrix in HBM scratch under
                                 the plain or learned proposal (no inner SK or
                                 DM, minimum degree) runs four trajectories per
                                 wave.  Results are identical either way     */

typedef struct {
    int32_t device;  /* HIP device ordinal                                 */
    uint32_t flags;  /* PE_FLAG_* bits; other bits must be 0               */
} perm_est_options;

/* Inputs of Alg. 2: R_V, K0, K, P_SK, P_DM and the two thresholds, plus
 * whether the shared initial DM filter (Alg. 2 preprocessing) runs. */
typedef struct {
    int32_t vertex_rule;  /* PE_VR_*                                        */
    int32_t sk_policy;    /* PE_SK_*                                        */
    int32_t dm_policy;    /* PE_DM_*                                        */
    int32_t initial_dm;   /* 1 = filter unsupported entries once, shared    */
    int32_t K0;           /* outer SK iterations (>= 0)                     */
    int32_t K;            /* inner SK cap (>= 0)                            */
    double theta_th;      /* Thrs threshold                                 */
    double theta_tr;      /* Trck threshold                                 */
    int32_t local_gate;   /* PE_SK_LEARNED only: 1 = gated local-repair
                             fallback.  The trajectory keeps its own r, c
                             (from the outer scaling); after a step whose
                             sampled probability z = w_u / sum w is below
                             theta_th, or after an inner DM call, it repairs
                             them by Eq. (local) (Sec. 3.3, Local policy),
                             and the next step draws from the scaled
                             proposal of Eq. (q) with z = r_rho c_gam
                             instead of the network.  0 = network only    */
    int32_t local_cap;    /* local repair (PE_SK_LOCAL, or the gated learned
                             fallback; else must be 0): 0 = Eq. (local)
                             exactly; B in [1, 65535] = bounded work for hub
                             vertices (Sec. 3.3 proposes it): a list of
                             L > B entries is examined at the B positions
                             (o + floor(k L / B)) mod L, k = 0..B-1, with
                             o = floor(R L / 2^32), R the low 32 bits of the
                             trajectory's draw (step t, draw 2^31 + vertex
                             id); its active entries stand for the vertex's
                             child neighbourhood in the two-hop sets, and
                             its new value is 1 / (sampled sum * residual
                             degree / sampled active count) (unchanged when
                             nothing active was sampled).  Lists of at most
                             B entries are used whole                     */
    int32_t reserved[2];  /* must be 0                                      */
} perm_est_schedule;

typedef struct {
    double log_estimate;  /* ln of the sample mean of X; -inf if none alive */
    double p_match;       /* fraction of trajectories with X > 0            */
    double rel_spread;    /* sd(X) (M-1 denominator) / |mean|, zeros incl.  */
    double rse;           /* rel_spread / sqrt(M)                           */
    double ess;           /* (sum X)^2 / sum X^2                            */
    double var_logw;      /* sample variance of ln X over the survivors     */
    double max_logw;      /* largest ln X                                   */
    int64_t n_traj;       /* M                                              */
    int64_t n_alive;
    int64_t n_dm;         /* inner DM calls, summed over trajectories       */
    int64_t n_full_sk;    /* full SK iterations, summed                     */
    int64_t n_local_sk;   /* local repairs, summed                          */
    int64_t n_steps;      /* completed matching steps, summed               */
    double seconds;       /* wall time of the trajectory + reduction work   */
    /* work units, summed over trajectories (drive the byte model) */
    int64_t n_entries_scanned; /* adjacency entries read at v and u         */
    int64_t n_decrements;      /* residual-degree decrements                */
    int64_t n_local_entries;   /* entries gathered or summed by local repair */
    int64_t n_local_values;    /* scaling values recomputed by local repair */
    int64_t n_mlp_tiles;       /* 16-candidate tiles through the learned
                                  proposal's network; where four
                                  trajectories share a wave they share
                                  tiles, so this count depends on the
                                  launch shape (the results do not)         */
    int64_t n_entries_scanned_v; /* the part of n_entries_scanned read at the
                                    selected vertex v                      */
    double kernel_seconds;     /* device time of the trajectory kernel alone
                                  (HIP events on the run's stream); equal to
                                  `seconds` for a replayed graph            */
    /* device time by phase, summed over the trajectories of the launch (each
       trajectory's wave reads the device wall clock; one trajectory per
       wave -- the kernels that run four per wave leave these 0) */
    double wave_seconds;          /* whole trajectories                      */
    double wave_seconds_full_sk;  /* full SK sweeps (Fixed, Adaptive)        */
    double wave_seconds_dm;       /* inner DM calls                          */
    double wave_seconds_local;    /* local repairs                           */
    int64_t n_dm_entries;         /* adjacency entries the inner DM calls
                                     examined (augmentation and SCC)         */
    /* the launch shape used */
    int32_t launch_blocks;            /* persistent workgroups               */
    int32_t launch_waves_per_block;
    int32_t launch_trajectories_per_wave; /* 1, or 4 (16-lane rows)       */
    int32_t launch_blocks_per_cu;     /* resident workgroups per CU the
                                         launch was sized for              */
} perm_est_result;

/* Create a handle for one n x n matrix A given in both CSR and CSC form
 * (Sec. 2, "Support filtering": rows and columns are the two vertex sides
 * of the bipartite graph G_A).
 *   row_ptr[n+1], col_idx[nnz]: CSR, column indices ascending and unique
 *                               within each row;
 *   col_ptr[n+1], row_idx[nnz]: CSC of the same entries, row indices
 *                               ascending within each column;
 *   values[nnz]: entry values in CSR order, all > 0, or NULL for a 0/1
 *                matrix.
 * All arrays are host memory; int32 indices (nnz < 2^31).
 * Errors: PE_EINVAL (inconsistent or out-of-range input), PE_ENOTSUP
 * (a row or column with more than 65534 entries), PE_ENOMEM, PE_EDEVICE. */
int perm_est_create(int32_t n, int64_t nnz,
                    const int32_t *row_ptr, const int32_t *col_idx,
                    const int32_t *col_ptr, const int32_t *row_idx,
                    const float *values, const perm_est_options *opts,
                    perm_est_t **out);

/* Fill *out with a named schedule: the five variants of Sec. 4 --
 * "fixed_all", "adaptive_threshold", "local_threshold", "adaptive_tracked",
 * "local_tracked" (two-sided MD, K0 = 100, K = 10, theta = 0.33, shared
 * initial DM) -- and "plain" (Alg. 2 with MD, no scaling, no filtering),
 * "rasmussen" (Alg. 1), "local_nodm" (local_threshold without inner DM),
 * "learned" and "learned_threshold" (PE_SK_LEARNED with no inner DM / with
 * Thrs, otherwise as the five variants; the network is set separately),
 * "learned_gated" and "learned_threshold_gated" (the same with local_gate).
 * Errors: PE_EINVAL for an unknown name. */
int perm_est_schedule_preset(const char *name, perm_est_schedule *out);

/* Run trajectories 0..n_traj-1 and reduce them (Alg. 2 per trajectory;
 * statistics of Sec. 2 and Sec. 4 "Metrics").
 *   res:       host, required; statistics over the n_traj trajectories.
 *   logw:      device double[n_traj], ln X (-inf when X = 0), or NULL.
 *   alive:     device uint8[n_traj], 1 iff X > 0, or NULL.
 *   path_hash: device uint64[n_traj], SplitMix64 fold of (v_t, u_t), 0 for
 *              dead trajectories, or NULL.
 * Errors: PE_EINVAL (n_traj < 1 or >= 2^32, bad schedule), PE_ENOTSUP
 * (schedule this build cannot run for this n), PE_ENOMEM, PE_EDEVICE. */
int perm_est_run(perm_est_t *h, int64_t n_traj, uint64_t seed,
                 const perm_est_schedule *sched, perm_est_result *res,
                 double *logw, uint8_t *alive, uint64_t *path_hash,
                 void *stream);

/* As perm_est_run for trajectories first..first+count-1 (for resuming or
 * sharding; results are identical to the same ids inside a larger run).
 * Outputs are indexed 0..count-1.  Additional optional device outputs:
 *   path:     int32[count][2n]: (v_t, u_t) vertex ids per completed step,
 *             rows 0..n-1, columns n..2n-1; -1 after the last step.
 *   counters: int32[count][4]: completed steps, inner DM calls, full SK
 *             iterations, local repairs. */
int perm_est_run_range(perm_est_t *h, int64_t first, int64_t count,
                       uint64_t seed, const perm_est_schedule *sched,
                       perm_est_result *res, double *logw, uint8_t *alive,
                       uint64_t *path_hash, int32_t *path, int32_t *counters,
                       void *stream);

/* Bytes of the per-device scratch array of perm_est_run_range_noalloc. */
#define PE_NOALLOC_SCRATCH_BYTES (64u << 20)

/* perm_est_run_range for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same results bit for bit, and no hipMalloc,
 * hipFree or other allocating routine.  Everything the launch needs beyond
 * the caller's inputs and outputs -- counters, argument blocks, the
 * statistics, the outputs left NULL (logw, alive, counters) and the
 * per-trajectory state slots -- lives in one static device array of
 * PE_NOALLOC_SCRATCH_BYTES bytes per GPU, looked up when the first handle
 * on that GPU is created and held until the process ends.  Counters are
 * cleared by kernels on `stream` before each launch.
 *   - The handle must hold one matrix whose preprocessing for this
 *     schedule's (initial_dm, K0) has already run (any earlier run or
 *     run_range call with them); otherwise PE_EINVAL.
 *   - With large per-trajectory state (state slots in device memory) fewer
 *     trajectories run concurrently than in perm_est_run_range: as many
 *     slots as the scratch left after the outputs holds.
 *   - PE_ENOTSUP when the outputs left NULL (25 bytes per trajectory at
 *     most) or one block of state slots do not fit the scratch.
 *   - Every call on one GPU shares its array: calls that overlap in time on
 *     the same GPU (other threads or streams) race and must not be issued.
 * Errors otherwise as perm_est_run_range. */
int perm_est_run_range_noalloc(perm_est_t *h, int64_t first, int64_t count,
                               uint64_t seed, const perm_est_schedule *sched,
                               perm_est_result *res, double *logw, uint8_t *alive,
                               uint64_t *path_hash, int32_t *path, int32_t *counters,
                               void *stream);

/* Create one handle holding `count` matrices (batching): matrix b is given
 * by n[b], nnz[b], row_ptr[b], col_idx[b], col_ptr[b], row_idx[b] and
 * values[b] (values may be NULL for all-0/1 input; a batch is all 0/1 or
 * all weighted), each with the layout and checks of perm_est_create.
 * Errors as perm_est_create; nothing is created if any matrix is invalid. */
int perm_est_create_batch(int32_t count, const int32_t *n, const int64_t *nnz,
                          const int32_t *const *row_ptr, const int32_t *const *col_idx,
                          const int32_t *const *col_ptr, const int32_t *const *row_idx,
                          const float *const *values, const perm_est_options *opts,
                          perm_est_t **out);

/* run flags */
#define PE_RUN_AUTOTUNE 1  /* pick the launch shape (waves per block, blocks
                              per CU) by timing candidates on a probe slice
                              the first time a schedule kind is run; results
                              do not depend on the shape                     */
#define PE_RUN_GRAPH 2     /* run the launch sequence (counter clears,
                              persistent trajectory kernel, reduction) as a
                              HIP graph captured once per launch shape and
                              replayed; per-run values (seed, counts, output
                              pointers) are uploaded before each replay.
                              Results are identical to an eager run          */

/* Run trajectories 0..n_traj[b]-1 of every matrix b of a batch handle in one
 * persistent launch (Alg. 2 per trajectory, matrix b uses counter word b)
 * and reduce each matrix separately (one reduction launch for all).
 *   n_traj:    host int64[count], each in [1, 2^32).
 *   res:       host perm_est_result[count]; the work-unit fields and
 *              `seconds` describe the whole launch.
 *   logw, alive, path_hash: device arrays of sum(n_traj) entries (matrix b
 *              at offset sum_{c<b} n_traj[c]), or NULL.
 *   flags:     PE_RUN_AUTOTUNE and/or PE_RUN_GRAPH, or 0.
 * Errors: PE_EINVAL, PE_ENOTSUP, PE_ENOMEM, PE_EDEVICE. */
int perm_est_run_batch(perm_est_t *h, const int64_t *n_traj, uint64_t seed,
                       const perm_est_schedule *sched, perm_est_result *res,
                       double *logw, uint8_t *alive, uint64_t *path_hash,
                       int32_t flags, void *stream);

/* ------------------------------------------------------------------
 * Learned proposal.  A per-edge network scores every candidate u of the
 * selected vertex v; its softmax, mixed with the uniform distribution,
 * replaces the proposal of Eq. (q).  The importance weight of Alg. 2 still
 * divides by the probability actually sampled, so every estimate stays
 * unbiased (Sec. 2, Eq. (per1)) whatever the network computes.
 *
 * Network: 8 features -> 64 ReLU -> 64 ReLU -> 1 logit; PE_MLP_NPARAM
 * float parameters packed as W1[8][64], b1[64], W2[64][64], b2[64], w3[64],
 * b3 (row-major, input index first).  Features of the candidate edge
 * (rho = its row end, gam = its column end) at step t:
 *   x0 = min(deg rho, 255)/64, x1 = min(deg gam, 255)/64 (residual degrees),
 *   x2 = Q(plog2(r0[rho])/4), x3 = Q(plog2(c0[gam])/4) (outer scaling
 *   after the K0 shared SK iterations, 1 if K0 = 0), x4 = Q(t/n),
 *   x5 = 1 if v is a row, x6 = x7 = 0;
 *   Q(y) = clamp(rint(64 y), -256, 255)/64 and plog2(m 2^e) = e - 2 + 2m for
 *   m in [0.5, 1).
 * Sampling uses the network on an exact grid (results are bit-reproducible
 * against a scalar evaluation): parameters snapped to multiples of 1/64 in
 * [-127/64, 127/64], hidden activations to multiples of 1/64 in
 * [0, 255/64], the logit to L = clamp(rint(16 y), -1024, 1023); then
 * E_i = rint(2^24 exp(-(L_max - L_i)/16)) (0 once the gap reaches 2048) and
 * integer weights w_i = max(1, rint(2^24 ((1 - alpha) E_i / sum E + alpha/k)))
 * over the k candidates.  z of the Thrs / Trck policies is w_u / sum w.
 * ------------------------------------------------------------------ */
#define PE_MLP_NPARAM 4801

/* Install the learned proposal's network on handle h.
 *   params:    device float[PE_MLP_NPARAM] (caller-owned, read once; the
 *              handle keeps its own snapped copy).
 *   mix_alpha: uniform share alpha in [0, 1].
 * Errors: PE_EINVAL (NULL params, alpha outside [0, 1], a non-finite
 * parameter), PE_ENOMEM, PE_EDEVICE. */
int perm_est_set_model(perm_est_t *h, const float *params, double mix_alpha, void *stream);

/* Save a network (host float[PE_MLP_NPARAM], e.g. from
 * perm_est_mlp_get_params) and its uniform share alpha to the file `path`:
 * the bytes "PEMLP001", the parameter count (uint32), a zero uint32, alpha
 * (double), the parameters (float), then a 64-bit FNV-1a checksum of all
 * preceding bytes, little-endian.  Host-only; touches no device.
 * Errors: PE_EINVAL (NULL, alpha outside [0, 1], a non-finite parameter),
 * PE_EIO (the file cannot be written). */
int perm_est_model_save(const char *path, const float *params, double mix_alpha);

/* Read a file written by perm_est_model_save into host params
 * float[PE_MLP_NPARAM] and *mix_alpha (both left unchanged on error); the
 * values can then go to perm_est_set_model (after a copy to the device) or
 * perm_est_mlp_create.  Host-only.
 * Errors: PE_EINVAL (NULL, wrong size, magic or parameter count, checksum
 * mismatch, non-finite value, bad alpha), PE_EIO (cannot be opened). */
int perm_est_model_load(const char *path, float *params, double *mix_alpha);

/* Training-pair buffers (all DEVICE memory, caller-owned).  A group is one
 * recorded step: the candidates of the selected vertex in adjacency order. */
typedef struct {
    float *x;          /* float[rec_cap][8] features (16-byte aligned)       */
    float *y;          /* float[rec_cap] proposal of the running schedule,
                          normalised over the group (the training target)   */
    int64_t *gstart;   /* int64[group_cap] first record of each group        */
    int32_t *ginfo;    /* int32[group_cap][4] = {k, matrix b, trajectory id
                          (bits of a uint32), step t}                       */
    int64_t rec_cap;   /* in [2, 2^31)                                      */
    int64_t group_cap; /* in [1, 2^31)                                      */
    int32_t stride;    /* record steps t with t % stride == 0 (>= 1)        */
    int32_t reserved;  /* must be 0                                         */
} perm_est_record_buffers;

/* Run the batch as perm_est_run_batch (same trajectories, same results in
 * res) and record training pairs from it: at every recorded step with at
 * least two candidates and a vertex list of at most 64 entries, the
 * features above and the schedule's own proposal of Eq. (q) (with
 * PE_SK_FIXED, K full SK iterations on the residual) for each candidate.
 * Groups that do not fit are dropped; the written groups are a prefix of
 * one claim order, with contiguous records, but that order is not
 * deterministic (compare sets keyed by ginfo).
 *   n_records, n_groups: host; how many were written.
 * Errors: as perm_est_run_batch; PE_EINVAL for PE_SK_LEARNED or bad
 * buffers. */
int perm_est_record(perm_est_t *h, const int64_t *n_traj, uint64_t seed,
                    const perm_est_schedule *sched, const perm_est_record_buffers *buf,
                    perm_est_result *res, int64_t *n_records, int64_t *n_groups,
                    void *stream);

/* Trainer of the network (float master parameters and Adam moments on one
 * device).  Training minimises the listwise softmax cross-entropy over
 * groups, loss = (1/G) sum_g -sum_{i in g} y_i ln softmax(L_g)_i, so
 * d loss / d L_i = (softmax_i - y_i) / G; the two hidden layers run on
 * bf16 matrix cores with float accumulation. */
typedef struct perm_est_mlp perm_est_mlp_t;

/* params: host float[PE_MLP_NPARAM] initial values.
 * Errors: PE_EINVAL, PE_ENOMEM, PE_EDEVICE. */
int perm_est_mlp_create(int32_t device, const float *params, perm_est_mlp_t **out);

/* Copy the trainer's current float[PE_MLP_NPARAM] parameters to `out`
 * (host or device memory).  Errors: PE_EINVAL (NULL), PE_EDEVICE. */
int perm_est_mlp_get_params(perm_est_mlp_t *t, float *out, void *stream);

/* logits[i] of the float network (no grid) for device x[n][8]; device
 * logits[n].  Errors: PE_EINVAL (n < 0, NULL), PE_EDEVICE. */
int perm_est_mlp_forward(perm_est_mlp_t *t, const float *x, int64_t n, float *logits, void *stream);

/* Loss over groups g0..g1-1 of a recording (gstart/ginfo as written by
 * perm_est_record: groups contiguous in records) into *loss (host) and its
 * gradient into device grad[PE_MLP_NPARAM] (overwritten; may be NULL).
 * Errors: PE_EINVAL (empty or negative window), PE_ENOMEM, PE_EDEVICE. */
int perm_est_mlp_loss_grad(perm_est_mlp_t *t, const float *x, const float *y, const int64_t *gstart,
                           const int32_t *ginfo, int64_t g0, int64_t g1, double *loss, float *grad,
                           void *stream);

/* Train for `epochs` passes over groups 0..n_groups-1 in windows of
 * `batch_groups` consecutive groups, window order reshuffled each epoch
 * from `seed`; Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr)
 * after every window.  The groups are first put in a canonical order,
 * sorted by (matrix, trajectory, step) from ginfo, on a device copy of the
 * recording (the caller's arrays are not changed), so that the trained
 * parameters do not depend on the order in which a recording claimed its
 * slots: the same set of groups, seed and settings give the same
 * parameters.  loss_per_epoch: host double[epochs] (mean window loss), or
 * NULL.  Errors: PE_EINVAL, PE_ENOMEM, PE_EDEVICE. */
int perm_est_mlp_train(perm_est_mlp_t *t, const float *x, const float *y, const int64_t *gstart,
                       const int32_t *ginfo, int64_t n_groups, int32_t epochs, int64_t batch_groups,
                       double lr, uint64_t seed, double *loss_per_epoch, void *stream);

void perm_est_mlp_destroy(perm_est_mlp_t *t);

/* Multi-seed consensus diagnostics for a matrix whose permanent is not
 * known (Sec. 4.4, "Real-world matrices with unknown permanents").  Host
 * only; touches no device.
 *   runs: host perm_est_result[n_variants][n_seeds] (variant-major), the
 *         final statistics of each run (log_estimate, rse, n_traj, n_alive,
 *         ess are read).
 * With Y = exp(log_estimate), e = rse * Y the within-run standard error,
 * per variant P: Ybar_P = mean over seeds, e_in = sqrt(sum e^2) / R,
 * e_seed = sd(Y) / sqrt(R) (R - 1 denominator), e_P = max(e_in, e_seed);
 * P_con = mean over variants of Ybar_P, e_con = sqrt(sum e_P^2) / V;
 * D_max = max over pairs |Ybar_P - Ybar_P'| / sqrt(e_P^2 + e_P'^2) against
 * c_Bonf = Phi^{-1}(1 - alpha / (2 C(V, 2))).  The checks of a provisional
 * consensus are the PE_CON_* bits; the variant-wise 95 % t-interval is
 * Ybar_P +- t_{0.975, R-1} e_P.
 *   log_ybar, rel_e: host double[n_variants] (ln Ybar_P, e_P / Ybar_P), or
 *         NULL.
 * Errors: PE_EINVAL (n_variants < 2, n_seeds < 2, alpha outside (0, 1),
 * NULL runs or out). */
#define PE_CON_ALL_RUNS 1u     /* every run has n_traj > 0 and a log_estimate */
#define PE_CON_T_INTERVALS 2u  /* the variant-wise t-intervals intersect     */
#define PE_CON_BONFERRONI 4u   /* D_max <= c_Bonf                             */
#define PE_CON_ALIVE 8u        /* every run has >= 1000 surviving trajectories */
#define PE_CON_ESS 16u         /* every run has ESS >= 1000                   */
#define PE_CON_HALF_WIDTH 32u  /* 1.96 e_con <= 0.1 P_con                     */
#define PE_CON_ALL 63u
typedef struct {
    double log_p_con;      /* ln of the equal-variant consensus P_con        */
    double log_e_con;      /* ln of its standard error e_con                 */
    double rel_half_width; /* 1.96 e_con / P_con                             */
    double variant_ratio;  /* largest variant mean / smallest                */
    double min_ess;        /* smallest run ESS                               */
    double d_max;
    double c_bonf;
    double t_crit;         /* t_{0.975, n_seeds - 1}                         */
    uint32_t checks;       /* PE_CON_* bits that hold                        */
    int32_t provisional;   /* 1 iff every check holds                        */
} perm_est_consensus_result;

int perm_est_consensus(int32_t n_variants, int32_t n_seeds, const perm_est_result *runs, double alpha,
                       perm_est_consensus_result *out, double *log_ybar, double *rel_e);

/* Release every device and host resource of the handle (NULL is a no-op). */
void perm_est_destroy(perm_est_t *h);

/* Message of the last failed call in this thread ("" if none). */
const char *perm_est_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PERM_EST_H */
