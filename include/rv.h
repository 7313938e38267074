/*
 * rv.h -- C ABI of the MI355X (gfx950) per-cluster velocity and heading
 * estimator of "Parallelized Instantaneous Velocity and Heading Estimation of
 * Objects using Single Imaging Radar" (Singh, Sil, Sharma).
 *
 * For every cluster of radar points the library
 *   1. runs RANSAC over the rigid-body velocity profile of Sec. 3.2, Eq. 6,
 *        v_d = vx cos(theta) + vy sin(theta):
 *      each hypothesis draws a pair of seed points, solves the 2x2 system for
 *      (vx, vy), and counts the points with |v_d - vx cos - vy sin| < tau
 *      (Sec. 3.1, Alg. 1, as the velocity-profile variant);
 *   2. keeps the hypothesis with the most inliers (Sec. 3.1; ties: lowest index);
 *   3. refits (vx, vy) by least squares on that hypothesis's inliers
 *      (Sec. 3.2, Eq. 7, Alg. 2: the pseudoinverse solution);
 *   4. reports heading = atan2(vy, vx) (Eq. 8, quadrant-correct).
 *
 * Memory and streams.  Every array argument of rv_estimate_velocity is a
 * DEVICE pointer owned by the caller; the library allocates nothing, keeps no
 * pointer after the call returns, and enqueues its work asynchronously on
 * `stream` (a hipStream_t; NULL is the default stream).  Results are valid
 * once the caller has synchronised that stream.  Calls that share a workspace
 * must be ordered on one stream.
 *
 * Errors.  Argument checks run on the host before anything is enqueued; a
 * negative rv_status_t means nothing was launched, and rv_last_error() returns
 * a message (thread-local).  Per-cluster conditions are not errors: they set
 * that cluster's status byte and NaN outputs, and the call returns RV_OK.
 */
#ifndef RV_H
#define RV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RV_OK = 0,
    RV_ERR_INVALID_ARG = -1, /* null pointer, bad size or scalar */
    RV_ERR_WORKSPACE = -2,   /* workspace missing or smaller than rv_workspace_bytes() */
    RV_ERR_HIP = -3,         /* a HIP launch failed; rv_last_error() has the HIP message */
    RV_ERR_BUSY = -4         /* server: its queue of waiting frames is full, submit again later */
} rv_status_t;

/* Per-cluster status byte. */
enum {
    RV_CLUSTER_OK = 0,
    RV_CLUSTER_TOO_FEW_POINTS = 1, /* fewer than two points */
    RV_CLUSTER_ALL_DEGENERATE = 2, /* no valid seed pair among the n_hyp draws */
    RV_CLUSTER_SINGULAR_REFIT = 3, /* the kept inlier set has fewer than two points
                                      or a non-positive normal-equation determinant */
    RV_CLUSTER_BAD_OFFSETS = 4,    /* offsets[k] < 0, offsets[k+1] < offsets[k], or
                                      offsets[k+1] > n_points */
    RV_CLUSTER_TOO_LARGE = 5       /* paper-literal variant only: more than
                                      RV_PAPER_MAX_POINTS points */
};

/* Largest cluster the paper-literal variant handles (its medians are sorted in
   on-chip memory). */
#define RV_PAPER_MAX_POINTS 4096

/* A seed pair is degenerate (its hypothesis invalid) when its two azimuths,
   promoted to double, differ by less than this many radians. */
#define RV_MIN_SEED_SEPARATION 1e-3
/* Half-width (m/s) of the "near tau" window counted in n_near_tau. */
#define RV_NEAR_TAU_WINDOW 1e-5
/* Largest accepted n_hyp. */
#define RV_MAX_HYP (1 << 20)

/*
 * Bytes of device workspace rv_estimate_velocity needs for these sizes
 * (a pure host computation; 0 for negative sizes).
 */
size_t rv_workspace_bytes(int64_t n_clusters, int64_t n_points, int32_t n_hyp);

/*
 * Estimate vx, vy (m/s) and heading (rad) of every cluster of one CSR frame.
 *
 * Inputs (device, read only):
 *   theta[n_points]   azimuth of each point, radians, float32.  Measured from
 *                     the +x (longitudinal) axis, counter-clockwise positive.
 *   vd[n_points]      radial Doppler velocity of each point, m/s, float32.
 *   cluster_offsets[n_clusters + 1]  int32; the points of cluster k are
 *                     [offsets[k], offsets[k+1]).  Expected: offsets[0] = 0,
 *                     non-decreasing, offsets[n_clusters] = n_points; a cluster
 *                     whose bounds are inconsistent gets RV_CLUSTER_BAD_OFFSETS
 *                     and no memory outside [0, n_points) is touched.
 * Scalars:
 *   n_clusters >= 0, 0 <= n_points <= INT32_MAX.
 *   n_hyp in [1, RV_MAX_HYP]: hypotheses per cluster (the paper's max_trials).
 *   tau > 0 and finite: a point is an inlier when |residual| < tau (strict).
 *   seed: hypothesis h of cluster k draws its pair from Philox4x32-10 with
 *     key = (seed & 0xffffffff, seed >> 32) and counter = (h, k, 0, 0), so a
 *     cluster's result depends only on (seed, k, its points, n_hyp, tau).
 * Outputs (device, written; [n_clusters] each):
 *   vx, vy, heading (float32; NaN when status != RV_CLUSTER_OK),
 *   n_inliers (int32; size of the refit set), status (uint8, RV_CLUSTER_*).
 * Optional outputs (device, may be NULL):
 *   n_near_tau[n_clusters]   int32: points of the kept hypothesis whose double-
 *                            precision |residual| is within RV_NEAR_TAU_WINDOW of tau.
 *   inlier_bits[ceil(n_points/32)]  uint32: the frame-wide inlier mask (Sec. 3.1:
 *                            logical OR of the per-cluster masks); bit p%32 of word
 *                            p/32 is point p.  Cleared by the call.
 *   hyp_counts[n_clusters * n_hyp]  int32: float32-stage inlier count of every
 *                            hypothesis (0 for invalid ones), cluster-major.
 *   best_hyp[n_clusters]     int32: index of the kept hypothesis, -1 if none.
 * Workspace: device memory of at least rv_workspace_bytes(n_clusters, n_points,
 *   n_hyp) bytes, 256-byte aligned; contents need no initialisation.
 * Returns RV_OK or a negative rv_status_t.
 */
int rv_estimate_velocity(const float *theta, const float *vd, const int32_t *cluster_offsets,
                         int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau,
                         uint64_t seed, float *vx, float *vy, float *heading, int32_t *n_inliers,
                         uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                         int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                         size_t workspace_bytes, void *stream);

/*
 * ---- Part of a frame -----------------------------------------------------------
 *
 * rv_estimate_velocity_part estimates clusters [first_cluster, first_cluster +
 * n_clusters) of a larger frame, so that a frame can be sent to the GPU and
 * estimated in pieces (the estimate of one piece overlapping the copy of the
 * next).  Each cluster draws its hypotheses with the counter of its index in
 * the whole frame, (h, first_cluster + k, 0, 0) for the part's k-th cluster
 * (Sec. 3.1: seed pairs drawn per cluster), so every per-cluster output is bit
 * for bit what rv_estimate_velocity gives for the whole frame.
 *   - theta and vd hold the part's n_points points: the whole frame's arrays
 *     from point first_point on.  cluster_offsets[n_clusters + 1] are the
 *     whole frame's offsets of the part's clusters (the whole frame's array
 *     from entry first_cluster on), so cluster k of the part owns the part's
 *     points [offsets[k] - first_point, offsets[k+1] - first_point); a cluster
 *     outside [0, n_points) of the part gets RV_CLUSTER_BAD_OFFSETS.
 *   - Outputs are indexed by the part's cluster k (the whole frame's outputs
 *     from entry first_cluster on, hyp_counts from first_cluster * n_hyp).
 *     inlier_bits covers the part's points, bit p of the part's point p, and
 *     ceil(n_points/32) words of it are cleared: a frame-wide mask can be
 *     shared by parts whose first points are multiples of 32, each given the
 *     word of its first point.
 *   - first_cluster in [0, 2^32 - 1] with first_cluster + n_clusters <= 2^32
 *     (the counter is 32 bits), first_point in [0, 2^31 - 1]; else
 *     RV_ERR_INVALID_ARG.
 *   - Workspace: rv_workspace_bytes(n_clusters, n_points, n_hyp) of the part.
 *     Parts ordered on one stream may share one workspace.
 * first_cluster = first_point = 0 with the whole frame is rv_estimate_velocity.
 */
int rv_estimate_velocity_part(const float *theta, const float *vd, const int32_t *cluster_offsets,
                              int64_t n_clusters, int64_t n_points, int64_t first_cluster,
                              int64_t first_point, int32_t n_hyp, float tau, uint64_t seed,
                              float *vx, float *vy, float *heading, int32_t *n_inliers,
                              uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                              int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                              size_t workspace_bytes, void *stream);

/*
 * rv_estimate_velocity_pipelined: one frame from host memory, copied to the
 * GPU and estimated in n_parts parts cut at cluster boundaries, part j's
 * estimate (rv_estimate_velocity_part) running on `stream` while part j + 1 is
 * copied on `copy_stream`.  Part j holds about a share n_parts - j out of
 * n_parts (n_parts + 1) / 2 of the points: the parts shrink toward the end,
 * since only the last part's estimate is not hidden behind a copy.  The
 * outputs are bit for bit those of rv_estimate_velocity on the whole frame.
 *   theta_host, vd_host [n_points], offsets_host [n_clusters + 1]: host memory,
 *     pinned (hipHostMalloc, torch's pin_memory()) for the copies to run
 *     asynchronously.  The host reads offsets_host during the call to cut the
 *     frame and size the copies: it must start at 0, not decrease and end at
 *     n_points (else RV_ERR_INVALID_ARG, nothing enqueued).  The caller keeps
 *     the host arrays unchanged until `stream` has finished the call's work.
 *   theta_dev, vd_dev [n_points], offsets_dev [n_clusters + 1]: device memory
 *     the call copies the frame into (the caller's; contents overwritten).
 *   Outputs as rv_estimate_velocity (device memory, or pinned host memory
 *     through rv_host_device_pointer), without the frame-wide inlier mask
 *     (parts cut at cluster boundaries need not start on 32-point words: use
 *     rv_estimate_velocity or rv_estimate_velocity_part for the mask).
 *   n_parts in [1, RV_MAX_PARTS]; workspace as rv_estimate_velocity.
 *   copy_stream: a stream of the same device other than `stream` (the same
 *     stream is correct but overlaps nothing).  The call's copies wait for the
 *     work already queued on `stream` and on copy_stream (so calls in a row
 *     may reuse the device buffers), and `stream` waits for each part's copy.
 * The call returns once everything is enqueued; the results are ready when
 * `stream` is.
 */
#define RV_MAX_PARTS 64

int rv_estimate_velocity_pipelined(const float *theta_host, const float *vd_host,
                                   const int32_t *offsets_host, int64_t n_clusters,
                                   int64_t n_points, int32_t n_parts, int32_t n_hyp, float tau,
                                   uint64_t seed, float *theta_dev, float *vd_dev,
                                   int32_t *offsets_dev, float *vx, float *vy, float *heading,
                                   int32_t *n_inliers, uint8_t *status, int32_t *n_near_tau,
                                   int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                                   size_t workspace_bytes, void *stream, void *copy_stream);

/*
 * ---- Allocation-free form ----------------------------------------------------
 *
 * For callers that cannot allocate device memory around the estimate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  rv_estimate_velocity_noalloc takes the arguments of
 * rv_estimate_velocity without the workspace and gives the same results bit
 * for bit (same kernels).  Its workspace is a device array of
 * RV_NOALLOC_SCRATCH_BYTES inside the library's code object: each GPU holds its
 * own copy from the library's first use on that GPU (the code object's load,
 * whichever entry point causes it) until the process ends.  The call itself
 * allocates and frees nothing and records no stage-timing events.  The caller still owns
 * every input and output.
 *   - A frame whose rv_workspace_bytes() exceeds RV_NOALLOC_SCRATCH_BYTES is
 *     rejected with RV_ERR_WORKSPACE before anything is enqueued (96 MiB: up to
 *     about 5 million points).
 *   - `stream` must belong to the current device (else RV_ERR_INVALID_ARG).
 *   - All calls on one GPU share its array: calls whose work may overlap on
 *     that GPU (different streams, or different threads without ordering) race
 *     and give undefined results.  Calls ordered on one stream are safe; each
 *     call overwrites what the previous one left there.
 */
#define RV_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)

int rv_estimate_velocity_noalloc(const float *theta, const float *vd,
                                 const int32_t *cluster_offsets, int64_t n_clusters,
                                 int64_t n_points, int32_t n_hyp, float tau, uint64_t seed,
                                 float *vx, float *vy, float *heading, int32_t *n_inliers,
                                 uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                                 int32_t *hyp_counts, int32_t *best_hyp, void *stream);

/*
 * ---- Many frames at once ---------------------------------------------------
 *
 * The frames share one CSR: frame f owns clusters [frame_offsets[f],
 * frame_offsets[f+1]) of cluster_offsets (frame_offsets[0] = 0, non-decreasing,
 * frame_offsets[n_frames] = n_clusters).  Cluster k of frame f draws its
 * hypotheses with key = (seeds[f] & 0xffffffff, seeds[f] >> 32) and counter =
 * (h, k - frame_offsets[f], 0, 0): every cluster's outputs are bitwise those
 * rv_estimate_velocity gives for its frame alone with seed seeds[f].  The
 * scoring runs as one persistent launch that drains a device work queue of
 * (cluster, block of 256 hypotheses) items, largest clusters first.
 */

/* Cluster-size buckets of the tuning table: bucket 0 holds n < 64, bucket b
   holds 32 * 2^b <= n < 64 * 2^b, bucket RV_TUNE_BUCKETS - 1 everything larger. */
#define RV_TUNE_BUCKETS 8

typedef struct {
    /* register rows of 64 points scored per pass, 1..16, per size bucket */
    int32_t rows_max[RV_TUNE_BUCKETS];
    /* persistent scoring grid: workgroups per compute unit; 0 = as many as fit */
    int32_t blocks_per_cu;
    /* clusters of at least this many points score their residuals in the FP16
       form (0 = none, the default; >= 0).  The FP16 form: half2 (cos, sin) and
       the float32 residual against a reference velocity, one v_dot2_f32_f16 per
       point and hypothesis (FP32 accumulation), a threshold widened by a proven
       bound on the FP16 error, then an exact float32 count of every hypothesis
       that could still be the best.  It keeps the same hypothesis as the
       float32 form, so every output is bitwise the same, except hyp_counts:
       there it holds the FP16 counts, upper bounds of the float32 counts. */
    int32_t fp16_min_points;
    /* clusters of at most this many points (0..256) score with lanes =
       hypotheses: each thread keeps the hypothesis it solved, the cluster's
       points are staged in LDS and read as broadcasts, and each lane counts its
       own inliers (four vector instructions per point and 64 hypotheses, no
       lanes idle for a cluster smaller than 64 points).  Same arithmetic, so
       the same results bit for bit; it takes precedence over the FP16 form. */
    int32_t lanes_max_points;
} rv_tuning_t;

/* Defaults: 16 rows in every bucket, as many workgroups per CU as fit, no
   FP16 form, lanes = hypotheses for clusters of at most 64 points. */
void rv_tuning_default(rv_tuning_t *tuning);

/* Device workspace bytes of rv_estimate_velocity_batch (0 for invalid sizes). */
size_t rv_batch_workspace_bytes(int64_t n_frames, int64_t n_clusters, int64_t n_points,
                                int32_t n_hyp);

/*
 * rv_estimate_velocity over n_frames >= 1 frames in one launch sequence.
 * Arguments as rv_estimate_velocity, plus:
 *   frame_offsets[n_frames + 1]  int32, device: the frames' cluster ranges;
 *   seeds[n_frames]              uint64, device: each frame's hypothesis seed;
 *   tuning                       host struct, nullable (defaults), read during the call.
 * Inconsistent frame offsets are never a memory error (a cluster is then
 * attributed to some frame in [0, n_frames)).  The workspace must hold
 * rv_batch_workspace_bytes(n_frames, n_clusters, n_points, n_hyp) bytes.
 */
int rv_estimate_velocity_batch(const float *theta, const float *vd, const int32_t *cluster_offsets,
                               const int32_t *frame_offsets, const uint64_t *seeds,
                               int64_t n_frames, int64_t n_clusters, int64_t n_points,
                               int32_t n_hyp, float tau, float *vx, float *vy, float *heading,
                               int32_t *n_inliers, uint8_t *status, int32_t *n_near_tau,
                               uint32_t *inlier_bits, int32_t *hyp_counts, int32_t *best_hyp,
                               const rv_tuning_t *tuning, void *workspace,
                               size_t workspace_bytes, void *stream);

/*
 * HIP graph of one rv_estimate_velocity_batch call.  Capture records the
 * launch sequence with these pointers and sizes (on a private stream; nothing
 * runs); the caller keeps every buffer alive and in place while the graph
 * exists, and may change their contents between launches.  rv_graph_launch
 * replays it on `stream`; replays on one stream are ordered, replays that share
 * a workspace must not overlap.  The graph holds no HIP memset nodes.
 */
typedef struct rv_graph rv_graph_t;
int rv_graph_capture_batch(const float *theta, const float *vd, const int32_t *cluster_offsets,
                           const int32_t *frame_offsets, const uint64_t *seeds, int64_t n_frames,
                           int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau,
                           float *vx, float *vy, float *heading, int32_t *n_inliers,
                           uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                           int32_t *hyp_counts, int32_t *best_hyp, const rv_tuning_t *tuning,
                           void *workspace, size_t workspace_bytes, rv_graph_t **graph);
int rv_graph_launch(rv_graph_t *graph, void *stream);
void rv_graph_destroy(rv_graph_t *graph);

/*
 * Paper-literal variant of the inlier kernel (Sec. 3.1, Alg. 1, Eq. 5),
 * followed by the same least-squares refit and heading (Sec. 3.2, Eq. 7,
 * Alg. 2, Eq. 8).  Per cluster, in FP64:
 *   - azimuth and Doppler are mapped onto [0, 1] by the cluster's min and max
 *     (Alg. 1's normalize(); a zero span maps to 0);
 *   - thresh = median |y - median(y)| of the normalised Doppler values y
 *     (Eq. 5, read as the median absolute deviation its text names; the median
 *     of an even count is the mean of the two middle values);
 *   - trial h draws its seed pair exactly as rv_estimate_velocity does (same
 *     seed, counter (h, k, 0, 0), same validity rule) and fits the line
 *     y = m x + c through the two normalised seeds;
 *   - a point is an inlier when |(-m) x + 1 y + (-c)| / sqrt(m^2 + 1) <= thresh
 *     (Alg. 1's distance and test, evaluated as written, no contraction);
 *   - the valid trial with the most inliers is kept (ties: lowest h), and
 *     (vx, vy) is the least-squares solution of v_d = vx cos + vy sin over its
 *     inliers; heading = atan2(vy, vx).
 * Arguments as rv_estimate_velocity without tau; thresh[n_clusters] (FP64,
 * device, nullable) receives each cluster's threshold.  Clusters of more than
 * RV_PAPER_MAX_POINTS points get RV_CLUSTER_TOO_LARGE.  The workspace must hold
 * rv_paper_workspace_bytes(n_clusters, n_points, n_hyp) bytes, 256-byte
 * aligned (16 B per point + 16 B per cluster).  The normalisation is per
 * cluster, so where offsets are not non-decreasing the clusters whose ranges
 * overlap another's get unspecified results (the decreasing one still gets
 * RV_CLUSTER_BAD_OFFSETS).  Without inlier_bits, frames of
 * at most 65,536 points and 65,536 clusters with n_hyp <= 256 run as one
 * launch with the same results bit for bit (for rv_stage_times it counts
 * wholly as the scoring stage).
 */
size_t rv_paper_workspace_bytes(int64_t n_clusters, int64_t n_points, int32_t n_hyp);
int rv_estimate_velocity_paper(const float *theta, const float *vd, const int32_t *cluster_offsets,
                               int64_t n_clusters, int64_t n_points, int32_t n_hyp, uint64_t seed,
                               float *vx, float *vy, float *heading, int32_t *n_inliers,
                               uint8_t *status, double *thresh, uint32_t *inlier_bits,
                               int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                               size_t workspace_bytes, void *stream);

/*
 * Frame server (request loop with continuous batching).
 *
 * A server owns one device arena of hbm_budget_bytes (allocated once, at
 * creation), a pool of pinned host buffers, n_streams launch slots and two
 * threads.  rv_server_submit copies a frame from caller HOST memory into a
 * pinned buffer and queues it (rv_server_submit_pinned queues a frame held in
 * the caller's pinned memory without copying it).  The scheduler thread admits waiting frames in
 * arrival order whenever a launch slot is free: as many as fit, together, in
 * the arena's largest free range (inputs, workspace and outputs of the batch)
 * and in max_batch_frames; it copies them to the device and launches them as
 * one rv_estimate_velocity_batch call on the slot's stream, followed by one
 * copy of the per-cluster results to pinned host memory.  Frames that arrive
 * while batches are on the GPU go into the next free slot, so their copies and
 * kernels overlap the running ones.  The completion thread waits for each
 * batch, hands the results to its frames and frees the batch's arena range.
 *
 * Each frame's results are those of rv_estimate_velocity on that frame alone
 * with its seed, whatever else is in flight (bitwise: the batched path draws a
 * cluster's hypotheses from its frame's seed and its index within the frame).
 *
 * Threading: submit, wait, result and stats may be called from any threads.
 * Tickets are unique per server; a ticket's results are held until
 * rv_server_result takes them.
 */
typedef struct rv_server rv_server_t;

typedef struct {
    int32_t n_hyp;               /* hypotheses per cluster, [1, RV_MAX_HYP] */
    float tau;                   /* inlier threshold, m/s, finite and > 0 */
    size_t hbm_budget_bytes;     /* device arena size, >= 1 MiB */
    int32_t max_batch_frames;    /* frames per launch, >= 1 */
    int32_t n_streams;           /* launch slots in flight, [1, 8] */
    int32_t max_waiting_frames;  /* submitted, not yet launched frames before RV_ERR_BUSY, >= 1 */
    int32_t keep_inlier_bits;    /* nonzero: every frame's inlier mask (Sec. 3.1: the OR of its
                                    clusters' masks) is computed and kept for rv_server_result;
                                    it costs ceil(n_points / 32) words per frame in the arena */
    rv_tuning_t tuning;
} rv_server_config_t;

/* Defaults: n_hyp 512, tau 0.15, 16 GiB, 64 frames per launch, 2 slots,
   1024 waiting frames, no inlier masks, default tuning. */
void rv_server_config_default(rv_server_config_t *cfg);

/* Device memory that one frame of n_clusters clusters and n_points points
   takes in the arena when it is launched alone (0 for invalid sizes). */
size_t rv_server_frame_bytes(const rv_server_config_t *cfg, int64_t n_clusters,
                             int64_t n_points);

/* Creates a server on the current device.  RV_OK, RV_ERR_INVALID_ARG or
   RV_ERR_HIP (arena, pinned memory, streams or threads could not be made). */
int rv_server_create(const rv_server_config_t *cfg, rv_server_t **server);

/*
 * Queues one frame.  theta[n_points], vd[n_points], cluster_offsets[n_clusters
 * + 1] are HOST arrays, copied before the call returns.  Offsets must satisfy
 * 0 <= offsets[k] <= offsets[k+1] <= n_points.  *ticket receives the frame's
 * ticket.  RV_ERR_INVALID_ARG for bad arguments or a frame larger than the
 * whole arena, RV_ERR_BUSY when max_waiting_frames frames are waiting.
 */
int rv_server_submit(rv_server_t *server, const float *theta, const float *vd,
                     const int32_t *cluster_offsets, int64_t n_clusters, int64_t n_points,
                     uint64_t seed, uint64_t *ticket);

/*
 * rv_server_submit without the copy: theta, vd and cluster_offsets are host
 * arrays that the server reads in place, the offsets on the host when the
 * frame's batch is launched and the points by the batch's host-to-device
 * copies.  They should be pinned (hipHostMalloc, torch's pin_memory()) for
 * those copies to be asynchronous; pageable arrays give the same results, with
 * copies that hold the server's scheduler thread.  The caller keeps them alive
 * and unchanged until rv_server_wait reports the ticket ready (or the ticket's
 * batch fails); several frames in flight may share read-only arrays.  Errors
 * and results as rv_server_submit, the results bit for bit.
 */
int rv_server_submit_pinned(rv_server_t *server, const float *theta, const float *vd,
                            const int32_t *cluster_offsets, int64_t n_clusters, int64_t n_points,
                            uint64_t seed, uint64_t *ticket);

/* Waits up to timeout_ms (negative: no limit) for a ticket's results: 1 ready,
   0 not yet, RV_ERR_INVALID_ARG for an unknown ticket, RV_ERR_HIP if its batch
   failed. */
int rv_server_wait(rv_server_t *server, uint64_t ticket, int64_t timeout_ms);

/* Host-clock times of one frame, nanoseconds since the server's creation. */
typedef struct {
    int64_t submitted_ns;   /* rv_server_submit copied it (queued it, without a copy) */
    int64_t launched_ns;    /* its batch was enqueued */
    int64_t done_ns;        /* its batch's results were in host memory */
    int32_t batch_frames;   /* frames in its batch */
    int32_t slot;           /* launch slot of its batch */
} rv_frame_times_t;

/* Copies a ready ticket's per-cluster results into HOST arrays of its
   n_clusters entries and forgets the ticket.  Nullable: n_near_tau, best_hyp
   (index of each cluster's kept hypothesis, -1 if none, as rv_estimate_velocity
   reports it), inlier_bits (HOST array of ceil(n_points / 32) words: bit p % 32
   of word p / 32 is the frame's point p; only from a server created with
   keep_inlier_bits) and times.  RV_OK, RV_ERR_INVALID_ARG (unknown ticket, NULL
   required output, inlier_bits from a server that keeps no masks; the ticket is
   then kept) or RV_ERR_BUSY (not ready yet). */
int rv_server_result(rv_server_t *server, uint64_t ticket, float *vx, float *vy, float *heading,
                     int32_t *n_inliers, uint8_t *status, int32_t *n_near_tau, int32_t *best_hyp,
                     uint32_t *inlier_bits, rv_frame_times_t *times);

typedef struct {
    int64_t frames_submitted, frames_done, batches, busy_rejections;
    int64_t max_batch_frames_seen;
    int64_t arena_bytes, arena_peak_bytes;  /* budget and the most of it ever in use */
    int64_t pinned_bytes;                   /* pinned host memory held by the pool */
    int64_t waiting_frames, inflight_batches;
} rv_server_stats_t;
int rv_server_stats(rv_server_t *server, rv_server_stats_t *stats);

/* Finishes every submitted frame, stops the threads and frees everything;
   results not taken are dropped.  No other call on this server may be in
   progress or start once destroy has begun. */
void rv_server_destroy(rv_server_t *server);

/* Message of the last failing call on this thread ("" if none). */
const char *rv_last_error(void);

/*
 * Instrumentation (not part of the estimate).  While enabled, every
 * rv_estimate_velocity, rv_estimate_velocity_batch or rv_estimate_velocity_paper
 * call (not graph replays) records HIP events around its kernels on its stream
 * (for the paper-literal variant the stages are: normalisation and threshold,
 * trials, refit).  rv_stage_times waits for the recorded events, writes
 * the summed milliseconds per stage (ms[0]: point staging and dispatch
 * planning, ms[1]: hypotheses and scoring, ms[2]: selection and refit) and the
 * number of calls into *n_calls, and clears the record.  A single-frame call
 * that takes the one-launch path for small frames (at most 65,536 points, at
 * most 256 hypotheses, no inlier mask requested; same results) counts wholly as
 * ms[1].  Returns RV_OK or RV_ERR_HIP.
 */
int rv_stage_timing(int enable);
int rv_stage_times(double *ms, int64_t *n_calls);

/*
 * Pinned host memory as estimate arguments.  Host memory from hipHostMalloc
 * (which is what torch's pin_memory() allocates) is mapped into the GPUs'
 * address space: the estimate entry points may read their inputs from it and
 * write their outputs to it directly, over PCIe, with no copies.  For small
 * frames, whose copies cost more than the kernels, this shortens the latency
 * from a frame in host memory to its results in host memory; the workspace
 * stays in device memory.  rv_host_device_pointer returns in *device_ptr the
 * address under which the current device sees host_ptr (an address inside a
 * hipHostMalloc allocation), or RV_ERR_INVALID_ARG (and NULL) when host_ptr is
 * not in such memory: pageable host memory must never be passed to the
 * kernels.  The caller keeps the memory allocated while the work that uses it
 * is in flight, writes inputs before the call and reads outputs only after
 * synchronising the stream.
 */
int rv_host_device_pointer(const void *host_ptr, void **device_ptr);

/*
 * Test hook: n independent Philox4x32-10 blocks computed on the GPU by the same
 * device function the estimator uses.  ctr[4n], key[2n], out[4n] are device
 * arrays of uint32 (block t uses ctr[4t..4t+3] and key[2t..2t+1]).  Enqueued on
 * `stream`.  Returns RV_OK or a negative rv_status_t.
 */
int rv_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                     void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RV_H */
