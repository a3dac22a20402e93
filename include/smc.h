/*
 * smc.h -- C ABI of the MI355X (gfx950) particle-filter rigid registration
 * library, after Uruththirakodeeswaran et al., "Accelerated 3D-3D rigid
 * registration of echocardiographic images obtained from apical window using
 * particle filter" (arXiv 2504.19930).
 *
 * The problem (Abstract; Methods, Registration, Eq. 1): given a source and a
 * target volume -- echo intensities or binary LV masks -- and rough bounds on
 * how far the rotation and the translation may range, estimate the rigid
 * transform (rx, ry, rz, tx, ty, tz) of Implementation Details (Euler 3D
 * transform, homogeneous matrix of Eq. 3) that best aligns the warped source
 * with the target, then apply it to every frame of the sequence.
 *
 * Conventions shared by every call:
 *  - Volumes are uint8, x fastest (index i + nx (j + ny k)), voxel (i,j,k) at
 *    s * (i,j,k) mm.  Volume and output pointers are DEVICE pointers owned by
 *    the caller; they must stay valid while work queued on the stream runs.
 *  - Angles are radians, translations mm.  The transform maps a target point p
 *    to the source point q = R (p - c) + c + t with R = Rz(rz) Rx(rx) Ry(ry)
 *    and c the target centre, (0.5 s_d)(n_d - 1).
 *  - Every call returns smc_status; none throws.  A failure leaves a message
 *    for smc_last_error() (thread-local).  Arguments are checked on the host
 *    before anything is launched.  Errors on a context are sticky: once a
 *    call on it fails, later calls on it return the same status.
 *  - Calls are asynchronous on the caller's HIP stream unless marked "syncs".
 */
#ifndef SMC_H
#define SMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SMC_OK = 0,
    SMC_EINVAL = -1,   /* bad argument (null pointer, size, NaN, unsupported combination) */
    SMC_ENOMEM = -2,   /* device allocation failed */
    SMC_EDEVICE = -3,  /* a HIP call or kernel launch failed */
    SMC_ESTATE = -4,   /* call not valid in the context's current state */
    SMC_ENOOVERLAP = -5 /* smc_estimate: every particle of the latest iteration scored -inf (no overlap
                           reached the minimum); the outputs are still written (uniform-weight mean) */
} smc_status;

/* Similarity used as the filter's measurement (Fig. 1 caption).
 * DICE: Eq. 4 on binary masks, over the whole target FOV, nearest neighbour.
 * NCC:  Eq. 2 (squared correlation, 0..1) over the overlap.
 * SSD:  mean squared difference of the mean-0 / std-1 normalised images
 *       (Implementation Details) over the overlap; the score is its negative.
 * MI:   mutual information (the metric Related Work lists beside NCC) over
 *       the overlap, TRILINEAR only: a 32 x 32 joint histogram of exact
 *       counts of (source bin, target bin), source bin = floor(256 s + 0.5)
 *       >> 11, target bin = t >> 3, scored as the symmetric uncertainty
 *       2 I(S;T) / (H(S) + H(T)) in [0, 1] (1 for images equal up to a
 *       bijection of bins); overlaps below the minimum score -inf. */
typedef enum { SMC_SCORE_DICE = 0, SMC_SCORE_NCC = 1, SMC_SCORE_SSD = 2, SMC_SCORE_MI = 3 } smc_score;

/* Sampling of the source at non-grid positions (Implementation Details:
 * trilinear interpolation).  DICE requires NEAREST. */
typedef enum { SMC_INTERP_NEAREST = 0, SMC_INTERP_TRILINEAR = 1 } smc_interp;

/* How rotations are treated (the paper's own search is the BOX: Euler angles
 * in x0 +- limit, weighted-mean estimate).  WIDE is for searches whose
 * rotation limits reach a half turn (views far apart, e.g. the apical to
 * parasternal pairs of the Discussion, about (90, -180) degrees about y and
 * z): the estimate's rotation is the normalised weighted sum of the
 * particles' unit quaternions, put on the hemisphere of the first particle of
 * largest weight, converted back to Euler angles within pi of x0; and every
 * rotation axis whose limit is >= pi wraps around the circle in the
 * prediction instead of reflecting.  Axes with smaller limits, the
 * translations, the prior and the weights are as in BOX. */
typedef enum { SMC_ROTATION_BOX = 0, SMC_ROTATION_WIDE = 1 } smc_rotation;

typedef struct {
    int32_t nx, ny, nz;      /* voxels, each 1 .. 65535; nx*ny < 2^24, nx*ny*nz < 2^31 */
    double sx, sy, sz;       /* spacing in mm, > 0 */
    const uint8_t *data;     /* device, nz*ny*nx bytes */
    const uint8_t *fov;      /* device or NULL; nonzero = inside the imaged field of view */
} smc_volume;

/* Filter parameters.  The paper defers them to its earlier work; the values
 * used here are documented readings (rotation / translation limits from the
 * Abstract, the rest tuned on synthetic data). */
typedef struct {
    uint32_t n_particles;    /* N, 1 .. 65535 (the resampling CDF, a sum of N values <= 2^48, is 64-bit) */
    uint32_t n_iters;        /* K >= 1: K evaluations, K-1 resample + predict steps */
    uint64_t seed;           /* Philox4x32-10 key */
    uint32_t pair_id;        /* third Philox counter word; distinguishes pairs of a batch */
    int32_t score;           /* smc_score */
    int32_t interp;          /* smc_interp */
    double x0[6];            /* centre of the prior box */
    double limit[6];         /* half-widths of the prior box, > 0 (rotation / translation limits) */
    double sigma_score;      /* likelihood width: log w = -(z_max - z)^2 / (2 sigma^2) */
    double sigma0[6];        /* random-walk width of the first prediction, >= 0 */
    double anneal;           /* width factor per iteration, 0 < anneal <= 1 */
    double min_overlap_frac; /* NCC / SSD: overlaps under this fraction of the target FOV get weight 0 */
    int32_t rotation_mode;   /* smc_rotation */
} smc_params;

typedef struct smc_ctx smc_ctx;

/* Fig. 1 (initialisation): validate the inputs, allocate the particle set and
 * workspaces on the current device, prepare the source / target layouts and
 * per-volume statistics, and draw the prior particle set uniformly in
 * x0 +- limit.  src_fov / tgt_fov may be given inside the volumes.  Syncs once
 * (to read the volume statistics).  *out owns its device memory until
 * smc_destroy.  hip_stream is a hipStream_t (NULL = default stream). */
smc_status smc_init(smc_ctx **out, const smc_volume *src, const smc_volume *tgt, const smc_params *p,
                    void *hip_stream);

/* Draw a fresh prior particle set with a new seed and rewind to iteration 0. */
smc_status smc_reset(smc_ctx *ctx, uint64_t seed);

/* Run n_iters iterations of Fig. 1 (evaluate -> update weights -> normalise
 * and estimate -> resample -> predict); the last of the K iterations does not
 * resample.  Fails with SMC_ESTATE past K. */
smc_status smc_step(smc_ctx *ctx, uint32_t n_iters);

/* The estimate after the last completed iteration: parameters, the 3x4
 * target-mm -> source-mm matrix (row-major, Eq. 3 without its last row), the
 * estimate's own score and the effective sample size.  Any output may be
 * NULL.  Syncs.  Returns SMC_ENOOVERLAP, with the outputs written, when the
 * latest iteration's weights were all -inf. */
smc_status smc_estimate(smc_ctx *ctx, double params[6], double mat3x4[12], double *score, double *ess);

/* Host copies of the current particle set (N x 6), the log-weights of the
 * last evaluation (N) and the last ancestors (N; -1 before any resampling).
 * Any output may be NULL.  Syncs. */
smc_status smc_get_particles(smc_ctx *ctx, double *states_n6, double *logw_n, int32_t *ancestors_n);

/* Per-iteration trace (Fig. 5): score of the estimate before iteration 1 and
 * after each iteration (K + 1 values), ESS per iteration (K) and the estimate
 * per iteration (6 K).  Entries of iterations not yet run are NaN.  Syncs. */
smc_status smc_trace(smc_ctx *ctx, double *score_k1, double *ess_k, double *est_6k);

/* Score an arbitrary host particle set (n x 6) with the context's warp-and-
 * score kernel and launch configuration, returning the raw sums per particle
 * (n x 6 int64): masks (n, a, c, b_ov, 0, 0); images (n, sum s_fx, sum t,
 * sum s_fx^2, sum t^2, sum s_fx t) with s_fx the interpolated source value in
 * units of 1/256.  Uses the context's buffers; leaves the filter state alone
 * but must not overlap smc_step on the same context.  Syncs.  SMC_EINVAL for
 * the MI score, which has no moments (use smc_score_particles). */
smc_status smc_evaluate(smc_ctx *ctx, const double *states_n6, uint32_t n, int64_t *moments_n6);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: smc_evaluate
 * on a DEVICE particle set (states_dev, n x 6 FP64) into DEVICE sums
 * (moments_dev, n x 6 int64, same meaning as smc_evaluate's), asynchronous on
 * the context's stream, calling no hipMalloc / hipFree.  The per-particle
 * recipe words (48 bytes each) go to a library-wide device array of
 * SMC_NOALLOC_MAX_PARTICLES particles (3 MiB, one per device, held until the
 * process ends); the sums accumulate in moments_dev, which the call zeroes
 * first.  Every call on a device shares that array: calls that overlap on one
 * device (any context, any stream) race, so order them on one stream or
 * synchronise between them.  Both buffers are caller-owned and must stay valid
 * until the work completes; states are not checked for finiteness (non-finite
 * states count no samples).  SMC_EINVAL for n > SMC_NOALLOC_MAX_PARTICLES,
 * NULL pointers or the MI score; n == 0 does nothing. */
#define SMC_NOALLOC_MAX_PARTICLES 65536u
smc_status smc_evaluate_noalloc(smc_ctx *ctx, const double *states_dev, uint32_t n, int64_t *moments_dev);

/* Exhaustive search (the EX baseline of Baseline and Evaluation Metrics):
 * score every point of the regular grid x_d = lo[d] + step[d] c_d,
 * c_d = 0 .. count[d] - 1 (axis 0 fastest), with the context's score, and
 * return the best point (ties: lowest grid index) and its score.  scores
 * (host, prod(count) doubles) may be NULL.  Uses the smc_evaluate workspace;
 * must not overlap smc_step on the same context.  Syncs. */
smc_status smc_exhaustive(smc_ctx *ctx, const double lo[6], const double step[6], const uint32_t count[6],
                          double best_params[6], double *best_score, double *scores);

/* Replace the particle set (host N x 6) as if k_done iterations had run;
 * for step-by-step replays and resumption.  The set is not treated as a
 * proposal draw (its first update carries no importance correction).  Syncs. */
smc_status smc_set_particles(smc_ctx *ctx, const double *states_n6, uint32_t k_done);

/* Serialise / restore the whole filter state (particles, weights, estimate,
 * trace, iteration count).  smc_get_state with buf == NULL returns the size in
 * *len.  Restoring into a context made with the same inputs and parameters
 * continues bit-identically.  The state holds no proposal densities: a set
 * restored before its first update is treated as not drawn from a proposal.
 * Both sync. */
smc_status smc_get_state(smc_ctx *ctx, void *buf, size_t *len);
smc_status smc_set_state(smc_ctx *ctx, const void *buf, size_t len);

/* Final scores z (as the filter sees them: Dice, NCC, -SSD or MI; -inf
 * below the minimum overlap) of n host particle states (n x 6, FP64).
 * Syncs.  SMC_EINVAL on NULL or non-finite input. */
smc_status smc_score_particles(smc_ctx *ctx, const double *states_n6, uint32_t n, double *scores_n);

/* Multi-frame score (Related Work: rigid registration with the ED and ES
 * frames together, or all frames of the cycle): every evaluation of this
 * context -- the filter's particles and estimate, smc_evaluate,
 * smc_exhaustive -- scores each particle on its own source / target pair and
 * on n_extra further frame pairs under the same transform, adding the
 * integer sums of all pairs before the score is formed (Dice from the pooled
 * counts and the pooled |T|; NCC over the union of the overlaps, with the
 * minimum overlap taken over all target FOVs).  src_frames[q] / tgt_frames[q]
 * (host arrays of n_extra volume descriptors; the volumes are device memory
 * owned by the caller and must outlive the context) must match the first
 * pair's shapes and spacings and carry FOV masks exactly where it does.
 * n_extra = 0 removes the frames.  SMC_EINVAL for SSD (its normalisation is
 * per volume) or mismatched frames, SMC_ESTATE after the first iteration
 * (smc_reset rewinds) or on a pair owned by a batch.  Syncs once per frame. */
smc_status smc_set_frames(smc_ctx *ctx, uint32_t n_extra, const smc_volume *src_frames,
                          const smc_volume *tgt_frames);

/* Launch tuning of the warp-and-score kernel; results do not depend on it.
 * layout: trilinear source layout, 0 raw bytes (eight gathers per sample),
 * 1 x-pairs (uint16, four), 2 2x2 quads (uint32, two), 3 2x2x2 octets
 * (uint64, one), 4 the same octets stored in 4 x 4 voxel tiles of a slice
 * (one 128-byte cache line per tile, so a rotated footprint touches fewer
 * lines), 5 the octet cell stored ready for the x-interpolations (four
 * starts and four steps times 256 in half precision, 16 bytes, one gather
 * and fewer instructions per sample; layout 4 is prepared beside it and
 * serves the first iteration over a prior drawn from the uniform box, whose
 * dispersed particles gather faster from the smaller, tiled elements); packed
 * layouts cost 2, 4, 8 or 16 bytes per source voxel of device memory,
 * prepared on the stream.  particles_per_group: particles sharing one pass
 * over a target column, 4, 8 or 16.  tile_depth: target
 * slices per tile, 1 .. 256 (a tile is 32 x 8 x tile_depth voxels; shallower
 * tiles cull more exactly -- a tile whose image cannot reach the source, or
 * in the filter the source mask's bounding box or any occupied 2^3-voxel
 * cell of the source mask, is skipped -- at the cost of more partial sums).  A negative value keeps the current setting.  Defaults
 * come from measurements on MI355X: 4 particles per group; tile depth 16 for
 * masks and 256 for images.  A packed layout addresses its source
 * with 32-bit offsets: SMC_EINVAL if the packed source reaches 4 GiB or one
 * packed slice 16 MiB.  smc_init starts from layout 5, else 3 if 5 does
 * not fit, else 0. */
smc_status smc_set_tuning(smc_ctx *ctx, int32_t layout, int32_t particles_per_group, int32_t tile_depth);
smc_status smc_get_tuning(smc_ctx *ctx, int32_t *layout, int32_t *particles_per_group, int32_t *tile_depth);

/* Autotuner: time every candidate tuning (layouts for trilinear images;
 * particles per group 4 / 8; tile depths) on this context's own volumes with
 * HIP events (the fastest of reps launches each, on a scratch sum buffer) over two particle
 * sets -- the current particles (after smc_init, the prior) and a cloud
 * concentrated within 5 % of the limits around x0, standing in for the
 * iterations after the first -- and apply the tuning with the least time per
 * registration (the first set once, the second n_iters - 1 times).  Results
 * are cached per problem shape for the life of the process.  best_ms (may be
 * NULL) receives that cost per launch.  Syncs. */
smc_status smc_autotune(smc_ctx *ctx, uint32_t reps, double *best_ms);

/* Measurement: how close the warp-and-score kernel runs to the cost of its
 * source gathers alone (the warp-and-score path is bound by on-chip gather
 * throughput; Implementation Details, full-resolution scoring).  On the
 * context's current particle set -- the set (and estimate) its next
 * iteration will score -- time (HIP events on the context's stream, one
 * untimed launch then the mean of reps) a probe kernel that runs the same
 * grid, culling, coordinates, offsets and source loads and nothing else, and
 * the production kernel itself into a scratch sum buffer.  Leaves the filter
 * state alone; must not overlap smc_step on the same context.  Outputs (ms
 * per launch) may be NULL.  Syncs.  SMC_EINVAL for MI, multi-frame contexts,
 * a target FOV, or a trilinear layout other than 3, 4 or 5. */
smc_status smc_gather_probe(smc_ctx *ctx, uint32_t reps, double *probe_ms, double *score_ms);

/* Kernel timing.  With enable != 0 every warp-and-score launch and every
 * filter launch of this context is bracketed by HIP events recorded on the
 * context's stream.  smc_profile_read syncs, returns the summed durations
 * (ms) and launch counts since the last read, and clears them.  Outputs may
 * be NULL. */
smc_status smc_profile(smc_ctx *ctx, int32_t enable);
smc_status smc_profile_read(smc_ctx *ctx, double *score_ms, uint64_t *score_launches, double *filter_ms,
                            uint64_t *filter_launches);

/* Work of the filter's culled mask launches (masks, Methods: the Dice
 * evaluation; image contexts report 0).  Tile culling skips a particle for a
 * target tile, and a tile's runs of four slices at its bottom and top for all
 * its particles, when no sample there can read an "on" source voxel: the
 * image's box misses the source mask's bounding box or covers only
 * unoccupied 2^3-voxel cells.  Returns, since the previous call (or
 * smc_init), the particle x voxel pairs those launches evaluated, the pairs
 * they covered (the skipped ones included) and, of the evaluated ones, those
 * of tiles whose every sample the cull bound places inside the source (scored
 * without the per-sample inside test), and clears all three.  Syncs the
 * context's stream.  Outputs may be NULL. */
smc_status smc_profile_work(smc_ctx *ctx, uint64_t *evaluated, uint64_t *covered, uint64_t *interior);

/* Free everything the context owns (after syncing its stream).  NULL is a no-op. */
void smc_destroy(smc_ctx *ctx);

/* Methods (whole-cycle registration): apply one 3x4 target-mm -> source-mm
 * matrix to n_frames source frames, writing uint8 volumes on the target grid
 * (nx, ny, nz, spacing sx, sy, sz).  NEAREST copies the source byte; TRILINEAR
 * writes floor(v + 0.5); target voxels whose source position falls outside
 * the source grid get 0.  Frame f is read at src->data + f * src_frame_stride
 * and written at dst + f * dst_frame_stride (bytes).  src->fov is ignored.
 * Asynchronous on hip_stream.  SMC_EINVAL for NULL pointers, non-finite
 * matrix entries, an unknown interp, output dimensions outside 1..65535 or an
 * output frame of 2^31 voxels or more, non-positive spacing, n_frames outside
 * 1..65535 or frame strides smaller than a frame; SMC_EDEVICE if the launch fails. */
smc_status warp_apply(const smc_volume *src, const double mat3x4[12], int32_t interp, uint8_t *dst,
                      int32_t nx, int32_t ny, int32_t nz, double sx, double sy, double sz, uint32_t n_frames,
                      int64_t src_frame_stride, int64_t dst_frame_stride, void *hip_stream);

/* ---- Learned proposal (the machine-learning direction of the Conclusion).
 * A 3D CNN reads the source / target pair downsampled to 64^3 (FP16, two
 * channels) and predicts, in units of the limits, a Gaussian over the
 * transform: 6 means and 6 log-variances.  Four 3x3x3 stride-2
 * convolutions (2 -> 16 -> 32 -> 64 -> 64 channels, zero padding 1, bias,
 * ReLU; bfloat16 weights and activations, FP32 accumulation on the matrix
 * cores), flatten (channel-major) and a linear head 4096 -> 12 (FP32).
 * Trained with the Gaussian negative log-likelihood of the filter's final
 * weighted particle cloud, 0.5 sum_d [(var_d + (xbar_d - mu_d)^2) e^-l_d + l_d]
 * averaged over the batch, and Adam (beta 0.9 / 0.999, eps 1e-8).
 * Flat parameter layout (229,916 FP32): W1[16][2][27] b1[16] W2[32][16][27]
 * b2[32] W3[64][32][27] b3[64] W4[64][64][27] b4[64] Wh[12][4096] bh[12], the
 * 27 kernel taps ordered (kz, ky, kx). */
typedef struct smc_cnn smc_cnn;

/* Workspaces for batches of up to max_batch (1 .. 1024) pairs. */
smc_status smc_cnn_create(smc_cnn **out, uint32_t max_batch, void *hip_stream);
smc_status smc_cnn_set_params(smc_cnn *net, const float *host_params, size_t n);   /* syncs; resets Adam */
smc_status smc_cnn_get_params(smc_cnn *net, float *host_params, size_t n);         /* syncs */
/* Downsample a source / target pair into input slot `slot`: trilinear at
 * half-pixel centres to 64^3, times `scale`, stored as FP16. */
smc_status smc_cnn_input(smc_cnn *net, uint32_t slot, const smc_volume *src, const smc_volume *tgt, float scale);
/* Copy input slot `slot` (2 x 64^3 FP16 bit patterns, source then target) to
 * the host.  Syncs. */
smc_status smc_cnn_read_input(smc_cnn *net, uint32_t slot, uint16_t *host);
/* Outputs of slots 0 .. B-1: B x 12 (6 means, 6 log-variances), host.  Syncs. */
smc_status smc_cnn_forward(smc_cnn *net, uint32_t B, float *out_host);
/* Forward + backward of slots 0 .. B-1 against targets (B x 12 host: the
 * cloud's means then variances, in units of the limits).  Returns the loss;
 * grads_host (229,916 floats) may be NULL.  Syncs. */
smc_status smc_cnn_backward(smc_cnn *net, uint32_t B, const float *target_host, float *loss, float *grads_host);
/* One Adam step with the gradients of the last smc_cnn_backward. */
smc_status smc_cnn_step(smc_cnn *net, float lr);
void smc_cnn_destroy(smc_cnn *net);

/* Draw the next prior (smc_reset) from the Gaussian N(mean, exp(logvar))
 * truncated to x0 +- limit instead of the uniform box; the first update of a
 * set so drawn is corrected by log p - log q.  mean == NULL returns to the
 * uniform prior for the next draw.  Neither changes the current particle set
 * or its correction: a set drawn from the uniform box is never corrected, a
 * set drawn from a proposal always is.  mean and logvar are host arrays of 6
 * (radians, mm; logvar in [-60, 60]).  SMC_EINVAL on non-finite values. */
smc_status smc_set_proposal(smc_ctx *ctx, const double mean[6], const double logvar[6]);

/* Training label of the proposal network: the weighted particle cloud after
 * the last completed iteration, summarised with the normalised weights
 * exp(lw_i - max lw) of that iteration's evaluation (uniform when every
 * log-weight is -inf) as its weighted mean and per-axis weighted variance,
 * in units of the limits about x0: mean[d] = (xbar_d - x0_d) / L_d,
 * var[d] = max(Var_d / L_d^2, var_floor).  Host outputs of 6.  Syncs.
 * SMC_ESTATE before the first iteration; SMC_EINVAL on NULL outputs or a
 * negative / non-finite var_floor. */
smc_status smc_cloud_moments(smc_ctx *ctx, double var_floor, double mean[6], double var[6]);

/* Set the proposal (as smc_set_proposal, for the next prior draw) from the
 * network's 12 outputs (host FP32: 6 means and 6 log-variances in units of
 * the limits): mean_d = x0_d + L_d clip(out_d, -1, 1), logvar_d =
 * clip(out_{6+d}, -20, 2) + 2 log L_d + log var_scale, where var_scale > 0
 * widens the predicted spread.  mean_out / logvar_out (host, may be NULL)
 * receive the values set.  SMC_EINVAL on non-finite outputs or var_scale. */
smc_status smc_set_proposal_from_network(smc_ctx *ctx, const float out[12], double var_scale, double mean_out[6],
                                         double logvar_out[6]);

/* ---- Batches: many registration pairs of uneven size and particle count
 * run together.  Every pair behaves exactly as its own smc_init /
 * smc_step context would (the pair id sits in the Philox counter), but the
 * warp-and-score work of all pairs of a class (masks; trilinear images)
 * shares one persistent launch per iteration, the filters of all pairs
 * share one launch, and the whole run -- prior draws, every iteration,
 * final scores -- is captured once into a HIP graph and replayed by each
 * smc_batch_run.  The batch owns a stream of its own; smc_batch_run orders
 * it after the caller's stream and the caller's stream after it. */
typedef struct smc_batch smc_batch;

/* src, tgt and p are arrays of n_pairs (1 .. 4096).  All trilinear image
 * pairs take the first image pair's launch tuning and all mask pairs the
 * first mask pair's particles per group (one kernel instance serves a
 * class); SMC_EINVAL if a pair cannot take it.  Syncs once per pair. */
smc_status smc_batch_init(smc_batch **out, uint32_t n_pairs, const smc_volume *src, const smc_volume *tgt,
                          const smc_params *p, void *hip_stream);
/* New prior seeds for the next run (one per pair; NULL keeps them). */
smc_status smc_batch_set_seeds(smc_batch *b, const uint64_t *seeds);
/* Run every pair's full registration (one graph launch).  Async. */
smc_status smc_batch_run(smc_batch *b);
/* Autotune the largest pair of each class (masks, trilinear images), apply
 * the result to every pair of that class and re-plan the batch (the graph is
 * recaptured at the next run).  Syncs. */
smc_status smc_batch_autotune(smc_batch *b, uint32_t reps);
/* The context of pair i, for smc_estimate / smc_get_particles / smc_trace
 * (do not step or destroy it); NULL if i is out of range. */
smc_ctx *smc_batch_pair(smc_batch *b, uint32_t i);
void smc_batch_destroy(smc_batch *b);

/* Message of the last failed call on this thread ("" if none). */
const char *smc_last_error(void);

/* Library version string. */
const char *smc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMC_H */
