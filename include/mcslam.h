/*
 * mcslam.h -- C ABI of the MI355X (gfx950) gradient-guided Monte Carlo SLAM
 * particle update.
 *
 * Paper: T. Nakao et al., "Range-based 6-DoF Monte Carlo SLAM with
 * Gradient-guided Particle Filter on GPU" (arXiv 2504.18056).
 *
 * The calls follow the paper's statement of the problem (Sec. III-A): a set
 * of N particles, each holding a current sensor pose T_i (and, with a
 * keyframe map, one pose per keyframe, Sec. III-A "Particle state"), is
 * updated from a range scan P_t of points in the sensor frame and the relative
 * motion dT from odometry (Sec. III-B).  One filter step is, per particle:
 *
 *   prediction    T_i <- T_i dT Exp(delta_i)                       Eq. 1
 *   likelihood    l_i = sum_j ln(G(u_ij) + eps), G the trilinear interpolant
 *                 of a likelihood grid at the transformed point
 *                 u_ij = (R_i p_j + t_i - o)/h - 1/2; with a keyframe map,
 *                 summed over neighbour keyframes under T_k^-1 T_i       Eq. 2-4
 *   gradient      g_i = d l_i(T_i Exp(xi)) / d xi, xi = [rho; phi]
 *   pose step     psi = [a_t g_rho; a_r g_phi] (norm-clamped per block),
 *                 T_i <- T_i Exp(psi)                                  Eq. 7
 *   weighting     logw_i += beta l_i                                   Eq. 11
 *   normalising   L = logsumexp(logw), logw -= L, ESS = 1 / sum w^2
 *   resampling    systematic, a_k = min{i : CDF_i > (u + k)/N}
 *                 (the library's counterpart of Sec. III-F's respawning of
 *                 particles from the weights of the remaining ones)
 *
 * Conventions
 *   Poses are rows [tx ty tz qw qx qy qz] of FP32: translation in metres and a
 *   unit Hamilton quaternion, active body-to-world.  Quaternions returned by
 *   the library have qw >= 0.
 *   Grids hold nx*ny*nz samples, x fastest, at world points
 *   origin + (i + 1/2) * res.  A point is inside when its index coordinate
 *   u satisfies 0 <= u < n - 1 on every axis.
 *   Scans are M rows [x y z] of FP32 in the sensor frame.
 *
 * Ownership and errors
 *   Host pointers passed in are read during the call only and copied; the
 *   caller keeps ownership.  Device pointers (the *_dev calls) are borrowed
 *   until the work enqueued by the call has completed on its stream.  Every
 *   call returns MCS_OK (0) or a negative mcs_status; no call aborts or throws
 *   across the ABI.  mcs_last_error() gives a message for the last failing
 *   call of the calling thread.
 *
 * Threading
 *   Map and session tables are locked per context.  A session must not be
 *   driven by two threads at the same time.  mcs_filter_step* only enqueue
 *   work; mcs_get_particles and mcs_session_sync wait for it.
 */
#ifndef MCSLAM_H
#define MCSLAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mcs_status;

#define MCS_OK         0
#define MCS_EINVAL    -1   /* bad argument (size, pointer, NaN in host input, ...) */
#define MCS_ENOMEM    -2   /* device allocation failed */
#define MCS_EBUDGET   -3   /* admission refused: the HBM budget would be exceeded */
#define MCS_ENOTFOUND -4   /* unknown context, map or session id */
#define MCS_EDEVICE   -5   /* HIP runtime error */
#define MCS_EBUSY     -6   /* object still in use (e.g. a map referenced by a session) */

typedef struct mcs_ctx mcs_ctx;

/* Grid storage types.  FP16 and BF16 grids are rounded from the FP32 values
 * to nearest, ties to even, when the map is loaded; all arithmetic is FP32. */
#define MCS_GRID_FP32 0
#define MCS_GRID_FP16 1
#define MCS_GRID_BF16 2

typedef struct {
    int32_t nx, ny, nz;     /* samples per axis, each >= 2 */
    float origin[3];        /* world position of the corner of voxel (0,0,0) */
    float res;              /* voxel edge h in metres, > 0 */
    int32_t dtype;          /* MCS_GRID_* */
} mcs_grid_desc;

/* Resampling policy. */
#define MCS_RESAMPLE_NEVER  0
#define MCS_RESAMPLE_ALWAYS 1
#define MCS_RESAMPLE_ESS    2   /* when ESS < ess_frac * N (strict) */
/* Dead-particle pruning (Sec. III-F) instead of resampling: a particle is dead
 * when its normalised weight is below prune_post or its likelihood relative
 * to the frame's best, exp(l_i - max l), is below prune_lik.  Each dead slot,
 * in index order, receives a copy (pose and keyframe poses) of a live
 * particle drawn systematically with offset u from the live weights; a
 * parent's weight is shared equally with its copies and the live mass is
 * renormalised.  Live particles keep their state and relative weights. */
#define MCS_RESAMPLE_PRUNE  3

/* Prediction noise: from the noise pointer (or none), or drawn on the device
 * (Eq. 1) from a counter-based SplitMix64 stream with Box-Muller normals:
 * the stream of frame f is keyed by the f-th output of SplitMix64(rng_seed);
 * particle i takes its uniforms 6i .. 6i+5, U = (x >> 11) 2^-53, in pairs
 * (U_a, U_b) -> sqrt(-2 ln(1 - U_a)) (cos, sin)(2 pi U_b); delta_c = sigma_c z_c. */
#define MCS_NOISE_INPUT  0
#define MCS_NOISE_DEVICE 1

/* Points outside the grid: ln(eps) (FLOOR) or no contribution (SKIP). */
#define MCS_OOB_FLOOR 0
#define MCS_OOB_SKIP  1

/* Keyframe maps: how a step corrects a particle's state (Sec. III-C.2).
 * FIXED: every pass steps the current pose; keyframe poses never change.
 * LOOP:  a particle whose neighbour keyframes include an old one (index below
 *        K - n_recent; keyframes are numbered in time order) has detected a
 *        loop; only such a particle is corrected: its current pose by the step
 *        psi (Eq. 7) and each keyframe k from its oldest neighbour o to the
 *        newest by psi_k = (d_k / d_t) psi, T_k <- T_k Exp(psi_k) (Eq. 8-10),
 *        where d_k is the path length along the particle's keyframe
 *        translations from o to k and d_t adds the segment from the newest
 *        keyframe to the current translation before the step.  Keyframes older
 *        than o do not move; when d_t = 0 none moves. */
#define MCS_KF_FIXED 0
#define MCS_KF_LOOP  1

typedef struct {
    int32_t iters;          /* gradient passes per step, >= 1 */
    float alpha_t;          /* translation gain a_t (m per unit gradient) */
    float alpha_r;          /* rotation gain a_r (rad per unit gradient) */
    float rho_max;          /* clamp of |psi_rho| per pass (m) */
    float phi_max;          /* clamp of |psi_phi| per pass (rad) */
    float eps;              /* likelihood floor in ln(G + eps), in [1e-5, 1] on
                               grid maps (MCS_EINVAL otherwise) */
    float beta;             /* weight exponent: logw += beta * l */
    int32_t oob;            /* MCS_OOB_* */
    int32_t post_eval;      /* 0: weight with l of the last pass (taken before
                               its step); 1: one more likelihood-only pass at
                               the final pose supplies l */
    int32_t resample;       /* MCS_RESAMPLE_* */
    double ess_frac;        /* threshold for MCS_RESAMPLE_ESS */
    double u;               /* systematic offset in [0, 1) */
    int32_t predict;        /* 1: apply Eq. 1 with delta_T (and noise) first */
    float delta_T[7];       /* odometry dT as a pose row */
    int32_t n_neighbors;    /* keyframe maps: neighbour keyframes per particle */
    int32_t kf_update;      /* keyframe maps: MCS_KF_FIXED or MCS_KF_LOOP */
    int32_t n_recent;       /* MCS_KF_LOOP: the newest n_recent keyframes are not old
                               (with n_recent < n_neighbors every particle loops;
                               n_recent = n_neighbors is the natural choice) */
    int32_t noise_mode;     /* MCS_NOISE_* (used when predict is set) */
    uint64_t rng_seed;      /* MCS_NOISE_DEVICE: stream seed */
    uint64_t rng_frame;     /* MCS_NOISE_DEVICE: frame counter */
    float noise_sigma[6];   /* MCS_NOISE_DEVICE: standard deviations [rho (m); phi (rad)] */
    float prune_post;       /* MCS_RESAMPLE_PRUNE: weight threshold (e.g. 1e-8), > 0 */
    float prune_lik;        /* MCS_RESAMPLE_PRUNE: likelihood-ratio threshold (e.g. 1e-16), > 0 */
} mcs_step_params;

typedef struct {
    double lse;             /* L = logsumexp of the updated log-weights */
    double ess;             /* effective sample size 1 / sum w^2 */
    int32_t resampled;      /* 1 when this step resampled */
    int32_t best;           /* index (before resampling) of the largest weight, lowest on ties */
    float best_pose[7];     /* that particle's pose after the step (the representative) */
    int32_t degenerate;     /* 1 when no log-weight was finite: weights reset to uniform */
    int32_t pruned;         /* MCS_RESAMPLE_PRUNE: dead particles respawned in this step */
} mcs_step_stats;

/* Library version string. */
const char *mcs_version(void);

/* Message describing the last failing call on this thread ("" if none). */
const char *mcs_last_error(void);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory that maps and sessions of this context may hold (0: no bound). */
mcs_status mcs_create(int32_t device, uint64_t hbm_budget_bytes, mcs_ctx **out);

/* Destroy a context: waits for all sessions' queued work, then frees
 * everything it owns.  NULL is accepted. */
mcs_status mcs_destroy(mcs_ctx *ctx);

/* Bytes of device memory currently held by the context's maps and sessions. */
mcs_status mcs_memory_in_use(mcs_ctx *ctx, uint64_t *bytes);

/* Load a likelihood grid map (the map M of Sec. III-A, as one grid).
 * values: host FP32, nx*ny*nz samples, x fastest, each a likelihood in
 * [0, 1] (MCS_EINVAL for a sample outside it or not finite).  The device keeps the grid
 * in a cell-major layout holding the 8 corner samples of each cell together,
 * converted to desc->dtype, (nx+1)(ny+1)(nz+1) records in all (32 B each for
 * FP32, 16 B for FP16/BF16); MCS_EINVAL for 2^32 records or more, MCS_EBUDGET
 * when they do not fit the context's budget.  Returns the map id in *map_id. */
mcs_status mcs_init_map(mcs_ctx *ctx, const mcs_grid_desc *desc, const float *values,
                        int32_t *map_id);

/* Load a keyframe map: K local grids, one per keyframe, each in its own
 * keyframe frame (Sec. III-A, "Particle state"; Fig. 2).  All descs must have
 * the same nx, ny, nz, res and dtype; origins may differ.  values[k] is host
 * FP32 for keyframe k, samples in [0, 1] as for mcs_init_map.  Sessions on such a map hold N*K keyframe poses.
 * Each grid's records must fit 4 GiB and (nx+1)(ny+1) stay below 2^24 (MCS_EINVAL otherwise). */
mcs_status mcs_load_keyframes(mcs_ctx *ctx, int32_t K, const mcs_grid_desc *descs,
                              const float *const *values, int32_t *map_id);

/* Keyframes inserted one at a time (Sec. III-E: the keyframe list grows as the
 * sensor moves; when to insert is the caller's decision).  A keyframe map
 * with room for K_cap grids of the shape and dtype of desc starts empty.
 * MCS_EBUDGET when the capacity does not fit the budget. */
mcs_status mcs_create_keyframe_map(mcs_ctx *ctx, int32_t K_cap, const mcs_grid_desc *desc,
                                   int32_t *map_id);

/* Append keyframe *index = K (keyframes are numbered in insertion, i.e. time,
 * order) to a keyframe grid map: desc gives its origin in its own frame and
 * must match the map's shape, res and dtype; values as for
 * mcs_load_keyframes.  MCS_EBUSY when the map is full.  Sessions on the map
 * see the keyframe once they add it (mcs_session_add_keyframe). */
mcs_status mcs_append_keyframe(mcs_ctx *ctx, int32_t map_id, const mcs_grid_desc *desc,
                               const float *values, int32_t *index);

/* Give the session's particles their pose of the next keyframe of its map
 * (index *index): each particle's current pose, copied on the session's
 * stream after its queued steps.  MCS_EINVAL when the map has no further
 * keyframe.  A session on a keyframe map needs at least one keyframe before
 * its first step. */
mcs_status mcs_session_add_keyframe(mcs_ctx *ctx, int32_t session_id, int32_t *index);

/* Release a map.  MCS_EBUSY while a session uses it. */
mcs_status mcs_release_map(mcs_ctx *ctx, int32_t map_id);

/* Create a filter session of N particles on a map, for scans of up to M_max
 * points.  poses: host N*7.  kf_poses: host N*K*7 (particle-major: particle
 * i's pose of keyframe k at (i*K + k)*7) for keyframe maps, else NULL.
 * Log-weights start at -ln N.  Returns MCS_EBUDGET when the session's device
 * memory would exceed the context budget. */
mcs_status mcs_session_create(mcs_ctx *ctx, int32_t map_id, int32_t N, int32_t M_max,
                              const float *poses, const float *kf_poses, int32_t *session_id);

/* Destroy a session after its queued work has completed. */
mcs_status mcs_session_destroy(mcs_ctx *ctx, int32_t session_id);

/* Bytes of device memory a session with these sizes would hold. */
mcs_status mcs_session_bytes(mcs_ctx *ctx, int32_t map_id, int32_t N, int32_t M_max,
                             uint64_t *bytes);

/* Overwrite the particle state (checkpoint restore).  Any pointer may be NULL
 * to keep that part.  poses N*7, logw N, kf_poses N*K*7. */
mcs_status mcs_set_particles(mcs_ctx *ctx, int32_t session_id, const float *poses,
                             const double *logw, const float *kf_poses);

/* One filter step (the sequence at the top of this file) on host inputs.
 * scan: M*3 host FP32 (1 <= M <= M_max); noise: N*6 host FP32 tangent-space
 * prediction noise [rho; phi] per particle, or NULL for none (used only when
 * p->predict).  Non-finite scan values give MCS_EINVAL.  Enqueues on the
 * session's stream and returns. */
mcs_status mcs_filter_step(mcs_ctx *ctx, int32_t session_id, const float *scan, int32_t M,
                           const float *noise, const mcs_step_params *p);

/* As mcs_filter_step with device pointers: scan_dev M*3 FP32, noise_dev N*6
 * FP32 or NULL.  stream: a hipStream_t to enqueue on, or NULL for the
 * session's stream.  Points with non-finite coordinates count as outside the
 * grid. */
mcs_status mcs_filter_step_dev(mcs_ctx *ctx, int32_t session_id, const float *scan_dev,
                               int32_t M, const float *noise_dev, const mcs_step_params *p,
                               void *stream);

/* Measurement aid: the gather floor of the evaluation passes.  Enqueues, like
 * mcs_filter_step_dev without prediction, weighting or resampling, p->iters
 * passes over the session's current poses with the same tiling, the same
 * transformed coordinates (FP64, Sec. III-C.1's u = (R p + t - o)/h - 1/2)
 * and the same grid-record loads as the likelihood passes, but with the
 * arithmetic cut to a checksum of the gathered words: its time is what the
 * record loads alone cost.  The session's l becomes that checksum and g zero;
 * translations are unchanged and quaternions renormalised.  With per-stage
 * timing on (mcs_session_profile) the passes count as the evaluation stage.
 * Single-grid sessions only (MCS_EINVAL otherwise); p is validated as for
 * mcs_filter_step (only iters and M are used). */
mcs_status mcs_gather_floor_dev(mcs_ctx *ctx, int32_t session_id, const float *scan_dev,
                                int32_t M, const mcs_step_params *p, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one filter
 * step, the same as mcs_filter_step_dev, of N particles on a single-grid map
 * (from mcs_init_map), with the particle state and the outputs in the
 * caller's device memory and every temporary of the step (packed scan,
 * resampling copies, CDF and partial sums, statistics) in one static device
 * area of 32 MiB per GPU, which the library holds from the first mcs_create
 * on that GPU until the process ends.  The call allocates nothing.
 *   pose_dev     [7][N] FP32, rows tx ty tz qw qx qy qz (in/out; quaternion
 *                signs as the step leaves them)
 *   logw_dev     [N] FP64 log-weights (in/out)
 *   loglik_dev   [N], grad_dev [6][N] FP32: l and g of the last gradient pass
 *   parents_dev  [N] int32 ancestors (identity when not resampled)
 *   scan_dev     M*3 FP32; noise_dev N*6 FP32 or NULL, as for
 *                mcs_filter_step_dev
 *   stats_dev    one mcs_step_stats in device memory, or NULL
 *   stream       hipStream_t to enqueue on (NULL: the null stream)
 * Limits: 1 <= N <= MCS_NOALLOC_MAX_PARTICLES, 1 <= M <=
 * MCS_NOALLOC_MAX_POINTS (MCS_EINVAL beyond them), single-grid maps only
 * (MCS_EINVAL for keyframe or GICP maps).  Every call on one GPU uses that
 * GPU's one area, which keeps the last call's contents: calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by
 * the caller.  The map must stay loaded until the enqueued work completes. */
#define MCS_NOALLOC_MAX_PARTICLES 262144
#define MCS_NOALLOC_MAX_POINTS    16384
mcs_status mcs_filter_step_noalloc(mcs_ctx *ctx, int32_t map_id, int32_t N, float *pose_dev,
                                   double *logw_dev, float *loglik_dev, float *grad_dev,
                                   int32_t *parents_dev, const float *scan_dev, int32_t M,
                                   const float *noise_dev, const mcs_step_params *p,
                                   mcs_step_stats *stats_dev, void *stream);

/* ------------------------------------------------------------------------ */
/* GICP likelihood and Gauss-Newton correction (Sec. III-C, Eq. 2-7)          */
/* ------------------------------------------------------------------------ */

/* A keyframe's voxel map for the distribution-to-distribution (GICP)
 * likelihood with voxel correspondences: voxel (i, j, k) covers
 * [origin + (i, j, k) edge, origin + (i+1, j+1, k+1) edge) in the keyframe's
 * frame. */
typedef struct {
    int32_t nx, ny, nz;     /* voxels per axis, 1 .. 65536 */
    float origin[3];
    float edge;             /* voxel edge (m), > 0 */
} mcs_voxel_desc;

/* Load K keyframe voxel maps (all of one shape and edge).  voxels[k]: host
 * nx*ny*nz*12 FP32, x fastest: the mean of the keyframe's points in the
 * voxel (3), their count (0: empty voxel), their covariance
 * (xx xy xz yy yz zz), 2 unused.  Sessions on the map carry per-particle
 * keyframe poses as for mcs_load_keyframes and are stepped with
 * mcs_filter_step_gicp*.  Errors: MCS_EINVAL, MCS_EBUDGET, MCS_ENOMEM. */
mcs_status mcs_load_gicp_keyframes(mcs_ctx *ctx, int32_t K, const mcs_voxel_desc *descs,
                                   const float *const *voxels, int32_t *map_id);

/* One filter step with the GICP likelihood (Eq. 2-4) and Gauss-Newton passes
 * (Eq. 5-7) on a voxel keyframe map.  mu: M*3 scan point means, cov: M*6
 * their covariances (xx xy xz yy yz zz), sensor frame.  For each particle and
 * each of its n_neighbors keyframes (chosen as for grid keyframes), a point
 * x = kT mu (kT = T_k^-1 T) takes the Gaussian (mu', S') of the voxel holding
 * it, if any; l = -sum e^T Omega e with e = mu' - x and
 * Omega = (S' + R Sigma R^T)^-1 (R the rotation of kT); H and b of Eq. 6 in
 * the body frame; psi = -H^-1 b (Cholesky; no step when H is not positive
 * definite), each block clamped to rho_max / phi_max, T <- T Exp(psi).  The
 * step's alpha_t, alpha_r and eps are not used.  kf_update, weights,
 * resampling and pruning work as in mcs_filter_step.  Returns MCS_EINVAL on a
 * grid map (and mcs_filter_step returns MCS_EINVAL on a voxel map). */
mcs_status mcs_filter_step_gicp(mcs_ctx *ctx, int32_t session_id, const float *mu, const float *cov,
                                int32_t M, const float *noise, const mcs_step_params *p);

/* As mcs_filter_step_gicp with device pointers and an optional stream. */
mcs_status mcs_filter_step_gicp_dev(mcs_ctx *ctx, int32_t session_id, const float *mu_dev,
                                    const float *cov_dev, int32_t M, const float *noise_dev,
                                    const mcs_step_params *p, void *stream);

/* The Gauss-Newton system of the last stepping pass of a GICP session (after
 * waiting for its work): H N*21 (upper triangle of the 6x6, row-major, [rho;
 * phi] order) and b N*6, indexed before resampling.  Either may be NULL. */
mcs_status mcs_get_gicp_system(mcs_ctx *ctx, int32_t session_id, float *H, float *b);

/* Wait for the session's queued work, then copy out the state.  Any output
 * may be NULL.  poses N*7; logw N (FP64, normalised); parents N (ancestor of
 * each particle in the last step, identity when it did not resample); loglik N
 * and grad N*6 (l and g of the last gradient pass, indexed before
 * resampling); kf_poses N*K*7; stats of the last step. */
mcs_status mcs_get_particles(mcs_ctx *ctx, int32_t session_id, float *poses, double *logw,
                             int32_t *parents, float *loglik, float *grad, float *kf_poses,
                             mcs_step_stats *stats);

/* Keyframe sessions: the neighbour keyframes each particle used in the last
 * step, nearest first (Sec. III-C.1; squared translation distances in FP32,
 * ties to the smaller index).  out: N * n_neighbors int32, particle-major,
 * indexed before resampling.  *n_neighbors receives the count (may be NULL). */
mcs_status mcs_get_neighbors(mcs_ctx *ctx, int32_t session_id, int32_t *out,
                             int32_t *n_neighbors);

/* Sizes of a session: N particles, K keyframes the session has (0 on a
 * single grid), M_max, and the neighbours per particle of its last keyframe
 * step (0 before one).  Any output may be NULL.  The outputs of
 * mcs_get_particles (N*7, N, N*6, N*K*7) and mcs_get_neighbors
 * (N*last_nb) must be sized from these; K grows with
 * mcs_session_add_keyframe and last_nb with each keyframe step. */
mcs_status mcs_session_info(mcs_ctx *ctx, int32_t session_id, int32_t *N, int32_t *K,
                            int32_t *M_max, int32_t *last_nb);

/* Pass trace, for checking the passes of a step one at a time (Sec. III-C.2,
 * Eq. 7: each pass evaluates l and g at the pose the previous pass stepped
 * to).  With max_passes >= 1 every later step of the session records, for
 * each of its passes (iters gradient passes, then the likelihood-only pass of
 * post_eval), the pose the pass evaluated, its l and its body-frame g;
 * max_passes = 0 stops recording and frees the record.  The record is
 * max_passes * 14 * N * 4 bytes of device memory, counted against the
 * budget (MCS_EBUDGET).  While it is on, a step with more than max_passes
 * passes returns MCS_EINVAL.  Likelihood-grid maps only (MCS_EINVAL on a
 * GICP map); 1 <= max_passes <= 65. */
mcs_status mcs_session_trace(mcs_ctx *ctx, int32_t session_id, int32_t max_passes);

/* Pass `pass` (0-based) of the last traced step, after waiting for it:
 * poses N*7 (the pose as the pass held it: pass 0 sees the input pose, or the
 * predicted one, with its quaternion normalised in FP32; the sign of the
 * quaternion is left as it is), loglik N and grad N*6, indexed before
 * resampling.  Any output may be NULL.  MCS_EINVAL without a trace or for a
 * pass outside [0, max_passes). */
mcs_status mcs_get_pass_trace(mcs_ctx *ctx, int32_t session_id, int32_t pass, float *poses,
                              float *loglik, float *grad);

/* Wait for the session's queued work. */
mcs_status mcs_session_sync(mcs_ctx *ctx, int32_t session_id);

/* The session's own stream (a hipStream_t), e.g. for event timing. */
mcs_status mcs_session_stream(mcs_ctx *ctx, int32_t session_id, void **stream);

/* GPU time per stage of the steps enqueued while profiling was on, from HIP
 * events recorded on the stream each step ran on. */
typedef struct {
    double predict_ms;      /* scan packing + prediction */
    double eval_ms;         /* likelihood, gradient and pose-step passes */
    double weights_ms;      /* weighting, log-sum-exp, ESS */
    double resample_ms;     /* normalisation and systematic resampling */
    int64_t steps;          /* steps measured */
    int64_t evals;          /* particle x point evaluations in those steps */
} mcs_profile;

/* Turn per-stage event timing on (1) or off (0) for a session; either way the
 * accumulated figures are reset. */
mcs_status mcs_session_profile(mcs_ctx *ctx, int32_t session_id, int32_t enable);

/* Wait for the session's profiled steps and return the accumulated times. */
mcs_status mcs_session_profile_read(mcs_ctx *ctx, int32_t session_id, mcs_profile *out);

/* VALU issue rates of the device by instruction class: a measurement aid for
 * the roofline of the evaluation kernels, not part of the filter.  Each class
 * runs eight independent dependency chains per lane over a grid that fills
 * the device several times; rates[c] is lane-operations per second (an FMA
 * counts once) for class c, timed with HIP events on the null stream. */
typedef enum {
    MCS_RATE_FP32_FMA = 0,     /* v_fmac_f32 */
    MCS_RATE_FP64_FMA = 1,     /* v_fmac_f64 */
    MCS_RATE_FP64_UNARY = 2,   /* v_fract_f64 (the class of v_floor_f64 and v_cvt_*_f64) */
    MCS_RATE_INT24 = 3,        /* v_mad_u32_u24 */
    MCS_RATE_TRANS = 4,        /* v_rcp_f32 (the class of v_log_f32) */
    MCS_RATE_FP32_FP64 = 5,    /* v_fmac_f32 and v_fmac_f64 alternating */
    MCS_RATE_COUNT = 6
} mcs_rate_class;

/* rates: caller's host array of n >= MCS_RATE_COUNT doubles.  Takes about a
 * second; runs on the context's device.  Errors: MCS_EINVAL (NULL, n too
 * small), MCS_EDEVICE. */
mcs_status mcs_measure_issue_rates(mcs_ctx *ctx, double *rates, int32_t n);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop over many concurrent sessions                     */
/* ------------------------------------------------------------------------ */

/* Each particle, and so each session, updates independently (Sec. III-A), so
 * the steps of many sessions can share the device.  A server owns a worker
 * thread that takes submitted frame requests and, in MCS_SERVE_BATCHED mode,
 * runs them in two lanes side by side.  Frames of sessions large enough to
 * fill the device on their own (a round of evaluation tiles: 512 x 64
 * particles on MI355X) are launched as they arrive with the per-session
 * launches on the session's own stream, so they overlap each other and the
 * ticks (at most 256 in flight).  Frames of smaller sessions run
 * in ticks: a tick takes the oldest pending frame, then the smallest pending
 * frames of other sessions (at most one per session, up to max_batch) while
 * its evaluations stay under a cap of one round's worth at 2,048 points and 3
 * passes; it writes a table of per-session step descriptors and work items
 * and replays one captured HIP graph of persistent kernels that process all
 * sessions' work items together; up to two ticks are in flight, so frames
 * arriving while a tick runs join a later one.  A session's frames always run
 * in submission order.
 * Results are identical to mcs_filter_step_dev on the same inputs (the
 * kernels and their reduction order do not depend on the batch).
 * MCS_SERVE_CONCURRENT launches each request as soon as it arrives, with the
 * plain per-session launches on the session's own stream, so frames of
 * different sessions run side by side on the device with no tick boundary
 * (at most 256 requests in flight).  While a server holds requests of a
 * session, the session must not be stepped directly.
 * MCS_SERVE_SERIAL runs one request at a time with the plain per-session
 * launches and waits for each (the one-session-at-a-time baseline).
 * A completion thread retires each request as soon as its work is done.
 * Sessions served must be single-grid sessions whose map has the server's grid
 * dtype; admission to device memory is the context's HBM budget
 * (mcs_session_create returns MCS_EBUDGET when it would be exceeded). */
typedef struct mcs_server mcs_server;

#define MCS_SERVE_BATCHED    0
#define MCS_SERVE_SERIAL     1
#define MCS_SERVE_CONCURRENT 2

typedef struct {
    int64_t submit_ns;      /* host steady-clock time of mcs_server_submit */
    int64_t launch_ns;      /* when the worker enqueued the request's work */
    int64_t done_ns;        /* when the worker saw the work complete */
    int32_t session_id;
    int32_t tick;           /* tick (or launch slot) that ran it */
} mcs_request_times;

typedef struct {
    int64_t requests;       /* completed requests */
    int64_t ticks;          /* ticks (or single-request launches) run */
    int64_t evals;          /* particle x point evaluations completed */
    int32_t max_batch_seen; /* most sessions in one tick (CONCURRENT: most requests in flight) */
    int32_t pad;
} mcs_server_stats;

/* Create a server on ctx.  mode: MCS_SERVE_*; dtype: grid dtype of the
 * sessions it serves; oob: MCS_OOB_*; max_batch: sessions per tick (>= 1);
 * max_items: capacity of each per-stage work list per tick (0: 262144). */
mcs_status mcs_server_create(mcs_ctx *ctx, int32_t mode, int32_t dtype, int32_t oob,
                             int32_t max_batch, int32_t max_items, mcs_server **out);

/* Complete every submitted request, stop the worker and free the server. */
mcs_status mcs_server_destroy(mcs_server *srv);

/* Queue one frame of a session: scan_dev (M*3 FP32) and noise_dev (N*6 FP32 or
 * NULL) are device pointers borrowed until the request completes; p as for
 * mcs_filter_step.  *request_id identifies the request. */
mcs_status mcs_server_submit(mcs_server *srv, int32_t session_id, const float *scan_dev,
                             int32_t M, const float *noise_dev, const mcs_step_params *p,
                             int64_t *request_id);

/* Wait until every request submitted so far has completed. */
mcs_status mcs_server_drain(mcs_server *srv);

/* Times of a completed request (MCS_EBUSY while it is still pending). */
mcs_status mcs_server_times(mcs_server *srv, int64_t request_id, mcs_request_times *out);

/* Counters of the server so far. */
mcs_status mcs_server_stats_get(mcs_server *srv, mcs_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* MCSLAM_H */
