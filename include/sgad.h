/*
 * sgad.h - C ABI of the MI355X splatting library (libsgad.so).
 *
 * Differentiable splatting of pixel-aligned simplified Gaussians at adjusted
 * depth (SGAD-SLAM, arXiv 2603.21055): the renderer of Sec. 3.2,
 * (V'_k, D'_k) = splat(G_i, p_k) for views k in {i, NN(i)}, its adjoint for
 * the learnable attributes of Sec. 3.1 (colour, radius, opacity, depth
 * offset) and the view pose, the per-pixel depth-distribution Gauss-Newton
 * tracker (abstract; Sec. 3.3), the L1 terms of Eq. 1, Adam, and a BF16
 * 3x3 conv net that warm-starts the offsets.
 *
 * Conventions (fixed here because the paper does not give formulas):
 *  - Pixel (u, v) is evaluated at the integer point (u, v); a keyframe pixel
 *    back-projects along ((u-cx)/fx, (v-cy)/fy, 1) to z-depth |D + delta|.
 *  - Poses are world->camera, X_c = R X_w + t, R row-major.
 *  - The Gaussian covariance is r^2 I (r a world-space standard deviation);
 *    screen covariance r^2 J J^T + 0.3 I; a pixel takes a Gaussian iff
 *    q <= 9 and alpha = min(0.99, o exp(-q/2)) >= 1/255; contributors are
 *    composited front to back by (depth rounded to float, gid) with
 *    gid = kf_index * H * W + v * W + u, stopping before the transmittance
 *    would drop below 1e-4; Gaussians with z < 0.2 are culled.
 *  - Outputs: RGB = sum w c, depth D' = sum w z (not divided by alpha),
 *    alpha = 1 - T.
 *  - Pose gradients are with respect to a left twist xi = (rho, phi) on the
 *    view's world->camera pose, T <- Exp(xi) T.
 *
 * Memory: every data pointer is a device pointer owned by the caller unless
 * stated otherwise; planes are float32 row-major [H][W]; colour is planar
 * [3][H][W].  The library owns only its internal workspace.
 *
 * Streams: calls enqueue on the given hipStream_t (passed as void*; NULL is
 * the null stream) and return without waiting unless documented.
 *
 * Errors: every call returns an sgad_status; no exception crosses the ABI.
 * Conditions found on the device (non-finite inputs, instance-list overflow)
 * are latched in the context and returned by sgad_sync().
 */
#ifndef SGAD_H
#define SGAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGAD_OK = 0,
    SGAD_EINVAL = 1, /* bad argument: sizes <= 0, null required pointer, non-finite pose */
    SGAD_ERANGE = 2, /* a size above a documented limit, or the instance list overflowed */
    SGAD_EHIP = 3,   /* a HIP runtime call failed (message in sgad_last_error) */
    SGAD_ENOMEM = 4, /* device or pinned allocation failed */
    SGAD_EDATA = 5   /* non-finite depth / offset / radius seen by a kernel */
} sgad_status;

typedef struct sgad_ctx sgad_ctx;
typedef struct sgad_saved sgad_saved;
typedef struct sgad_graph sgad_graph;

/* Pinhole camera: image H x W, focal lengths and principal point in pixels. */
typedef struct {
    int32_t H, W;
    float fx, fy, cx, cy;
} sgad_cam;

/* World->camera pose: X_c = R X_w + t, R row-major. */
typedef struct {
    float R[9];
    float t[3];
} sgad_pose;

/* One keyframe's pixel-aligned Gaussians (Sec. 3.1-3.2): one per pixel. */
typedef struct {
    sgad_cam cam;
    sgad_pose T_cw;
    const float* depth;   /* observed depth D, [H][W] */
    const float* offset;  /* learnable depth offset delta, [H][W] */
    const float* radius;  /* world-space std r, [H][W] */
    const float* opacity; /* o, [H][W] */
    const float* rgb;     /* colour, [3][H][W]; may be NULL for tracking */
    const float* sigma;   /* per-pixel depth std (tracking only), else NULL */
} sgad_keyframe;

/* A render job: keyframes (bit f = keyframe f, f < 64) splatted into view. */
typedef struct {
    int32_t view;
    uint32_t kf_mask_lo, kf_mask_hi;
} sgad_job;

/* Per-keyframe gradient outputs, same layouts as the inputs; ACCUMULATED. */
typedef struct {
    float* d_rgb;     /* [3][H][W] */
    float* d_opacity; /* [H][W] */
    float* d_radius;  /* [H][W] */
    float* d_offset;  /* [H][W]; equals the gradient w.r.t. depth */
} sgad_kf_grads;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  *out receives ownership. */
sgad_status sgad_create(int device, sgad_ctx** out);
/* Destroy a context and free its workspace (waits for its device work). */
void sgad_destroy(sgad_ctx* ctx);
/* Message of the last failing call on this context (never NULL). */
const char* sgad_last_error(const sgad_ctx* ctx);
/* Wait for all work the context enqueued and return the first latched
 * device-side condition (SGAD_EDATA, SGAD_ERANGE) since the previous call,
 * clearing it. */
sgad_status sgad_sync(sgad_ctx* ctx);
/* Tile shape of the compositing kernels: (8,8) (one tile per wavefront,
 * per-pixel candidate masks), (16,8), (16,16) or (32,8) (one tile per
 * workgroup, full-list walk); (0,0), the default, uses the configuration
 * sgad_autotune measured for the workload, else (8,8).  Forward outputs do
 * not depend on the tile shape; gradients agree to rounding. */
sgad_status sgad_set_tile(sgad_ctx* ctx, int tile_w, int tile_h);
/* Tile shape used by the last forward (after autotuning). */
sgad_status sgad_get_tile(const sgad_ctx* ctx, int* tile_w, int* tile_h);
/* Kernel variant used with a tile of (8,8) set by sgad_set_tile:
 * fwd_chunks = 64-entry chunks the forward publishes at once (1, 2 or 4;
 * default 4), bwd_sub = entries per adjoint sub-chunk (16 or 32; default
 * 16).  Forward outputs do not depend on it; gradients agree to rounding
 * (the adjoint's sums are grouped differently).  SGAD_EINVAL for other
 * values. */
sgad_status sgad_set_tile_variant(sgad_ctx* ctx, int fwd_chunks, int bwd_sub);
/* Kernel variant of the last forward's 8x8 wave tiles (after autotuning):
 * *fwd_chunks = 64-entry chunks the forward publishes at once (1, 2 or 4),
 * *bwd_sub = entries per adjoint sub-chunk (16 or 32).  Meaningless for the
 * other tile shapes.  SGAD_EINVAL on a null pointer. */
sgad_status sgad_get_tile_variant(const sgad_ctx* ctx, int* fwd_chunks, int* bwd_sub);

/* Per-kernel timing (tracing): when enabled, every library kernel is
 * bracketed by hipEvents recorded on its launch stream.  Enabling or
 * disabling resets the accumulators. */
sgad_status sgad_timing_enable(sgad_ctx* ctx, int enable);
/* Restrict timing to the kernel called `name` (as in the report; NULL or ""
 * times every kernel).  Fewer events per call keep the host cost of timing
 * small.  The name is copied. */
sgad_status sgad_timing_only(sgad_ctx* ctx, const char* name);
/* Waits for the recorded events and writes one line per kernel name,
 * "<name> <launches> <total_ms>\n", into buf (capacity cap bytes, NUL
 * terminated); SGAD_ERANGE if it does not fit. */
sgad_status sgad_timing_report(sgad_ctx* ctx, char* buf, size_t cap);

/* ---------------------------------------------------------------- render */

/*
 * Forward splat (Sec. 3.2): for each job j, the Gaussians of the keyframes
 * in its mask are rendered into view jobs[j].view.
 *   kf[n_kf]               keyframes; all share H x W (1 <= n_kf <= 64)
 *   vcam[n_views], vpose[n_views]  views; all share H x W
 *   out_rgb   [n_jobs][3][Hv][Wv]  written
 *   out_depth [n_jobs][Hv][Wv]     written (unnormalised)
 *   out_alpha [n_jobs][Hv][Wv]     written
 *   out_count [n_jobs][Hv][Wv]     int32 contributor count, or NULL
 *   *saved    receives a handle to the sorted instance lists and per-pixel
 *             state needed by sgad_render_bwd; owned by the context until
 *             sgad_saved_release.  Input arrays must stay alive and unchanged
 *             until the backward has been enqueued.
 */
sgad_status sgad_render_fwd(sgad_ctx* ctx, int n_kf, const sgad_keyframe* kf,
                            int n_views, const sgad_cam* vcam, const sgad_pose* vpose,
                            int n_jobs, const sgad_job* jobs,
                            float* out_rgb, float* out_depth, float* out_alpha,
                            int32_t* out_count, sgad_saved** saved, void* stream);

/*
 * Adjoint of sgad_render_fwd (gradient of Eq. 1's rendered terms).
 *   g_rgb [n_jobs][3][Hv][Wv], g_depth, g_alpha [n_jobs][Hv][Wv]: upstream
 *     grads; g_depth / g_alpha may be NULL (treated as zero).
 *   grads[n_kf]: per-keyframe outputs, ACCUMULATED (+=); only keyframes whose
 *     bit is set in the learnable mask (lo | hi << 32) are written, the others
 *     stay fixed (Sec. 3.2: neighbours are not learnable).
 *   d_pose [n_jobs][6]: WRITTEN, (rho, phi) left-twist gradient of each job's
 *     view pose; may be NULL.
 * With 8x8 tiles the tiles' shares are first summed per keyframe Gaussian in
 * a 32-byte record of the saved slot's workspace (n_kf * H * W records) and
 * then added to grads by one more launch, which clears the records again.
 */
sgad_status sgad_render_bwd(sgad_ctx* ctx, sgad_saved* saved,
                            const float* g_rgb, const float* g_depth, const float* g_alpha,
                            const sgad_kf_grads* grads, float* d_pose,
                            uint32_t learn_lo, uint32_t learn_hi, void* stream);

/*
 * Device workspace (bytes) that sgad_render_fwd and sgad_render_bwd of this
 * workload hold in one saved slot: preprocessed records, tile tables, the
 * instance keys and contributor masks, per-pixel state, pose partials and
 * the adjoint's per-Gaussian gradient records.
 * instances: the instance count the key list is sized for (0: the size of a
 * first call, before the exact count is known; after it the library sizes
 * the list to 1.25x the count + 65536).  Computed for 8x8 tiles, the shape
 * with the most tiles, so it bounds every tile shape.  Pinned host staging
 * and the L1-loss scratch are not included.  Keyframe planes may be null.
 * SGAD_EINVAL for invalid sizes, jobs or a null `bytes`.
 */
sgad_status sgad_workspace_bytes(sgad_ctx* ctx, int n_kf, const sgad_keyframe* kf, int n_views,
                                 const sgad_cam* vcam, int n_jobs, const sgad_job* jobs, uint64_t instances,
                                 size_t* bytes);

/* Return a saved handle to the context. */
sgad_status sgad_saved_release(sgad_ctx* ctx, sgad_saved* saved);

/*
 * Graph capture of a sequence of library calls (e.g. one mapping iteration:
 * sgad_render_fwd, sgad_l1_loss, sgad_render_bwd, sgad_saved_release,
 * sgad_adam_step) so that it can be replayed with one launch per iteration.
 *
 * sgad_graph_begin waits for `stream` and the device, then records every
 * library call made from this thread until sgad_graph_end; the recorded calls
 * do not run at record time and ignore their stream argument.  A recorded
 * call must find its workspace already sized by an earlier eager call of the
 * same workload (else SGAD_EINVAL); sgad_sync, sgad_autotune, sgad_track_gn,
 * sgad_saved_instances and the timing calls return SGAD_EINVAL while a
 * capture is open.  Device pointers and the values of the call arguments are
 * frozen into the graph, except that each recorded sgad_adam_step advances
 * its step count by one per launch (the first launch uses the `step` given
 * at record time).  Kernels timed while sgad_timing_enable is on at record
 * time are timed on every launch.
 *
 * sgad_graph_end instantiates the graph (*out is owned by the caller; free it
 * with sgad_graph_destroy before sgad_destroy).  The saved slots it recorded
 * belong to the graph until it is destroyed and are never reused or resized:
 * if a replayed forward overflows its instance list, its outputs are NaN,
 * SGAD_ERANGE is latched, and the graph must be destroyed and captured
 * again.  sgad_graph_launch enqueues one replay on `stream` (plus the
 * read-back of the replayed forwards' status); sgad_graph_destroy waits for
 * the device.
 */
sgad_status sgad_graph_begin(sgad_ctx* ctx, void* stream);
sgad_status sgad_graph_end(sgad_ctx* ctx, sgad_graph** out);
sgad_status sgad_graph_launch(sgad_ctx* ctx, sgad_graph* graph, void* stream);
sgad_status sgad_graph_destroy(sgad_ctx* ctx, sgad_graph* graph);

/*
 * Debug export of job `job`'s sorted instance list (waits for the stream).
 * tile_ranges: host [n_tiles][2] (start, end) relative to the job; keys: host
 * [cap] of (float bits of z << 32 | gid); *n_keys and *n_tiles are written.
 */
sgad_status sgad_saved_instances(sgad_ctx* ctx, const sgad_saved* saved, int job,
                                 uint32_t* tile_ranges, uint64_t* keys, size_t cap,
                                 size_t* n_keys, int* n_tiles);

/*
 * Autotuner: times forward + adjoint of exactly this workload (the same
 * arguments as sgad_render_fwd) for every tile configuration, reps times
 * each after one warm-up, using internal scratch outputs and gradients (the
 * caller's buffers are not touched), and remembers the fastest for the
 * workload key (view H, W, Gaussians per keyframe, pairs, jobs, keyframes);
 * forwards with tile (0,0) then use it.  Waits for the stream.  The best
 * tile and its average ms per forward + adjoint are returned if non-NULL.
 */
sgad_status sgad_autotune(sgad_ctx* ctx, int n_kf, const sgad_keyframe* kf, int n_views,
                          const sgad_cam* vcam, const sgad_pose* vpose, int n_jobs,
                          const sgad_job* jobs, int reps, int* best_tw, int* best_th,
                          float* best_ms, void* stream);

/* ---------------------------------------------------------------- tracking */

#define SGAD_TRACK_GRAPH 1u /* capture the iteration loop in a hipGraph and replay it */

/*
 * Gauss-Newton tracking of a new frame against the previous frame's
 * per-pixel depth distributions (abstract; Sec. 3.3).
 *   geo: pixel-aligned geometry Gaussians (depth, offset, radius, opacity
 *     and the per-pixel depth std `sigma` are required; rgb is ignored).
 *   vcam: the new frame's camera; obs_depth [H][W]: its observed depth
 *     (<= 0 marks a missing value).
 *   pose: DEVICE double[12] (R row-major, t) world->camera pose of the new
 *     frame; read as the starting point and overwritten with the result.
 *   iters: fixed number of iterations (no early exit), 1..1000.
 *   trace: DEVICE double[iters][40] or NULL; record k holds H (upper
 *     triangle, 21), g (6), log-likelihood, valid-pixel count, the damping
 *     used (-1 when no step was taken) and the step dxi (6).
 * Per iteration: splat sigma^2 into the view (same rule as the renderer),
 * per pixel mu = D'/A, s^2 = S/A, valid iff A >= 0.9 and D_obs > 0,
 * r = (D_obs - mu)/s, J = dr/dxi with s fixed; H = sum J^T J, g = sum J^T r
 * summed in FP64; dxi = -H^-1 g by Cholesky (damping 1e-9 tr(H), x10 per
 * retry); pose <- Exp(dxi) pose.  With SGAD_TRACK_GRAPH the loop is captured
 * once per (shapes, pointers, iters) and replayed.
 */
sgad_status sgad_track_gn(sgad_ctx* ctx, const sgad_keyframe* geo, const sgad_cam* vcam,
                          const float* obs_depth, double* pose, int iters, double* trace,
                          uint32_t flags, void* stream);

/* ---------------------------------------------------------------- mapping */

/*
 * L1 terms of Eq. 1 for n_jobs rendered views:
 *   L_j = w_rgb * mean|rgb - t_rgb| + w_depth * sum_U |depth - t_depth| / |U|,
 *   U = [t_depth > 0] (valid-depth mask).  The supplement's weights are
 *   w_rgb = 0.8, w_depth = 1.0; the SSIM term is not part of this call.
 *   rgb, t_rgb, g_rgb [n_jobs][3][H][W]; depth, t_depth, g_depth [n_jobs][H][W]
 *   g_rgb, g_depth: WRITTEN with dL/d(rgb), dL/d(depth) (subgradient 0 at 0).
 *   loss: device double [n_jobs], WRITTEN.
 */
sgad_status sgad_l1_loss(sgad_ctx* ctx, int n_jobs, int H, int W,
                         const float* rgb, const float* depth, const float* t_rgb, const float* t_depth,
                         float w_rgb, float w_depth, float* g_rgb, float* g_depth, double* loss,
                         void* stream);

/*
 * The whole of Eq. 1 for n_jobs rendered views:
 *   L_j = w_rgb * mean|rgb - t_rgb| + w_ssim * L_S + w_depth * sum_U |depth - t_depth| / |U|,
 * the L1 terms as in sgad_l1_loss, and L_S = 1 - mean over the three colour
 * channels and all pixels of SSIM(t_rgb, rgb) with the SSIM reference's
 * statistics (11 x 11 Gaussian window of standard deviation 1.5, normalised,
 * 'same' correlation with zero padding; C1 = 0.01^2, C2 = 0.03^2).  The
 * supplement's weights are (w_rgb, w_ssim, w_depth) = (0.8, 0.2, 1.0).
 * Same layouts as sgad_l1_loss; g_rgb, g_depth and loss are WRITTEN.  The
 * SSIM statistics are evaluated in FP64.  Uses a context workspace of
 * about 36 bytes per pixel and job when w_ssim != 0 (the three derivative
 * maps per channel and one partial sum per 16 x 16 tile; grown by the first
 * call that needs more; SGAD_EHIP if that happens while calls are captured).
 * SGAD_EINVAL on null pointers, sizes < 1 or non-finite weights;
 * SGAD_ERANGE above 21845 jobs.
 */
sgad_status sgad_eq1_loss(sgad_ctx* ctx, int n_jobs, int H, int W,
                          const float* rgb, const float* depth, const float* t_rgb, const float* t_depth,
                          float w_rgb, float w_ssim, float w_depth, float* g_rgb, float* g_depth, double* loss,
                          void* stream);

/* ---------------------------------------------------------------- GICP */
/*
 * Tracking a depth frame against a set of geometry Gaussians with
 * Generalized ICP (Sec. 3.3, Eq. 2; the supplement's sampling ratio R and
 * neighbour count K_c; Tab. 11's point-to-surface correspondences and
 * "ellipse" scale normalisation).  A set is a caller-owned device buffer of
 * 12 * n doubles, SoA [12][n] = (x, y, z, c00, c01, c02, c11, c12, c22, nx,
 * ny, nz) for the n = sgad_gicp_set_size(H, W, R) pixels of the frame's
 * stride-R grid (row-major): the back-projected point in its camera's frame,
 * the normalised covariance C' = U diag(max(l0/l2, 1e-3), max(l1/l2, 1e-3),
 * 1) U^T of its K_c nearest points of the set (the point itself included,
 * ties by index) and the normal (eigenvector of the smallest eigenvalue).
 * Grid pixels without depth are all zero (z = 0) and take no part.
 * Poses are camera-to-target P = (R, t): device double[12], R row-major
 * then t; a source point a maps to X = R a + t.
 */
/* Points of the stride-`ratio` grid of an H x W frame; -1 on bad sizes. */
int32_t sgad_gicp_set_size(int H, int W, int ratio);
/* Build a set from a depth map [H][W] (metres; <= 0: no depth) with the
 * pinhole camera cam (cam->H, cam->W give the frame size).  K_c = k in
 * 1..32 (SGAD_ERANGE otherwise).  `set` is WRITTEN. */
sgad_status sgad_gicp_prepare(sgad_ctx* ctx, const float* depth, const sgad_cam* cam, int ratio, int k,
                              double* set, void* stream);
/* One linearisation of Eq. 2 at the device pose: each valid source point X
 * is matched among its K_c nearest target points within 0.1 m (Euclidean,
 * ties by index; none: no pair) to the one minimising (n_b . e)^2 +
 * 1e-3 |e|^2, e = X - b (first minimum in distance order); with M = (C_b +
 * R C_a R^T)^-1 and J = de/dxi = [-I | [X]x] for the left twist
 * xi = (rho, phi): out (device double[29]) = H = sum J^T M J (upper
 * triangle, row-major, 21), g = sum J^T M (b - X) (6), the cost sum
 * e^T M e and the pair count, WRITTEN.  corr (device int32[n_src], may be
 * NULL): the matched target index per source point, -1 for none.  Uses a
 * context workspace of 29 doubles per 8 source points (one wavefront per
 * point).  tgt_cam / tgt_ratio: the camera and stride the target set was
 * prepared with (SGAD_EINVAL unless they give n_tgt grid points): the
 * neighbour search scans windows of grid cells around the one X projects
 * to, growing until a distance bound proves that no point outside can be
 * among the K_c nearest or within 0.1 m. */
sgad_status sgad_gicp_linearise(sgad_ctx* ctx, const double* src, int n_src, const double* tgt, int n_tgt,
                                const sgad_cam* tgt_cam, int tgt_ratio, int k, const double* pose, double* out,
                                int32_t* corr, void* stream);
/* `iters` Gauss-Newton steps from the device pose (updated in place):
 * dxi = -H^-1 g by a damped Cholesky (1e-9 tr H, x10 per retry, FP64),
 * P <- Exp(dxi) P.  trace (device double[iters][48], may be NULL): per step
 * H (21), g (6), cost, pair count, damping (-1: no solve), dxi (6) and the
 * pose before the step (R 9, t 3). */
sgad_status sgad_gicp_track(sgad_ctx* ctx, const double* src, int n_src, const double* tgt, int n_tgt,
                            const sgad_cam* tgt_cam, int tgt_ratio, int k, double* pose, int iters, double* trace,
                            void* stream);

/*
 * The global set T of geometry Gaussians that frames are tracked against
 * (Sec. 3.3, matching a frame to the scene and updating T).  T holds world
 * Gaussians (point, normalised covariance, normal) in the layout of a GICP
 * set with row stride `capacity`: data = [12][capacity] doubles, the first
 * *count columns in use.  T keeps at most one Gaussian per cubic voxel of
 * side `voxel` (the voxel of p is floor(p / voxel) per axis), found through
 * an open-addressing hash: keys (int64[slots]) and vals (int32[slots]),
 * `slots` a power of two >= 2 * capacity.  All four arrays are caller-owned
 * device memory; the struct itself is read on the host.  voxel must be at
 * least D_MAX / 32 = 3.125 mm, and coordinates within +-(2^20 - 41) voxels:
 * Gaussians outside are not inserted and queries outside find nothing.
 */
typedef struct {
    double* data;    /* device [12][capacity] */
    int64_t* keys;   /* device [slots] */
    int32_t* vals;   /* device [slots] */
    int32_t* count;  /* device [1]: Gaussians in T */
    int32_t capacity;
    int32_t slots;
    double voxel;    /* metres */
} sgad_gmap;

/* Empty T (count 0, every slot free). */
sgad_status sgad_gmap_reset(sgad_ctx* ctx, const sgad_gmap* map, void* stream);
/* Add a tracked frame's set (as sgad_gicp_prepare builds it, n points) to T
 * under its camera-to-world pose (device double[12], R row-major then t):
 * each valid Gaussian is moved into the world (p = R a + t summed as ((r0
 * a0 + r1 a1) + r2 a2) + t; C = R C_a R^T; n = R n_a) and appended unless
 * its voxel already holds a Gaussian of T or of this frame with a lower
 * index; new Gaussians are appended in index order.  Once T is at capacity
 * further Gaussians are dropped.  Calls on one map are ordered by their
 * stream; overlapping calls on one map race. */
sgad_status sgad_gmap_insert(sgad_ctx* ctx, const sgad_gmap* map, const double* set, int n, const double* pose,
                             void* stream);
/* sgad_gicp_linearise / sgad_gicp_track with T as the target: the pose is
 * camera-to-world, corr holds indices into T, and the K_c nearest are found
 * by an exact search over voxel shells around X. */
sgad_status sgad_gicp_linearise_map(sgad_ctx* ctx, const double* src, int n_src, const sgad_gmap* map, int k,
                                    const double* pose, double* out, int32_t* corr, void* stream);
sgad_status sgad_gicp_track_map(sgad_ctx* ctx, const double* src, int n_src, const sgad_gmap* map, int k,
                                double* pose, int iters, double* trace, void* stream);
/*
 * Depth with its holes filled from a render (Sec. 3.2: Gaussians are
 * initialised where the depth map has no value from what the previous
 * keyframe renders there): out = depth where depth > 0, else D'/A where the
 * rendered alpha A >= alpha_min (D' the rendered depth, the sum of alpha
 * blended depths), else 0.  Device float[P] each, P = H * W; out may alias
 * depth.  SGAD_EINVAL on null pointers, P < 1 or alpha_min not in (0, 1].
 */
sgad_status sgad_fill_depth(sgad_ctx* ctx, int P, const float* depth, const float* rdepth, const float* ralpha,
                            float alpha_min, float* out, void* stream);

/* One parameter tensor for sgad_adam_step (all device pointers, n floats;
 * the pointers may be null when n is 0).  Arrays that start on a 16-byte
 * boundary are read and written four floats at a time. */
typedef struct {
    float* param;
    float* grad;
    float* m;
    float* v;
    int64_t n;
    float lr;
    float lo, hi;  /* the parameter is clamped to [lo, hi] after the step */
    int32_t space; /* SGAD_SPACE_*: the space Adam steps in */
} sgad_adam_group;

#define SGAD_SPACE_LINEAR 0 /* theta = p */
#define SGAD_SPACE_LOG 1    /* theta = log p (radius), dL/dtheta = p dL/dp */
#define SGAD_SPACE_LOGIT 2  /* theta = log(p / (1 - p)) (opacity), dL/dtheta = p (1 - p) dL/dp */

/*
 * Adam step (t = step >= 1) over up to 32 tensors in one launch.  The
 * parameter p is mapped to theta (per group `space`), g to dL/dtheta, then
 *   m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *   theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps),
 * and p = inverse map of theta, clamped to [lo, hi].  m and v hold the
 * moments of dL/dtheta.  Logit maps clamp p to [1e-6, 1 - 1e-6] first, log
 * maps to >= 1e-12.
 * The grads are zeroed afterwards when zero_grad != 0 (the backward
 * accumulates).  The supplement gives the learning rates (colour 0.0025,
 * radius 0.005, opacity 0.05, offset 0.01); they are the 3DGS values for
 * log-scale and logit-opacity parameters, so the driver steps radius in
 * SGAD_SPACE_LOG and opacity in SGAD_SPACE_LOGIT; Adam itself is this
 * library's reading of the unnamed optimiser.
 */
sgad_status sgad_adam_step(sgad_ctx* ctx, int n_groups, const sgad_adam_group* groups, int step,
                           float beta1, float beta2, float eps, int zero_grad, void* stream);

/* ---------------------------------------------------------------- conv net */
/*
 * Learned offset warm start (this library's addition; the paper starts the
 * offsets at zero, Sec. 3.2): delta0 = Net(R, G, B, h), six 3x3 'same'
 * convolutions 4 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 with ReLU after the first
 * five.  Activations are bf16 NHWC ([H][W][C]); weights [9][cout][cin]
 * (tap = 3 ky + kx, taps reading x[y + ky - 1][x + kx - 1]); products run on
 * BF16 MFMA with FP32 accumulation.  Supported layers: (cin, cout) = (4, 32),
 * (32, 32), (32, 1).  All pointers are device pointers; the bf16 activation
 * and weight pointers and the forward's output must be 16-byte aligned
 * (SGAD_EINVAL otherwise: the kernels move a pixel's channels in 16-byte loads).
 */
#define SGAD_CONV_RELU_BF16 0  /* y = relu(conv + bias), bf16 [H][W][cout] */
#define SGAD_CONV_LINEAR_F32 1 /* y = conv + bias, f32 [H][W] (cout == 1) */

/* bf16 copy of FP32 weights [9][cout][cin] and, if wt_bf16 is non-NULL, the
 * transposed tap-flipped copy wt[8 - t][ci][co] the input gradient uses. */
sgad_status sgad_conv_weights(sgad_ctx* ctx, int cin, int cout, const float* w, uint16_t* w_bf16,
                              uint16_t* wt_bf16, void* stream);
/* Forward of one layer (mode SGAD_CONV_*); y is written. */
sgad_status sgad_conv3x3_fwd(sgad_ctx* ctx, int H, int W, int cin, int cout, int mode, const uint16_t* x,
                             const uint16_t* w_bf16, const float* bias, void* y, void* stream);
/* Input gradient of a layer whose input passed a ReLU: dx = (conv^T dy) * [mask > 0],
 * dy bf16 [H][W][cout] (gradient of the layer's pre-activation), mask = the
 * layer's input activations bf16 [H][W][cin], dx bf16 [H][W][cin] written
 * (the gradient of the previous layer's pre-activation). */
sgad_status sgad_conv3x3_dgrad(sgad_ctx* ctx, int H, int W, int cin, int cout, const uint16_t* dy,
                               const uint16_t* wt_bf16, const uint16_t* mask, uint16_t* dx, void* stream);
/* Weight and bias gradients, ACCUMULATED into FP32 dw [9][cout][cin], db [cout].
 * Partial sums go through a context-owned device workspace (one row per
 * workgroup, up to 512 x (9 cout cin + cout) floats, grown by the first call
 * that needs more; SGAD_EHIP if that happens while calls are captured):
 * wgrad calls of one context that overlap on different streams race on it. */
sgad_status sgad_conv3x3_wgrad(sgad_ctx* ctx, int H, int W, int cin, int cout, const uint16_t* x,
                               const uint16_t* dy, float* dw, float* db, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * weight and bias gradients as sgad_conv3x3_wgrad (ACCUMULATED into dw, db),
 * with the partial-sum rows taken from a static device array of the library
 * (512 rows x (9 * 32 * 32 + 32) floats = 18.9 MB per device, resident on
 * every device the library runs on until the process ends) instead of the
 * context's growable workspace.  Allocates nothing and issues no memset: each
 * workgroup writes its whole row before the rows are summed.  SGAD_ERANGE if
 * the layer's rows would not fit (not reachable for the supported layers),
 * SGAD_EINVAL as sgad_conv3x3_wgrad.  All calls on one device share the
 * array: calls that overlap on one device (any context, any stream) race. */
sgad_status sgad_conv3x3_wgrad_noalloc(sgad_ctx* ctx, int H, int W, int cin, int cout, const uint16_t* x,
                                       const uint16_t* dy, float* dw, float* db, void* stream);
/* Network input (R, G, B, h) as bf16 [H][W][4] from planar rgb [3][H][W] and depth [H][W]:
 * h = (D - mean of D over the 3x3 neighbourhood inside the image) / 0.02 m. */
sgad_status sgad_net_input(sgad_ctx* ctx, int H, int W, const float* rgb, const float* depth, uint16_t* x0,
                           void* stream);
/* Training loss mean |pred - target| over n values (device double, written)
 * and its gradient as bf16 (n values, written). */
sgad_status sgad_offset_l1(sgad_ctx* ctx, int n, const float* pred, const float* target, uint16_t* grad,
                           double* loss, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SGAD_H */
