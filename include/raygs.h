/*
 * raygs.h -- C ABI of the MI355X (gfx950) ray-based Gaussian splatting
 * renderer.
 *
 * The method is that of "Hardware-Rasterized Ray-Based Gaussian Splatting"
 * (Rota Bulo et al., CVPR 2025):
 *   - a scene is a set of 3D Gaussians (centre, covariance R S^2 R^T, prior
 *     opacity, colour features) and an image is, per pixel ray x, the front to
 *     back composition of the rendered opacities (Sec. 3, eqs. 1-2);
 *   - the rendered opacity uses the ray-based divergence D_ray, the
 *     Mahalanobis distance of the point of maximum density along the ray
 *     (Sec. 3.2, eq. 5);
 *   - each Gaussian's screen support is bounded by the projection of the
 *     smallest enclosing 3D quad of Sec. 4.1 (eqs. 12-15, App. A.1-A.3), and
 *     D_ray is evaluated per pixel from the quad-local coordinate of the ray's
 *     hit on the quad plane, D = (c^-2 + |zeta|^-2)^-1 (Sec. 4.2, eq. 16);
 *   - optionally, the approximate MIP anti-aliasing of Sec. 5 (eq. 17).
 * The paper's fixed-function rasteriser and blender are replaced by compute
 * kernels: tile binning, a stable radix sort, and a persistent per-tile
 * compositing kernel.  Multi-view batching and the backward pass are
 * extensions; the paper has neither.
 *
 * Conventions shared by every entry point
 *   - Every pointer named "device" is memory on the context's GPU; the caller
 *     owns it (allocates, frees) and the library never keeps it past a call,
 *     except that a plan remembers the pointers it was captured with.
 *   - Gaussians are structure-of-arrays float32 planes of length n:
 *       means[3][n] (world), log_scales[3][n] (s = exp), quats[4][n] as
 *       (w, x, y, z) (normalised inside), opacity_logits[n] (o = sigmoid),
 *       sh[(d+1)^2][3][n] with d = sh_degree in 0..3, real spherical-harmonic
 *       coefficients indexed k = l^2 + l + m; colour = max(0, SH(dir) + 0.5)
 *       with dir the unit vector from the camera centre to the mean.
 *   - Cameras are pinhole, OpenCV axes (x right, y down, z forward), host
 *     memory, double precision: world_to_cam is row-major [R | t] (3x4); a
 *     pixel (x, y) is the ray through ((x + 1/2 - cx)/fx, (y + 1/2 - cy)/fy, 1).
 *   - Images are float32, planar: rgb[3][H][W]; final_T[H][W] is the
 *     transmittance left after compositing; n_contrib[H][W] (int32) is the
 *     number of entries of the pixel's tile list that compositing consumed:
 *     the whole list, or the entries before the one at which it stopped
 *     (the backward pass walks them back).
 *   - All work is queued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = the null stream) and is asynchronous unless stated.
 *   - Errors are returned as rgs_status codes, never by abort; the message
 *     of the last failure is available from rgs_last_error.  Degenerate
 *     Gaussians (non-finite values, zero quaternion, prior opacity below
 *     p_min, camera inside the support, centre at or before the near plane)
 *     are culled, not errors.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef RAYGS_H
#define RAYGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rgs_context rgs_context;
typedef struct rgs_plan rgs_plan;

typedef enum {
    RGS_OK = 0,
    RGS_EINVAL = -1,       /* invalid argument (null pointer, bad size or option) */
    RGS_EWORKSPACE = -2,   /* workspace smaller than rgs_workspace_size reports */
    RGS_EOVERFLOW = -3,    /* more Gaussian-tile instances than the workspace holds */
    RGS_EHIP = -4,         /* a HIP runtime call failed */
    RGS_ECAPTURE = -5,     /* HIP graph capture or instantiation failed */
    RGS_EUNSUPPORTED = -6  /* a valid request the library does not implement */
} rgs_status;

typedef struct {
    const float *means;          /* device [3][n] */
    const float *log_scales;     /* device [3][n] */
    const float *quats;          /* device [4][n], (w, x, y, z) */
    const float *opacity_logits; /* device [n] */
    const float *sh;             /* device [(sh_degree+1)^2][3][n] */
    int64_t n;                   /* >= 0; n * n_views < 2^28 */
    int32_t sh_degree;           /* 0..3 */
} rgs_gaussians;

typedef struct {
    double world_to_cam[12]; /* row-major [R | t], OpenCV axes */
    double fx, fy, cx, cy;   /* pixels; fx, fy > 0 */
    int32_t width, height;   /* 1..16384 */
} rgs_camera;

/* Divergences (rgs_options.divergence). */
#define RGS_DIVERGENCE_RAY 0
#define RGS_DIVERGENCE_GS 1

typedef struct {
    double p_min;          /* cut-off opacity of the support, eq. 3; in (0, 1); default 1/255 */
    double alpha_max;      /* opacity clamp, in (p_min, 1); default 0.99 */
    double t_eps;          /* compositing stops before T would fall below it; [0, 1); default 1e-4 */
    double near_z;         /* centres with z <= near_z are culled (Sec. 4.1, near plane); > 0; default 0.2 */
    int32_t mip;           /* 0 = none (default); 1 = approximate MIP of Sec. 5, eq. 17; 2 = exact MIP of
                              Sec. 5 / App. A.5: per ray, Sigma + sigma_x^2 tau(x)^2 I with sigma_x^2 the
                              pixel's area at unit distance along the ray, opacity times
                              sqrt(|Sigma| x.Sigma^-1 x / (|Sigma^_x| x.Sigma^_x^-1 x));
                              3 = the widening of eq. 17 without its opacity modulation (the dilation-only
                              ablation of Sec. 6.2); forward only */
    double mip_sigma2_px;  /* MIP pixel variance in px^2 at the principal point (Sec. 6 uses 0.1); >= 0 */
    double background[3];  /* added as T_final * background; default 0 */
    int32_t tile_w, tile_h;/* each 8, 16 or 32; 0, 0 = the shape rgs_autotune_training or rgs_autotune
                              last chose on this context for the same configuration class (render or
                              training step, MIP, Gaussian count in octaves, each view's pixel count in
                              half-octaves), training choices first, else 8x16; resolved at every call,
                              so query workspace sizes again after an autotune */
    int32_t divergence;    /* RGS_DIVERGENCE_RAY (default): D_ray of eq. 5; RGS_DIVERGENCE_GS: the
                              linearised D_gs of Sec. 3.1, (p - pi(mu))^T (J Sigma J^T)^-1 (p - pi(mu))
                              with J the projection's Jacobian at mu (no MIP; differentiable) */
} rgs_options;

typedef struct {
    float *rgb;          /* device [3][H][W] */
    float *final_T;      /* device [H][W] */
    int32_t *n_contrib;  /* device [H][W] */
} rgs_view_out;

typedef struct { /* device, same shapes as rgs_gaussians; gradients are ADDED (+=) */
    float *means, *log_scales, *quats, *opacity_logits, *sh;
} rgs_gaussian_grads;

/* Flags of a workspace. */
#define RGS_WS_BACKWARD 1 /* reserve the per-record gradients used by rgs_render_backward */

/* A caller-owned device workspace.  It holds all intermediate state of a frame
 * (per Gaussian-view raster records, depth keys and tile rectangles, sort
 * buffers, tile ranges) and, with RGS_WS_BACKWARD, the per-record gradients.
 * It needs no initialisation and must stay untouched between rgs_render and
 * the matching rgs_render_backward.  `capacity` is the number of
 * Gaussian-tile instances it can hold; `bytes` must be at least what
 * rgs_workspace_size reports for the same (capacity, flags). */
typedef struct {
    void *ptr;         /* device, 256-byte aligned */
    size_t bytes;
    int64_t capacity;  /* >= 1 */
    int32_t flags;     /* RGS_WS_* */
} rgs_workspace;

/* Create a context on HIP device `device` (queries its compute-unit count).
 * Returns RGS_EINVAL for a bad device or NULL out, RGS_EHIP on runtime
 * failure.  The context holds tuning state and timing events only. */
rgs_status rgs_create(int device, rgs_context **out);
void rgs_destroy(rgs_context *ctx);

/* Message describing the last error on this context ("" if none).  The string
 * is owned by the context and valid until the next call on it. */
const char *rgs_last_error(const rgs_context *ctx);

/* Bytes of device workspace needed to render `n_views` cameras of a scene of
 * n Gaussians with room for `capacity` Gaussian-tile instances.  Pure host
 * arithmetic; no GPU work; ctx may be NULL (no error message is kept then).
 * A capacity of about 8 n n_views instances covers typical scenes;
 * rgs_render_status reports the count a frame needed.  RGS_EINVAL when
 * n n_views >= 2^28 or the views hold 2^29 tiles or more in total. */
rgs_status rgs_workspace_size(rgs_context *ctx, int64_t n, const rgs_camera *cams, int32_t n_views,
                              const rgs_options *opts, int64_t capacity, int32_t flags, size_t *bytes);

/* Forward render of n_views cameras in one batch (Sec. 3 eqs. 1-2 with D_ray
 * of eq. 5, the quad bound of Sec. 4.1 and, with opts->mip = 1, eq. 17; with
 * opts->mip = 2 the exact MIP weight of Sec. 5 per pixel, binned by the quad
 * of a widened Gaussian that bounds its support, or by the whole view where
 * no such bound exists).  A quad with a vertex at z <= 0 is drawn unclipped;
 * its pixel box is that of the part of it inside the view frustum, and it is
 * culled when no part is inside.  Tiles are binned from the part of the
 * pixel box whose pixel centres lie in the support ellipse's bounding box
 * (no other pixel can hold support); a Gaussian-view with no such pixel is
 * culled.
 * cams, outs: host arrays of n_views (outs entries hold device pointers);
 * opts: one struct for the whole batch.  Stream-ordered, no host
 * synchronisation.  If the frame needs
 * more instances than ws->capacity, every view is rendered as background and
 * rgs_render_status reports RGS_EOVERFLOW with the count needed. */
rgs_status rgs_render(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                      const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): rgs_render without a workspace argument.
 * The frame's intermediate state lives in a scratch array the library holds
 * on each device (256 MiB, reserved when the first context on that device is
 * created and kept until the process ends); the call allocates nothing, on
 * the device or the host.  The frame is laid out in the scratch with the
 * largest instance capacity that fits.  A frame that does not fit with room
 * for a single instance (about 180 bytes per Gaussian-view plus a few MiB)
 * is rejected with RGS_EINVAL and a message giving both sizes.  tile_w =
 * tile_h = 0 means 8x16 here (the autotuned shapes are not consulted).
 * instances_needed (device, 8-byte aligned, may be NULL) receives, in stream
 * order, the Gaussian-tile instances the frame needed; when that exceeds the
 * capacity every view is rendered as background.  Every call on a device
 * shares that device's scratch, which keeps the last frame's contents: calls
 * that overlap in time on one device (other streams, other host threads)
 * race and give wrong images.  Not for HIP graph capture: the view table is
 * copied from host memory that the call does not keep.  No backward pass
 * reads this scratch (use rgs_render with an RGS_WS_BACKWARD workspace). */
rgs_status rgs_render_noalloc(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                              const rgs_options *opts, const rgs_view_out *outs, int64_t *instances_needed,
                              void *stream);

/* Synchronises `stream`, then reads the instance count of the last frame
 * rendered into `ws` (*instances, may be NULL).  Returns RGS_OK, or
 * RGS_EOVERFLOW when that count exceeded ws->capacity. */
rgs_status rgs_render_status(rgs_context *ctx, const rgs_workspace *ws, void *stream, int64_t *instances);

/* Gradients of a loss with respect to the Gaussian parameters, given
 * dL_drgb[v] (device [3][H][W] per view) for the frame last rendered into
 * `ws` (which must carry RGS_WS_BACKWARD) with the same g, cams, opts and
 * outs.  The context remembers, per workspace address, the tile shape, MIP
 * mode, divergence, Gaussian and view counts, capacity and flags of the last
 * frame rendered into it (by rgs_render or rgs_batch_launch): opts->tile_w =
 * tile_h = 0 takes that frame's tile shape (whatever the autotuners chose
 * since), and any of these that differs from that frame is RGS_EINVAL.
 * Walks each pixel's list back from n_contrib starting at final_T.
 * Gradients are added into `grads`.  With opts->mip = 1 they also flow
 * through the MIP widening and opacity modulation (eq. 17), with opts->mip
 * = 2 through the per-ray widening and modulation of the exact MIP; opts->mip
 * = 3 returns RGS_EUNSUPPORTED.  With RGS_DIVERGENCE_GS they flow through
 * pi(mu), the projection's Jacobian J(mu) and Sigma_pi = J Sigma J^T.
 * Uses float atomics: results are order-nondeterministic in the last bits. */
rgs_status rgs_render_backward(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                               const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs,
                               const float *const *dL_drgb, const rgs_gaussian_grads *grads, void *stream);

/* Batched persistent rendering with HIP graphs.  A plan fixes the view
 * count, resolutions, options, Gaussian count, SH degree and the workspace's
 * capacity and flags; the first rgs_batch_launch captures the whole frame
 * (all views, one persistent compositing launch) into one HIP graph and later
 * launches replay it, re-capturing if the Gaussian, workspace or output
 * pointers change.  Camera poses and intrinsics may change between launches
 * (image sizes may not).  rgs_batch_plan reports the workspace size. */
rgs_status rgs_batch_plan(rgs_context *ctx, int64_t n, int32_t sh_degree, const rgs_camera *cams, int32_t n_views,
                          const rgs_options *opts, int64_t capacity, int32_t flags, size_t *ws_bytes,
                          rgs_plan **out);
rgs_status rgs_batch_launch(rgs_plan *plan, const rgs_gaussians *g, const rgs_camera *cams, const rgs_workspace *ws,
                            const rgs_view_out *outs, void *stream);

/* Overflow check of a plan's last launch (eq. 1's compositing needs every
 * Gaussian-tile instance of the frame): synchronises the stream of that
 * launch, then writes the number of instances the frame needed to
 * *instances_needed (may be NULL).  RGS_OK when they fit the plan's capacity,
 * RGS_EOVERFLOW when they did not (the views were then rendered as
 * background: make a plan with a larger capacity); RGS_EINVAL before the
 * first launch. */
rgs_status rgs_batch_status(rgs_plan *plan, int64_t *instances_needed);
void rgs_plan_destroy(rgs_plan *plan);

/* Times every supported tile shape on this frame (hipEvent timing, `reps`
 * renders each after one warm-up, synchronising `stream`) and writes the
 * fastest into *best (a copy of *opts with tile_w, tile_h set) and its mean
 * milliseconds into *best_ms.  Shapes whose instances exceed ws->capacity, or
 * whose tile tables exceed the workspace, are skipped: a workspace sized for
 * 8x8 tiles (the most tiles and instances) lets every shape run. */
rgs_status rgs_autotune(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                        const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs, int32_t reps,
                        void *stream, rgs_options *best, double *best_ms);

/* As rgs_autotune for a training step: each timed step is a render followed
 * by rgs_render_backward with the upstream gradients dL_drgb[v] (device
 * [3][H][W] per view); `ws` must carry RGS_WS_BACKWARD and opts->mip be 0, 1 or 2.
 * Every backward pass adds into `grads`, so pass scratch buffers.  *best_ms
 * is the mean forward + backward milliseconds of the chosen shape. */
rgs_status rgs_autotune_training(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                                 const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs,
                                 const float *const *dL_drgb, const rgs_gaussian_grads *grads, int32_t reps,
                                 void *stream, rgs_options *best, double *best_ms);

/* Byte offsets of the intermediate buffers inside a workspace (for tests and
 * profiling tools).  Counts are element counts.  Pure host arithmetic; ctx
 * may be NULL. */
typedef struct {
    size_t counters;       /* int64[8]: [0] instances needed (tiles of all binning boxes), [1] capacity,
                              [2] tile rows of all binning boxes, [3] listed instances (sorted; the rest are
                              empty), [4] kept (not culled) Gaussian-views, [5] quads with a vertex at
                              z <= 0 (65536 of them, in no fixed order, have their box clipped to the
                              view frustum; any others keep the whole view) */
    size_t views;          /* per-view device table */
    size_t records;        /* float[16] per Gaussian-view (float[28] with mip = 2), index v * n + i */
    size_t depth_keys;     /* uint32 per Gaussian-view: the kept views' keys, sorted, in [0, counters[4]) */
    size_t boxes;          /* uint16[4] per Gaussian-view: pixel box x0, x1, y0, y1 (inclusive) */
    size_t bin_boxes;      /* uint16[4] per Gaussian-view: binning box, the pixels of the pixel box whose
                              centres lie in the support ellipse's bounding box (the whole pixel box when
                              the support is unbounded; tiles are listed from it) */
    size_t conics;         /* double[8] per Gaussian-view: support ellipse P00, P01, P11, h0, h1, f0, u0, v0 */
    size_t tile_counts;    /* uint32 per Gaussian-view: tiles of its binning box (0 = culled) */
    size_t order;          /* uint32 per Gaussian-view: the kept views' ids sorted by (depth key, id), in
                              [0, counters[4]) */
    size_t offsets;        /* uint32 per Gaussian-view: first instance of each sorted entry */
    size_t inst_tiles;     /* uint32 per instance: global tile id, sorted, [0, counters[3]) (binning box tiles
                              whose pixel-centre rectangle misses the support are dropped by the sort) */
    size_t inst_ids;       /* uint32 per instance: Gaussian-view id (low 28 bits) sorted by (tile, depth, id);
                              with tile shapes of at most 4 pixel slots of 64 pixels, the top 4 bits
                              flag the slots that the support reaches (0 with more slots) */
    size_t tile_ranges;    /* uint32[2] per global tile: [start, end) into the instance arrays */
    size_t record_grads;   /* float[16] per Gaussian-view (float[32] with mip = 2; RGS_WS_BACKWARD only, else 0) */
    size_t total_bytes;    /* what rgs_workspace_size reports */
    int64_t n_records;     /* n * n_views */
    int64_t capacity;      /* instances */
    int64_t total_tiles;   /* over all views */
    int32_t tile_w, tile_h;
    int32_t tile_bits;     /* sorted bits of a tile id: 2^tile_bits > total_tiles */
    int32_t reserved;
} rgs_workspace_layout;

rgs_status rgs_get_workspace_layout(rgs_context *ctx, int64_t n, const rgs_camera *cams, int32_t n_views,
                                    const rgs_options *opts, int64_t capacity, int32_t flags,
                                    rgs_workspace_layout *out);

/* Per-view completion clocks, for latency measurement of batched renders.
 * While `stamps` is non-null, every rgs_render on this context (not batch
 * plans or rgs_autotune) also writes, in stream order, stamps[0] = the
 * device wall clock when the frame starts and stamps[1 + v] = the wall clock
 * when the last compositing work item of view v finished; ticks are
 * 1 / rgs_wall_clock_hz seconds.  `stamps` is caller-owned device memory of
 * max_views + 1 uint64, 8-byte aligned, max_views in 1..256; a render with
 * more views fails with RGS_EINVAL.  Passing NULL turns the clocks off.  The
 * clocks add one store per work item and a small reduction kernel. */
rgs_status rgs_set_view_clocks(rgs_context *ctx, uint64_t *stamps, int32_t max_views);
double rgs_wall_clock_hz(rgs_context *ctx);

/* Per-stage GPU timing.  While enabled, rgs_render and rgs_render_backward
 * record HIP events around each stage on the caller's stream (graph replays
 * are not timed); rgs_stage_times synchronises, adds the elapsed times of all
 * frames recorded since the last read into ms[0..n) in the order of
 * rgs_stage_names (a ';'-separated list), sets *frames to the number of
 * forward renders timed since then, and resets.  Returns the number of
 * stages. */
rgs_status rgs_set_stage_timing(rgs_context *ctx, int32_t enable);
int32_t rgs_stage_times(rgs_context *ctx, double *ms, int32_t n, int64_t *frames);
const char *rgs_stage_names(void);

/* Box downsampling for anti-aliasing evaluation (Sec. 6.2 compares against
 * 4-ray multisampling): dst[p][y][x] = the mean of the factor x factor block
 * src[p][y factor + r][x factor + c], r, c < factor.  A view rendered with
 * its focal lengths, principal point and size multiplied by `factor` has
 * factor^2 rays per output pixel on an ordered grid, so this gives
 * multisampled (factor 2) or supersampled images.  src: device
 * [planes][height factor][width factor] floats; dst: device
 * [planes][height][width]; both caller-owned, not overlapping.  factor in
 * 1..16, width and height in 1..16384, planes in 1..4; RGS_EINVAL otherwise
 * or for NULL pointers.  Stream-ordered. */
rgs_status rgs_downsample_box(rgs_context *ctx, const float *src, int32_t width, int32_t height, int32_t factor,
                              int32_t planes, float *dst, void *stream);

/* Measured ceilings of this device, for roofline context beside the published
 * peaks: *fma_tflops = FP32 FMA rate of register-resident chains on every
 * compute unit (non-packed instructions, as every kernel here is built);
 * *exp_tops = rate of the hardware exp2 (tera-operations/s); *copy_gbs =
 * device-to-device copy bandwidth counting bytes read plus written.  Not for
 * use during a frame: it allocates (about 1 GiB, freed before returning) and
 * synchronises `stream`.  RGS_EINVAL for NULL outputs, RGS_EHIP on runtime
 * failure. */
rgs_status rgs_calibrate(rgs_context *ctx, void *stream, double *fma_tflops, double *exp_tops, double *copy_gbs);

#ifdef __cplusplus
}
#endif
#endif /* RAYGS_H */
