/*
 * gs3.h - C ABI of the MI355X (gfx950) low-resolution 3DGS rasterizer with
 * analytic screen-space image gradients.
 *
 * The rasterizer renders the low-resolution frame that feeds gradient-aware
 * super sampling and frame interpolation in 3DGS^3: RGB (Sec. 3, Eq. 2),
 * alpha, depth (the depth map consumed in Sec. 4.1 and 4.2) and the image
 * gradients dI/dx, dI/dy (Sec. 3, Eq. 3 and Eq. 4), from a set of 3D
 * Gaussians (Sec. 3, Eq. 1, Sigma = R S S^T R^T) projected by EWA splatting
 * and depth-sorted per 16x16 screen tile.
 *
 * Conventions (not stated by the paper; fixed here):
 *   - camera: p_cam = R_wc p_world + t, OpenCV axes (x right, y down,
 *     z forward); pinhole u = fx x/z + cx, v = fy y/z + cy; pixel (i, j) has
 *     its centre at (i + 0.5, j + 0.5);
 *   - quaternions are (w, x, y, z), not necessarily unit; scale =
 *     exp(log_scale); opacity = sigmoid(logit); colour = max(SH(d) + 0.5, 0)
 *     with d the unit vector from the camera centre to the Gaussian mean,
 *     real SH with the Condon-Shortley phase, m = -l..l within a degree;
 *   - culls: z < near_z; |x/z| > 1.3 (W/2)/fx or |y/z| > 1.3 (H/2)/fy;
 *     a 2D covariance (after adding `dilation` to its diagonal) with
 *     determinant <= 0; radius = ceil(3 sqrt(lambda_max));
 *   - compositing: alpha = min(o exp(-q/2), 0.99); alpha < 1/255 is
 *     skipped; a Gaussian whose blend would leave transmittance below 1e-4
 *     ends the pixel without being blended (all three constants are the
 *     float32 values nearest these numbers);
 *   - ties between equal float32 view depths are broken by Gaussian index.
 *
 * Memory: every pointer in these structs and calls is a DEVICE pointer owned
 * by the caller, unless marked otherwise.  Arrays are float32, contiguous,
 * row major.  Calls are asynchronous on the given HIP stream (a hipStream_t
 * passed as void*; NULL is the default stream) unless stated otherwise.
 *
 * Errors: every call returns GS_OK (0) or a negative GS_ERR_* code; nothing
 * throws across the ABI.  gs_last_error() returns a thread-local message for
 * the last failing call on the calling thread.  Errors raised by kernels
 * themselves (key capacity exceeded) are written to the workspace and read
 * by gs_forward_status() after the stream has been synchronised.
 */
#ifndef GS3_H
#define GS3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_OK 0
#define GS_ERR_INVALID_ARG (-1)
#define GS_ERR_OOM (-2)
#define GS_ERR_TOO_LARGE (-3)   /* request larger than the whole memory budget */
#define GS_ERR_AGAIN (-4)       /* server queue full; retry later */
#define GS_ERR_NOT_READY (-5)   /* poll: request still in flight */
#define GS_ERR_HIP (-6)         /* HIP runtime error; message has the hipError_t text */
#define GS_ERR_CAPACITY (-7)    /* the frame produced more keys than the workspace holds */
#define GS_ERR_NOT_FOUND (-8)   /* unknown ticket or scene id */

#define GS_TILE 16
#define GS_MAX_SH_DEGREE 3
#define GS_MAX_BATCH 64

/* Gaussian set (Sec. 3, Eq. 1): n Gaussians, structure of arrays.
 *   means [n,3], log_scales [n,3], quats [n,4] as (w,x,y,z),
 *   opacity_logits [n], sh [n,(sh_degree+1)^2,3] coefficient-major. */
typedef struct gs_scene {
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opacity_logits;
    const float* sh;
    int64_t n;
    int32_t sh_degree;          /* 0..3 */
    int32_t reserved;
} gs_scene;

/* Pinhole camera.  Host memory (passed by value inside the calls). */
typedef struct gs_camera {
    double R_wc[9];             /* world -> camera rotation, row major */
    double t[3];
    double fx, fy, cx, cy;
    int32_t width, height;      /* raster size in pixels, 1..4096 each */
} gs_camera;

/* Tile overlap of a Gaussian (which tiles' lists it joins).
 * GS_OVERLAP_SQUARE: the tiles of the square of half-width ceil(3 sqrt(lambda_max))
 *   around the 2D mean (3DGS^3 Sec. 3 builds on this rasterizer); the default,
 *   and the one the keys of gs_sorted_keys are defined by.
 * GS_OVERLAP_OPACITY: that square intersected with the bounding box of the
 *   ellipse where o exp(-q/2) >= 1/255 (enlarged by margins far above float
 *   rounding; ill-conditioned conics keep the square).  Only (Gaussian, tile)
 *   pairs whose alpha stays below 1/255 at every pixel centre of the tile are
 *   dropped, so rgb, alpha, depth, dcdx, dcdy and final_T are bit-identical to
 *   GS_OVERLAP_SQUARE; n_contrib counts list positions of the shorter lists.
 * GS_OVERLAP_ELLIPSE: of GS_OVERLAP_OPACITY's tiles, those whose pixel
 *   centres the ellipse can reach, row by row: for each tile row the span of
 *   columns that the ellipse's chords over the row's pixel-centre band cover
 *   (FP64, from the record's float32 conic and opacity, with the same
 *   margins).  Same guarantee: only pairs below 1/255 over the whole tile are
 *   dropped, so the image buffers are bit-identical to GS_OVERLAP_SQUARE. */
#define GS_OVERLAP_SQUARE 0
#define GS_OVERLAP_OPACITY 1
#define GS_OVERLAP_ELLIPSE 2

typedef struct gs_render_opts {
    float bg[3];                /* background colour added as T_final * bg */
    int32_t overlap;            /* GS_OVERLAP_SQUARE (0, default), _OPACITY or _ELLIPSE */
    double near_z;              /* default 0.2 */
    double dilation;            /* default 0.3, added to the 2D covariance diagonal */
} gs_render_opts;

/* Per-pixel outputs, planar float32 unless noted: rgb [3,H,W], alpha [H,W],
 * depth [H,W] (alpha-blended view z, not normalised), dcdx and dcdy [3,H,W]
 * (Eq. 3, per low-resolution pixel, including bg * dT), final_T [H,W] and
 * n_contrib [H,W] uint32 (1-based list position of the last blended
 * Gaussian).  final_T and n_contrib are the saved state of the backward pass
 * and must be non-NULL; the others may be NULL to skip the write.
 * n_evaluated and n_blended [H,W] uint32 are optional instrumentation: the
 * number of (Gaussian, pixel) pairs whose alpha the pixel evaluated (up to
 * and including the one that ended it) and the number it blended; when
 * either is non-NULL a counting variant of the compositing kernel runs.
 * normal [3,H,W] and nv [H,W] are the optional normal map N and normal-view
 * map Nv (3DGS^3 Sec. 4.1 and 4.2 take them as inputs; Sec. 5.1 renders them
 * the RaDe-GS way): each Gaussian's normal is the direction of its shortest
 * axis (the column of R(q) with the smallest log-scale, the first on ties),
 * in camera axes and flipped to face the camera (n . p_cam <= 0, p_cam the
 * view-space mean), computed in FP64 in one fixed order and stored as
 * float32; N = sum of n alpha T over the blended Gaussians (the weights of
 * the colour; the background adds nothing), and Nv = -N . r / |r| with
 * r = ((i + 0.5 - cx)/fx, (j + 0.5 - cy)/fy, 1) the pixel's ray.  When any
 * frame of a batch asks for either, projection also writes the per-Gaussian
 * normals to the workspace (layout.normals) and a normal-blending variant of
 * the compositing kernel runs; the other outputs are unchanged by it. */
typedef struct gs_outputs {
    float* rgb;
    float* alpha;
    float* depth;
    float* dcdx;
    float* dcdy;
    float* final_T;
    uint32_t* n_contrib;
    uint32_t* n_evaluated;
    uint32_t* n_blended;
    float* normal;
    float* nv;
} gs_outputs;

/* Parameter gradients, same shapes as gs_scene.  overwrite = 0: accumulated
 * (+=), the caller zeroes them; overwrite = 1: written (=), every Gaussian's
 * gradients including zeros for those that reach no tile, so the arrays may
 * hold anything on entry.  quats is 16-byte aligned, and so is sh when
 * 3 (degree + 1)^2 is a multiple of 4 (the scene's own alignment rules). */
typedef struct gs_grads {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
    int32_t overwrite;
    int32_t reserved;
} gs_grads;

/* One frame of a batch. */
typedef struct gs_job {
    gs_scene scene;
    gs_camera cam;
    gs_render_opts opts;
    gs_outputs out;
} gs_job;

/* Byte offsets (from the workspace base) of the intermediate buffers the
 * forward pass leaves in a workspace.  Indices of Gaussians are "flat": job j's
 * Gaussian g has flat index gauss_base[j] + g; tile t of job j has global
 * tile id tile_base[j] + t. */
typedef struct gs_ws_layout {
    size_t total_bytes;
    int64_t n_flat;             /* padded total of Gaussians over the batch */
    int64_t n_tiles;            /* total tiles over the batch */
    int64_t key_capacity;
    size_t records;             /* n_flat x 48 B {double u, v; float A, B, C, o, r, g, b, z} */
    size_t depth_keys;          /* n_flat x uint32 float32 bits of view z (0xFFFFFFFF: culled) */
    size_t rects;               /* n_flat x uint32 tile rectangle, bytes (tx0, ty0, tx1, ty1) low to high;
                                   0x000000FF when the Gaussian covers no tile */
    size_t touched;             /* n_flat x uint32 tiles covered */
    size_t depth_order;         /* n_flat x uint32 flat indices sorted by (z key, index) */
    size_t depth_rects;         /* n_flat x uint32 the packed rectangles in depth order */
    size_t chunk_counts;        /* tile counts of 256- and 4096-position chunks of the depth order (uint32),
                                   once per tile band when the batch is cut into bands */
    size_t tile_keys;           /* key_capacity x uint32 scratch: the sorted global tile ids when the tile
                                   sort takes two passes (over 2048 tiles in more than 64 bands, or with
                                   the ellipse overlap) */
    size_t tile_values;         /* key_capacity x uint32 flat Gaussian indices, sorted */
    size_t ranges;              /* n_tiles x 2 x uint32 [start, end) into the sorted arrays */
    size_t counters;            /* uint32[144]: key count, capacity-exceeded flag, the serving
                                   compositing queue's head (word 2), tiles composited per frame
                                   (words 16..79, serving only), the pair count of each tile band
                                   (from word 80) */
    size_t grads2d;             /* n_flat x 10 float backward scratch (when sized for it) */
    size_t normals;             /* n_flat x float4 (nx, ny, nz, 0) camera-facing normals when a frame
                                   of the batch asks for normal or nv outputs, else 0 */
    int64_t gauss_base[GS_MAX_BATCH];
    int64_t tile_base[GS_MAX_BATCH];
} gs_ws_layout;

/* Workspace size for a batch of n_jobs frames whose tile lists hold at most
 * key_capacity (tile, Gaussian) pairs in total; with_backward also reserves
 * the backward scratch.  Host-only call.  Returns GS_ERR_INVALID_ARG for
 * n_jobs outside 1..GS_MAX_BATCH or invalid scene / camera fields. */
int gs_forward_layout(const gs_job* jobs, int n_jobs, int64_t key_capacity,
                      int with_backward, gs_ws_layout* layout);

/* Number of (tile, Gaussian) pairs each frame of the batch produces: runs
 * the projection on the stream and synchronises it, then writes
 * keys_per_job[j] (host memory).  Lets a caller size key_capacity exactly.
 * `workspace` must hold gs_forward_layout(jobs, n_jobs, 0, 0).total_bytes. */
int gs_count_keys(const gs_job* jobs, int n_jobs, void* workspace, size_t ws_bytes,
                  int64_t* keys_per_job, void* stream);

/* Forward pass over a batch (3DGS^3 Sec. 3: EWA projection and SH colour,
 * tile binning and depth sort, front-to-back compositing with Eq. 2-4 in the
 * same pass).  Writes every job's outputs; leaves the intermediates described
 * by gs_ws_layout in `workspace` (device memory of at least
 * layout.total_bytes, 256-byte aligned).  Never synchronises the stream.  If
 * the frame needs more than key_capacity pairs, the extra pairs are dropped,
 * the outputs are invalid and gs_forward_status() reports GS_ERR_CAPACITY. */
int gs_render_forward_batch(const gs_job* jobs, int n_jobs, void* workspace, size_t ws_bytes,
                            int64_t key_capacity, void* stream);

/* gs_render_forward_batch for callers that cannot size key_capacity in
 * advance (a training loop whose Gaussians move every step): launches the
 * whole pass, then blocks the calling thread until the projection, depth
 * sort and pair count are done (not the whole pass: emission, tile sort and
 * compositing go on on the device) and reads the pair total (*keys_needed,
 * host memory, may be NULL).  GS_OK: the pairs fit key_capacity and the
 * outputs, once the stream reaches them, are the frame.  GS_ERR_CAPACITY:
 * the pairs did not fit, the extra pairs were dropped and the outputs are
 * invalid; the caller grows the workspace to *keys_needed and calls again
 * (in stream order the new call's outputs replace them).  with_backward:
 * the workspace was sized with with_backward = 1 (only its size is
 * checked).  Unlike gs_count_keys it projects once and copies four bytes.
 * Uses a pinned word and an event per host thread and device, created on
 * the first call. */
int gs_render_forward_checked(const gs_job* jobs, int n_jobs, void* workspace, size_t ws_bytes,
                              int64_t key_capacity, int with_backward, int64_t* keys_needed, void* stream);

/* gs_render_forward_batch for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc): no workspace argument and no allocation; the pass runs in a
 * file-scope device array of the library, 384 MiB on each GPU the library
 * runs on, held until the process ends (a 1M-Gaussian 960x540 frame with its
 * 10.8M pairs needs 264 MiB).  A batch whose workspace
 * (gs_forward_layout(jobs, n_jobs, key_capacity, 0).total_bytes plus the
 * sort scratch) exceeds it returns GS_ERR_TOO_LARGE before any launch.
 * counts_out (device, 2 x uint32, may be NULL) receives the pair count and
 * the capacity-exceeded flag (nonzero: pairs were dropped and the outputs are
 * invalid).  Every call on one GPU shares that GPU's array, and the array
 * keeps the last call's contents: calls that overlap on one GPU (on
 * different streams, or from different threads) race and corrupt each
 * other's frames; the intermediates of gs_ws_layout are not exposed. */
int gs_render_forward_noalloc(const gs_job* jobs, int n_jobs, int64_t key_capacity, uint32_t* counts_out,
                              void* stream);

/* Single-frame form of gs_render_forward_batch. */
int gs_render_forward(const gs_scene* scene, const gs_camera* cam, const gs_render_opts* opts,
                      const gs_outputs* out, void* workspace, size_t ws_bytes,
                      int64_t key_capacity, void* stream);

/* Reads the counters of a workspace after the forward's stream has been
 * synchronised: GS_OK, or GS_ERR_CAPACITY with *keys_needed the pair count the
 * frame asked for.  keys_needed may be NULL.  Blocking host call. */
int gs_forward_status(const void* workspace, const gs_ws_layout* layout, int64_t* keys_needed);

/* Sorted 64-bit keys of job `job`: key[i] = (tile << 32) | float32_bits(z),
 * with `tile` local to the job, and the matching local Gaussian indices,
 * for the job's pairs in sorted order (its tiles' ranges are contiguous).
 * keys_out [count] uint64 and values_out [count] uint32 are device buffers
 * of at least the job's key count (gs_count_keys).  Inspection entry point. */
int gs_sorted_keys(const gs_job* jobs, int n_jobs, int job, const void* workspace,
                   const gs_ws_layout* layout, uint64_t* keys_out, uint32_t* values_out,
                   void* stream);

/* Backward (adjoint) pass of one frame, after gs_render_forward on the same
 * workspace (sized with with_backward = 1) and the same outputs.  Per-tile
 * transmittance is recomputed in reverse from final_T and n_contrib rather
 * than stored.  dL_drgb [3,H,W] is required; dL_dalpha [H,W] and
 * dL_ddepth [H,W] may be NULL.  Gradients through dcdx / dcdy are not formed.
 * Accumulates into `grads` (+=), or writes them when grads->overwrite is set.
 * Float atomics make the low bits of the
 * result depend on scheduling.  Returns GS_ERR_INVALID_ARG for null or
 * misaligned gradient arrays or a workspace too small, before any launch. */
int gs_render_backward(const gs_scene* scene, const gs_camera* cam, const gs_render_opts* opts,
                       const gs_outputs* fwd_out, void* workspace, size_t ws_bytes,
                       int64_t key_capacity, const float* dL_drgb, const float* dL_dalpha,
                       const float* dL_ddepth, const gs_grads* grads, void* stream);

/* Gradient-aware interpolation (3DGS^3 Sec. 4.1, Eq. 5-7): the
 * low-resolution image and its image gradients (the rgb, dcdx and dcdy
 * outputs of a forward pass) to an image of scale x scale times the pixels.
 * Each low-resolution pixel's scale x scale block is M times the 27 values,
 * x-derivatives and y-derivatives at the 3x3 pixel centres around it, M being
 * the least-squares fit of the polynomials of total degree <= 5 to those 27
 * conditions evaluated at the block's pixel centres (offsets
 * ((k + 0.5)/scale - 0.5, (l + 0.5)/scale - 0.5) in low-resolution pixels);
 * neighbours outside the image repeat the edge pixel.  Every polynomial of
 * total degree <= 5 sampled with its exact derivatives is reproduced.
 *   rgb, dcdx, dcdy  device, planar float32 [3, height, width]
 *   out              device, planar float32 [3, height*scale, width*scale]
 *   width, height    1..4096; scale 1..4
 * Asynchronous on `stream`.  Returns GS_ERR_INVALID_ARG for null pointers or
 * sizes out of range, GS_ERR_HIP when the launch fails. */
int gs_gradient_upsample(const float* rgb, const float* dcdx, const float* dcdy, int32_t width,
                         int32_t height, int32_t scale, float* out, void* stream);

/* Pose-derived motion vectors and forward warping (3DGS^3 Sec. 4.2, Eq. 12
 * and Eq. 13) of one rendered frame (camera `src`, raster src->width x
 * src->height = W x H) to another camera `dst` (raster W' x H').
 *
 * Motion (Eq. 12): a source pixel (i, j) has geometry where alpha >=
 * float32(1/255); its centre (i + 0.5, j + 0.5) is un-projected at the
 * surface depth z = depth / alpha and projected into `dst`, giving (u', v')
 * and the destination view z'; V = (u' - i - 0.5, v' - j - 0.5), 0 where
 * there is no geometry.  These values are FP64 in one fixed order of
 * correctly rounded operations (no contraction):
 *   Xc  = (((u - cx)/fx) z, ((v - cy)/fy) z, z)
 *   Xw_i = (R0i (Xc0 - t0) + R1i (Xc1 - t1)) + R2i (Xc2 - t2)
 *   Xd_i = ((R'i0 Xw0 + R'i1 Xw1) + R'i2 Xw2) + t'_i,  z' = Xd2
 *   u' = fx' (Xd0 / z') + cx',  v' = fy' (Xd1 / z') + cy'
 * (R, t: world -> camera of the source; primed: of the destination).
 * Warping (Eq. 13, read as a forward splat): a source pixel with geometry
 * and z' >= 0.2 lands on destination pixel (floor(u'), floor(v')) if that
 * is inside the raster; of the pixels landing on one destination pixel the
 * smallest float32(z') wins, ties to the smaller source index j*W + i.  The
 * winner's colour is copied, depth is float32(z'), and its image gradient is
 * mapped by the chain rule, (dC/dx', dC/dy') = (I + dV/dx)^-T (dC/dx, dC/dy),
 * with dV/dx by central differences over source pixels with geometry
 * (one-sided where one neighbour is outside the raster or has no geometry,
 * zero where both are; gradients 0 where det(I + dV/dx) = 0).  Destination
 * pixels nobody lands on are holes: all outputs 0, weight 0, source -1.
 *
 *   rgb, dcdx, dcdy  device, planar float32 [3, H, W] (the forward's outputs);
 *                    rgb may be NULL when out->rgb is, dcdx and dcdy when
 *                    out->dcdx and out->dcdy both are
 *   normal           device, planar float32 [3, H, W], the normal map in the
 *                    source camera's axes (the forward's normal output), or
 *                    NULL when out->normal is NULL.  The winner's normal is
 *                    re-expressed in the destination camera's axes,
 *                    n' = R' R^T n: w_i = (R0i n0 + R1i n1) + R2i n2, then
 *                    n'_i = (R'i0 w0 + R'i1 w1) + R'i2 w2 in FP64
 *   alpha, depth     device, float32 [H, W], required
 *   motion           device, float32 [2, H, W] (Vx plane, Vy plane), or NULL
 *   out              host struct of device planes on the W' x H' raster; a
 *                    NULL plane is not written (see gs_warp_outputs)
 *   workspace        device, 16-byte aligned, at least gs_warp_workspace_size
 *                    bytes (8 B per destination pixel for the depth test's
 *                    z-buffer, 16 B per source pixel for the FP64 motion
 *                    vectors); contents on entry do not matter
 * Asynchronous on `stream`; the outputs must not overlap the inputs.
 * Returns GS_ERR_INVALID_ARG for null required pointers, rasters outside
 * 1..4096, non-finite or non-positive intrinsics, non-finite poses or a short
 * workspace; GS_ERR_HIP when a launch fails. */
typedef struct gs_warp_outputs {
    float* rgb;                 /* [3, H', W'] */
    float* depth;               /* [H', W'] destination view z of the winner */
    float* dcdx;                /* [3, H', W'] */
    float* dcdy;                /* [3, H', W'] */
    float* weight;              /* [H', W'] 1 where a source pixel landed, else 0 */
    int32_t* source;            /* [H', W'] winning source index j*W + i, -1 for holes */
    float* normal;              /* [3, H', W'] warped normal map (needs the normal input) */
} gs_warp_outputs;

int gs_warp_workspace_size(const gs_camera* src, const gs_camera* dst, size_t* bytes);
int gs_motion_warp(const gs_camera* src, const gs_camera* dst, const float* rgb, const float* alpha,
                   const float* depth, const float* dcdx, const float* dcdy, const float* normal, float* motion,
                   const gs_warp_outputs* out, void* workspace, size_t ws_bytes, void* stream);

/* Stage instrumentation.  Between gs_profile_start and gs_profile_stop every
 * `every`-th forward pass (the 1st, the every+1-th, ...) records HIP events
 * on its own stream at its stage boundaries (at most max_frames passes are
 * recorded; each event costs the stream a few microseconds, so sampling
 * keeps the instrumentation out of a throughput measurement).
 * gs_profile_stop waits for those events and writes the summed milliseconds
 * of each stage to stage_ms (host memory, GS_N_STAGES entries) and the number
 * of recorded passes to *frames.  Stages: 0 projection, 1 depth sort, 2 key
 * offsets + pair emission, 3 tile sort + tile ranges, 4 compositing.
 * max_frames 1..10^6, every 1..10^6. */
#define GS_N_STAGES 5
int gs_profile_start(int max_frames, int every);
int gs_profile_stop(double* stage_ms, int64_t* frames);

/* ---------------------------------------------------------------- serving
 * A server keeps scenes resident in device memory and renders requests
 * (scene, camera, options) in continuous batches: requests that arrive while
 * others are on the GPU are admitted as soon as a batch slot and enough of
 * the memory budget are free, and run in the next launch beside requests of
 * other scenes and resolutions (one gs_render_forward_batch per batch, so a
 * single grid covers every frame of the batch); up to n_streams batches are
 * in flight at once and overlap on the device.  This is the serving analog
 * of running super sampling and frame interpolation concurrently on one GPU
 * (3DGS^3 Sec. 5.1, 5.3).
 *
 * Cost-aware admission: each (scene, raster size) class keeps an estimate of
 * its frame time, first from its pair count, then from the measured time of
 * its single-frame batches (an exponential average).  A frame estimated at
 * or above heavy_ms starts on an idle device and only tiny frames (at most a
 * quarter of heavy_ms) start beside it, so that sharing the device barely
 * stretches the longest frames; lighter frames are batched and overlap on
 * the streams.  A heavy frame at the head of the queue holds back the frames
 * behind it until it has started (arrival order is kept).
 *
 * A batch's stages are single launches over the concatenated Gaussians,
 * pairs and tiles of all its frames, the frames ordered by estimated time
 * (shortest first).  With work_queue = 1, the compositing of a batch of
 * several frames is a persistent grid (no more workgroups than the device
 * holds at once) that takes the batch's tiles from a queue counter in device
 * memory, frame after frame.  A workgroup leaving a frame adds its tiles to
 * the frame's count, and the one that completes it stores the batch's
 * sequence number into that frame's word of a pinned, coherent host array,
 * after releasing the frame's outputs at system scope; gs_poll reports the
 * frame done as soon as that word matches, without waiting for the rest of
 * the batch (the batch's last frame is done with the batch).  Each
 * publication writes back an L2 of the device (one per workgroup and frame),
 * which costs more compositing time than the early reports save at the
 * rates measured here, so the mode is off by default.  A batch whose pairs
 * overflow its key capacity composites nothing and is re-run as below.
 *
 * Memory: scenes are copied into server-owned device memory; every admitted
 * request holds its outputs (52 B per pixel) and its share of the batch
 * workspace; all of it is charged to hbm_budget_bytes and handed out by a
 * first-fit arena.  The workspace is sized from a per-(scene, resolution)
 * estimate of the frame's (tile, Gaussian) pairs (first request of a class:
 * a synchronous projection probe; afterwards the largest count seen) times
 * key_factor; a frame that needs more pairs is re-run once with enough room.
 *
 * All server calls are host calls and thread safe.  gs_submit and gs_poll
 * never block on the GPU; gs_server_destroy waits for work in flight.
 * With simulate = 1 no device call is made at all: scenes and outputs are
 * bookkeeping only and every batch "runs" for sim_batch_us microseconds
 * (a dry run of the admission and batching policy); sim_fail_every = k > 0
 * then makes every k-th batch report GS_ERR_HIP for its requests. */
typedef struct gs_server gs_server;

typedef struct gs_server_opts {
    size_t hbm_budget_bytes;    /* device memory for scenes + requests in flight */
    int32_t max_batch;          /* frames per launch, 1..GS_MAX_BATCH */
    int32_t queue_depth;        /* pending requests before gs_submit says AGAIN */
    int32_t n_streams;          /* batches in flight at once, 1..8 */
    int32_t fifo;               /* 1: one frame per launch, one launch at a time, arrival order */
    double key_factor;          /* key capacity = factor x estimated pairs (>= 1) */
    int32_t simulate;           /* 1: no device calls (policy dry run) */
    int32_t sim_fail_every;     /* simulate only: every k-th batch fails */
    double sim_batch_us;        /* simulate only: duration of a batch */
    double heavy_ms;            /* a frame whose class is estimated at or above this many
                                   milliseconds starts on an idle device, and only frames
                                   estimated at a quarter of it or below start beside it;
                                   0: every frame may share the device */
    int32_t work_queue;         /* 1: batches of several frames are composited by the
                                   persistent work-queue kernel, which reports every frame but
                                   the batch's last done as soon as it is complete; 0: one
                                   workgroup per tile, every frame done with its batch */
} gs_server_opts;

typedef struct gs_result {
    int32_t status;             /* GS_OK, GS_ERR_NOT_READY or the request's error */
    int32_t width, height;
    int32_t batch_size;         /* frames in the launch that rendered it */
    int32_t retries;
    int32_t flag_done;          /* 1: completion was read from the frame's completion word
                                   (work_queue) while its batch may still have been running;
                                   0: at the batch's end */
    gs_outputs out;             /* device pointers into server memory, valid until gs_release */
    double t_submit, t_start, t_done;   /* seconds, CLOCK_MONOTONIC; t_done is poll-visible completion */
} gs_result;

/* Returns GS_ERR_INVALID_ARG for bad options, GS_ERR_OOM if the budget
 * cannot be reserved on the current device. */
int gs_server_create(const gs_server_opts* opts, gs_server** server);
int gs_server_destroy(gs_server* server);
/* Copies a scene (device arrays as in gs_scene) into server memory and
 * charges it to the budget: GS_ERR_OOM when it does not fit. */
int gs_scene_register(gs_server* server, const gs_scene* scene, int32_t* scene_id);
/* Queues a request; *ticket identifies it.  GS_ERR_AGAIN when queue_depth
 * requests are pending, GS_ERR_TOO_LARGE when the request alone (its
 * outputs and a workspace for its projection) needs more memory than the
 * resident scenes leave of the budget, GS_ERR_NOT_FOUND for an unknown
 * scene.  A request admitted before more scenes were registered and no
 * longer fitting finishes with GS_ERR_TOO_LARGE. */
int gs_submit(gs_server* server, int32_t scene_id, const gs_camera* cam,
              const gs_render_opts* opts, uint64_t* ticket);
/* GS_ERR_NOT_READY while in flight; GS_OK with *result when done (result
 * status carries a failed request's error code); GS_ERR_NOT_FOUND for an
 * unknown or released ticket. */
int gs_poll(gs_server* server, uint64_t ticket, gs_result* result);
/* Returns a finished request's output memory to the budget. */
int gs_release(gs_server* server, uint64_t ticket);
/* stats9 (host): submitted, completed, failed, rejected, batches launched,
 * frames in the largest batch, arena bytes in use, arena bytes peak, frames
 * completed from their completion word. */
int gs_server_stats(gs_server* server, int64_t* stats9);

const char* gs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GS3_H */
