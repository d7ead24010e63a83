/*
 * lucidraster.h -- C ABI of an MI355X (gfx950) software rasterizer for exact
 * order-independent transparency of planar quads, after "LucidRaster: GPU
 * Software Rasterizer for Exact Order-Independent Transparency"
 * (K. Jakubowski, arXiv 2405.13364).
 *
 * The problem (paper, Section 1): for every pixel, find every fragment that
 * contributes to it, sort the fragments by depth and blend them in order.
 * The pipeline follows Section 2: quad setup (Stage 1), binning into
 * screen-space bins by prefix sums (Stage 2), and bin rasterization with a
 * two-stage sort -- depth-sorted blocks of fragments refined by a per-pixel
 * fixed-size sorter -- and front-to-back blending (Stage 3).  Unlike the
 * paper, pixels whose per-pixel sorter would emit fragments out of order are
 * detected exactly and recomputed by a full per-pixel sort, so every image is
 * exact (Stage 3, "Sample blending", describes the detection; the paper
 * leaves such pixels unfixed).
 *
 * Conventions (numeric readings of the paper, stated once here):
 *   - camera space c = R (v - pos); the camera looks down +z, y up; screen x
 *     points right, y down; f = (H/2) / tan(fov_y/2) is computed on the host;
 *   - vertices are snapped to a 1/256-pixel grid; pixel (i, j) samples its
 *     centre; a quad covers a sample when one of its triangles (P0,P1,P2),
 *     (P0,P2,P3) does, under a top-left fill rule; one fragment per quad;
 *   - depth order: reciprocal view depth from the plane through the vertex
 *     centroid normal to the diagonals, evaluated in fp64 and rounded to
 *     fp32; nearer first, ties by ascending quad index;
 *   - blending: front to back from transparent black, fp32; the output is
 *     premultiplied RGBA8 (rounded half up).
 *
 * Memory: the caller owns all device memory.  lr_create takes a device arena
 * the library sub-allocates from (it never calls hipMalloc); render outputs
 * are device pointers.  Every call returns an
 * lr_status; no exception or abort crosses the ABI; outputs are only written
 * on LR_OK.  Rendering calls are asynchronous on the given HIP stream; errors
 * found by kernels (capacity overflow) are latched in the context and
 * reported by the next lr_sync / lr_get_stats.
 */
#ifndef LUCIDRASTER_H
#define LUCIDRASTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lr_status;
#define LR_OK 0
#define LR_ERR_INVALID_ARG -1   /* a NULL pointer, zero size, size out of range */
#define LR_ERR_OUT_OF_MEMORY -2 /* the arena cannot hold the request */
#define LR_ERR_DEVICE -3        /* a HIP call failed (text in lr_last_error) */
#define LR_ERR_CAPACITY -4      /* a frame overflowed a device capacity; re-render */
#define LR_ERR_NOT_FOUND -5     /* unknown scene handle */
#define LR_ERR_BUSY -6          /* the context is in use by another thread */

typedef struct lr_context_s *lr_context;
typedef uint64_t lr_scene; /* 0 is never a valid handle */

/* One input quad: four world-space vertices and one straight-alpha RGBA8
 * colour (R in the low byte).  52 bytes, packed.  A quad's index in the
 * uploaded array is its id (the depth tie-break). */
#pragma pack(push, 4)
typedef struct {
    float v[4][3];
    uint32_t rgba;
} lr_quad;
#pragma pack(pop)

/* A quad with one straight-alpha RGBA8 colour per vertex (R in the low
 * byte).  64 bytes, packed. */
#pragma pack(push, 4)
typedef struct {
    float v[4][3];
    uint32_t rgba[4];
} lr_quad_vc;
#pragma pack(pop)

/* Pinhole camera: rows of rot are the camera x, y, z axes in world space. */
typedef struct {
    float pos[3];
    float rot[3][3];
    float fov_y;  /* radians */
    float z_near; /* quads with any vertex at view depth <= z_near are culled */
} lr_camera;

/* Context configuration.  Zero fields take defaults. */
typedef struct {
    int32_t device;           /* HIP device ordinal */
    void *stream;             /* default hipStream_t for calls given NULL */
    void *arena;              /* device memory owned by the caller (required) */
    uint64_t arena_bytes;     /* its size in bytes (at least 1 MiB) */
    uint32_t bin_size;        /* 16, 32 (default) or 64 pixels */
    uint32_t block_h;         /* depth-sort granularity: 8 for 8x8 blocks
                                 (default), 4 for 8x4 half-blocks (Stage 3,
                                 Phase 2); images are identical either way */
    uint32_t sorter_depth;    /* per-pixel sorter capacity K: 2, 4, 8
                                 (default), 12, 16, 24 or 32 */
    uint32_t flags;           /* LR_FLAG_* */
    uint64_t hbm_budget_bytes;/* serving admission budget (0: arena size) */
    uint32_t batch_slots;     /* batch workspaces that may be in flight at
                                 once, on different streams (default 2, at
                                 most 8) */
    uint32_t reserved;
} lr_config;

#define LR_FLAG_TIMING 1u     /* record per-stage times (hipEvents) */
#define LR_FLAG_NO_GRAPH 2u   /* lr_render_batch launches directly instead
                                 of replaying captured hipGraphs */
#define LR_FLAG_ALPHA_CUTOFF 4u /* transmittance cutoff, the tolerance-safe
                                 form of the alpha threshold of Stage 3
                                 ("Sample blending"): a pixel stops after the
                                 first fragment (in exact depth order) that
                                 brings its fp32 transmittance below 2^-20,
                                 so the colour differs from the full blend by
                                 less than 2^-20 per channel.  Pixels whose
                                 transmittance gets there skip the rest of
                                 their fragments once per-entry depth bounds
                                 show none of them can come earlier.  Parity
                                 dumps then report the blended prefix
                                 (counts, order).  The unsorted baseline
                                 ignores it. */
#define LR_FLAG_BBOX_BINNING 16u /* bin every quad to every bin its pixel
                                 bbox meets.  By default a large quad (bbox
                                 over more than 4 bins of 32 x 32 pixels, the
                                 small/large split of Stage 1, Phase 1) is
                                 binned only to the bins its edges do not
                                 trivially reject (Stage 2, "Triangle
                                 rasterization": a bin-level scan with a
                                 trivial-reject test).  Setup lists the large
                                 quads and every binning workgroup takes a
                                 share of the list after its own small quads,
                                 with each large quad's bins spread over the
                                 lanes of a wave; a bin list then holds its
                                 small quads in ascending order and its large
                                 quads in no set order (the unsorted baseline,
                                 which blends in quad order, always bins by
                                 bbox).  Images are identical either way. */
#define LR_FLAG_CULL_BACKFACES 32u /* cull quads facing away from the camera
                                 (Stage 1): with n the cross product of the
                                 diagonals and m the vertex centroid in camera
                                 space, n . m < 0, i.e. the vertices wind
                                 clockwise on the display (front faces wind
                                 counter-clockwise, as OpenGL's default) */
#define LR_FLAG_DENSITY_CLASSES 8u /* density classes (Section 4 proposes
                                 adapting bins to the density and running the
                                 low- and high-density rasterizers at the
                                 same time): with a sorter depth above 4,
                                 binning also estimates each bin's depth
                                 complexity (the bbox pixels of its quads per
                                 pixel), and one raster launch takes the
                                 bins above 32 first and runs those at most
                                 2 with a depth-4 sorter.  Images are
                                 identical either way; off by default, since
                                 on the workloads measured here it is slower
                                 (the estimate costs the count stage, and
                                 dense bins run together contend where screen
                                 order mixes them with light ones). */

/* Statistics of the last render call on the context (for a batch, summed over
 * its frames; error_word is the OR of theirs). */
typedef struct {
    uint64_t quads;           /* input quads */
    uint64_t visible;         /* quads that passed setup */
    uint64_t culled[8];       /* [1] near [2] guard band [3] degenerate
                                 [4] no sample [5] edge-on plane
                                 [6] back-facing ([0], [7] unused) */
    uint64_t bin_pairs;       /* (bin, quad) pairs written by binning */
    uint64_t block_entries;   /* non-empty (block, quad) pairs */
    uint64_t fragments;       /* covered (pixel, quad) pairs */
    uint64_t flagged_pixels;  /* pixels recomputed by the exact per-pixel sort */
    uint64_t dense_blocks;    /* blocks with more entries than one on-chip sort
                                 (1024), processed in depth slices */
    uint32_t error_word;      /* device error bits (0: none) */
    uint32_t reserved;
    float stage_us[8];        /* setup, bin count, bin scan, bin scatter,
                                 raster, (unused), exact per-pixel pass, total */
} lr_stats;

/* A request for lr_render_batch.  A zero tuning field takes the first
 * matching rule set by lr_set_tuning, else the context default.  (Batching is
 * this library's own addition; each frame is the render of Section 2.) */
typedef struct {
    lr_scene scene;
    lr_camera camera;
    uint32_t width, height;
    uint8_t *out_rgba8;       /* device, width*height*4 bytes */
    uint32_t bin_size;        /* 16, 32, 64 or 0 */
    uint32_t sorter_depth;    /* as lr_config.sorter_depth, or 0 */
    uint32_t block_h;         /* 4, 8 or 0 */
    uint32_t reserved;
    uint32_t *status;         /* NULL, or a device word that receives the
                                 frame's error bits, stream-ordered after the
                                 frame's kernels: 0 when the image was
                                 written, else LR_FRAME_ERR_* bits.  Lets a
                                 caller that polls completion events find a
                                 failed frame without a device-wide lr_sync. */
} lr_request;

/* Error bits of a frame (lr_request.status, lr_stats.error_word). */
#define LR_FRAME_ERR_CAPACITY 1u  /* its bin lists overflowed: the image was
                                     not written; lr_sync raises the capacity
                                     and a second render succeeds */
#define LR_FRAME_ERR_DENSE 4u     /* a block held more equal-depth entries
                                     than one on-chip sort; its pixels were
                                     recomputed by the exact per-pixel sort
                                     (informational: the image is exact) */

/* A tuning rule: applies to frames of at most max_pixels pixels with at most
 * max_quads_per_pixel quads per pixel (resident quads / (width*height)).
 * The autotuner writes these from a sweep of frame shapes (the paper's
 * Section 4 suggests adapting the bin size to the scene). */
typedef struct {
    uint32_t max_pixels;
    float max_quads_per_pixel;
    uint32_t bin_size, block_h, sorter_depth;
    uint32_t reserved;
} lr_tune_rule;

/* Human-readable name of a status code (static storage).  This library's
 * own error reporting; the paper has no API. */
const char *lr_status_string(lr_status s);

/* Last error message of the context (or of the process when ctx is NULL).
 * This library's own error reporting. */
const char *lr_last_error(lr_context ctx);

/* Create a context on cfg->device over the caller's device arena (the
 * renderer's state of Section 2: resident scenes and per-frame buffers).
 * Fails with LR_ERR_INVALID_ARG for a bad config or a NULL arena,
 * LR_ERR_DEVICE when HIP is unavailable.  *out is written only on LR_OK. */
lr_status lr_create(const lr_config *cfg, lr_context *out);

/* Wait for the context's work and free its host state.  Caller memory (the
 * arena, outputs) is left untouched.  This library's own lifetime call. */
lr_status lr_destroy(lr_context ctx);

/* Make quads resident on the device: the input of Stage 1 ("Phase 1:
 * processing input quads"), off the per-frame work.  q points to n lr_quad
 * records in host memory (q_on_device == 0) or device memory (q_on_device !=
 * 0).  The data is copied and transposed into the arena (structure of
 * arrays); the call waits for the copy, so q may be freed or reused when it
 * returns.  1 <= n <= 2^24; LR_ERR_OUT_OF_MEMORY when the arena is full. */
lr_status lr_upload_scene(lr_context ctx, const lr_quad *q, uint32_t n, int q_on_device,
                          lr_scene *out);

/* Make quads with per-vertex colours resident (host memory; the call waits
 * for the copy).  Every render of such a scene interpolates the colours per
 * sample (Stage 3, "Sample shading"): a covered sample takes triangle T0 =
 * (P0, P1, P2) if T0 covers it, else T1 = (P0, P2, P3), and the barycentric
 * mix of that triangle's vertex colours where the ray through the pixel
 * centre meets the triangle's plane (perspective-correct), blended in fp32
 * without rounding to 8 bits.  Such frames sort at depth 16 at most (a
 * deeper sorter depth is lowered to 16; the image never depends on it).
 * Rendering such a scene with LR_FLAG_ALPHA_CUTOFF fails with
 * LR_ERR_INVALID_ARG.  1 <= n <= 2^24;
 * LR_ERR_OUT_OF_MEMORY when the arena is full (68 bytes per quad). */
lr_status lr_upload_scene_vertex_colors(lr_context ctx, const lr_quad_vc *q, uint32_t n, lr_scene *out);

/* Return a scene's arena space (after the device drains).  This library's
 * own memory management. */
lr_status lr_release_scene(lr_context ctx, lr_scene scene);

/* Render a scene into out_rgba8 (device, width*height*4 bytes, row-major, top
 * row first, premultiplied RGBA8): the whole pipeline of Section 2 -- setup
 * (Stage 1), binning (Stage 2), rasterization with the two-stage sort and
 * front-to-back blending (Stage 3), plus the exact per-pixel pass for pixels
 * the per-pixel sorter could not order ("Sample blending").
 * 1 <= width, height <= 16384.  Runs on stream (NULL: the context stream) and
 * returns without waiting.  The bin size, block shape and sorter depth come
 * from the first matching tuning rule (lr_set_tuning), else from the context
 * configuration; the image does not depend on them. */
lr_status lr_render(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                    uint32_t height, uint8_t *out_rgba8, void *stream);

/* For callers that cannot allocate device memory during a render: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The same render as lr_render, bit-identical for the same tuning, but its
 * frame workspace (quad records, bin lists, block entries, counters, the
 * flagged-pixel queue) lives in a fixed array of 128 MiB that each device
 * loading the library holds until the process ends; the call allocates
 * nothing (no hipMalloc, hipFree or arena sub-allocation).  The scene must
 * already be resident (lr_upload_scene) and out_rgba8 is the caller's.
 * Returns LR_ERR_OUT_OF_MEMORY, without launching anything, when the frame's
 * workspace would exceed 128 MiB (a 1280x720 frame of 200k quads at bin 32
 * fits; lr_request_bytes gives the figure).  Every call on one device, from any
 * context, shares that array and leaves its contents behind: calls that
 * overlap on one device race.  Calls of one context are ordered after each
 * other even on different streams; calls of different contexts on one
 * device must be ordered by the caller.  Capacity overflows are reported as
 * for lr_render (the next lr_sync), after which a second call succeeds. */
lr_status lr_render_noalloc(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                            uint32_t height, uint8_t *out_rgba8, void *stream);

/* Same render (Section 2), plus parity artefacts (each may be NULL):
 *   rgba_f32  [H][W][4] fp32 premultiplied colour before rounding;
 *   counts    [H][W] fragments per pixel;
 *   flagged   [H][W] 1 where the per-pixel sorter detected an order
 *             violation (those pixels were recomputed exactly; Stage 3,
 *             "Sample blending");
 *   order_offsets [W*H+1] (input, e.g. the exclusive scan of counts) and
 *   order_ids [order_cap]: quad ids of each pixel in blend order. */
lr_status lr_render_debug(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                          uint32_t height, uint8_t *out_rgba8, void *stream, float *rgba_f32,
                          uint32_t *counts, uint8_t *flagged, const uint32_t *order_offsets,
                          uint32_t *order_ids, uint32_t order_cap);

/* The unsorted baseline: the same setup and binning, then per pixel the
 * covering quads blended in quad order with the "over" operator (fp32), as
 * hardware alpha blending would without sorting (Section 3, "Performance
 * results", the hardware reference).  rgba_f32 may be NULL. */
lr_status lr_render_unsorted(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                             uint32_t height, uint8_t *out_rgba8, void *stream, float *rgba_f32);

/* Render n requests (uneven sizes and tunings allowed) on one stream.  Each
 * stage runs as one launch over up to 64 frames at a time (one per distinct
 * sorter depth for the raster stage), so small frames share the GPU; the
 * launch sequence is captured once per batch shape into a hipGraph and
 * replayed (unless LR_FLAG_NO_GRAPH).  Every output is bit-identical to
 * lr_render of the same request with the same tuning.  The batch uses one of
 * the context's batch workspaces: batches on different streams run
 * concurrently, up to lr_config.batch_slots at a time.  Returns
 * LR_ERR_OUT_OF_MEMORY when one frame alone does not fit the arena.
 * Batching is this library's own addition (each frame is the render of
 * Section 2); a request's status word, if given, reports its frame's errors. */
lr_status lr_render_batch(lr_context ctx, const lr_request *reqs, uint32_t n, void *stream);

/* Replace the tuning rules (copied; n = 0 clears them).  Rules are tried in
 * order; max_pixels must be non-zero and the tuning values valid.  Section 4
 * suggests adapting the bin size to the scene; the rules are this library's
 * per-frame form of it. */
lr_status lr_set_tuning(lr_context ctx, const lr_tune_rule *rules, uint32_t n);

/* Device memory one request needs while in flight (its frame workspace,
 * after tuning), for admission control.  Does not allocate.  Section 4 names
 * memory use as the method's cost; admission is this library's own. */
lr_status lr_request_bytes(lr_context ctx, const lr_request *req, uint64_t *bytes);

/* Wait for all work the context issued; report a latched kernel error
 * (LR_ERR_CAPACITY) and clear it.  This library's own. */
lr_status lr_sync(lr_context ctx);

/* Wait, then fill *out with the statistics of the last render (the per-stage
 * quantities Section 3 reports: samples, stage times).  This library's own. */
lr_status lr_get_stats(lr_context ctx, lr_stats *out);

/* Per-stage times (microseconds, layout of lr_stats.stage_us) of the last
 * min(max_frames, frames rendered, 1024) frames, oldest first, into
 * us[frame][8]; *n_out receives the number of frames.  Needs a context
 * created with LR_FLAG_TIMING; synchronises.  The stages are those of
 * Section 3's timing tables (setup, binning, rasterization). */
lr_status lr_get_stage_times(lr_context ctx, uint32_t max_frames, float *us, uint32_t *n_out);

/* Parity dump of the setup stage (Stage 1, Phases 1 and 2) for a render
 * configuration (synchronous).  Per quad: X, Y [n][4] snapped vertices; bbox
 * [n][4] (imin, imax, jmin, jmax of a visible quad); plane [n][3] (A, B, C0);
 * cull [n] (0 visible, else the reason as in lr_stats.culled).  Host
 * pointers; any may be NULL. */
lr_status lr_debug_setup(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                         uint32_t height, int32_t *X, int32_t *Y, int32_t *bbox, double *plane,
                         uint8_t *cull);

/* Parity dump of binning (Stage 2, synchronous): per-bin counts [nbins] and,
 * when ids is not NULL, the concatenated per-bin lists of quad ids (ids_cap
 * entries at most; *total receives the number of pairs). */
lr_status lr_debug_bins(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                        uint32_t height, uint32_t bin_size, uint32_t *counts, uint32_t *ids,
                        uint64_t ids_cap, uint64_t *total);

#ifdef __cplusplus
}
#endif
#endif /* LUCIDRASTER_H */
