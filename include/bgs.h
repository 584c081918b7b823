/*
 * bgs.h -- C ABI of the binocular 2D Gaussian Splatting frame path for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: "From Mono to Stereo: Accelerating Binocular Gaussian Splatting
 * via Reprojection and Selective Patching".  The path renders the dominant
 * eye completely, with RGB and an alpha-weighted depth proxy accumulated
 * from the same blending weights (Sec. 3.1 Stage 1); reprojects it to the
 * affiliated eye with the pinhole model (Sec. 3.4, Eq. 3-5); classifies
 * the uncovered pixels into interpolated gaps and regions of interest
 * (Sec. 3.1 Stage 3, Sec. 3.5 Step 1 Eq. 6-8 and Step 2); and re-renders
 * only the 16x16 tiles those ROIs touch (Sec. 3.1 Stage 4).
 *
 * Conventions used by every call:
 *   - All image, scene and output pointers are DEVICE pointers owned by the
 *     caller; the library never allocates device memory.  Scratch memory is
 *     a caller-provided workspace sized with bgs_workspace_size().
 *   - Images are planar fp32: RGB is [3][H][W], single channels [H][W],
 *     row-major, pixel (i, j) = column i, row j, pixel centres at integer
 *     coordinates.
 *   - Camera frame: x right, y down, z forward; depth is z along the
 *     optical axis (Eq. 3).  A pose (R, t) maps camera to world,
 *     X_w = R X_c + t (Eq. 4), so X_c = R^T (X_w - t) (Eq. 5).
 *   - Every call is enqueued on the context's HIP stream.  In synchronous
 *     mode (the default) the render calls wait for the stream once at the
 *     end to read the key count and the overflow flags; in asynchronous mode
 *     no call waits and bgs_poll_status() reports them later.
 *   - Every call returns a bgs_status.  On an error nothing is guaranteed
 *     about the outputs and bgs_last_error() describes the failure.
 *     Arguments are validated on the host before anything is launched.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef BGS_H
#define BGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BGS_API __attribute__((visibility("default")))

typedef enum bgs_status {
    BGS_OK = 0,
    BGS_ERR_INVALID_ARG = -1,  /* null pointer, size out of range, bad parameter */
    BGS_ERR_WORKSPACE = -2,    /* workspace smaller than bgs_workspace_size() */
    BGS_ERR_CAPACITY = -3,     /* more tile keys than the workspace holds */
    BGS_ERR_HIP = -4,          /* a HIP runtime call or launch failed */
    BGS_ERR_UNSUPPORTED = -5   /* a valid but unsupported setting (e.g. an ROI tile other than 8, 16, 32) */
} bgs_status;

/* Pinhole camera (Eq. 3-5).  width, height in [1, 16384]; fx, fy > 0;
 * R orthonormal within 1e-6; 0 < z_near < z_far.  Surfels whose centre
 * depth is not beyond z_near are culled, and ray hits at depth <= z_near
 * are ignored.  z_far only bounds the depth range when an image has no
 * covered pixel. */
typedef struct bgs_camera {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9]; /* camera-to-world rotation, row-major */
    double t[3]; /* camera centre in world */
    double z_near, z_far;
} bgs_camera;

/* A static trained 2DGS scene (Sec. 3.3, Eq. 1): structure of arrays of
 * activated fp32 values on the device.
 *   pos[3][n]            centres p_k
 *   quat[4][n]           rotation quaternion (w, x, y, z); its matrix has
 *                        columns t_u, t_v, t_w = t_u x t_v
 *   scale[2][n]          in-plane scales s_u, s_v > 0
 *   opacity[n]           in [0, 1]
 *   sh[(deg+1)^2*3][n]   real spherical-harmonic colour coefficients,
 *                        plane index = coef*3 + channel, coef = l*l+l+m,
 *                        Condon-Shortley phase; colour = max(0, sum + 0.5)
 *                        evaluated towards the surfel from the camera centre.
 * 0 <= n < 2^31; sh_degree in 0..3.  n = 0 renders the background. */
typedef struct bgs_scene {
    int64_t n;
    int32_t sh_degree;
    int32_t reserved;
    const float* pos;
    const float* quat;
    const float* scale;
    const float* opacity;
    const float* sh;
} bgs_scene;

/* Compositing constants of the 2DGS rasteriser the method builds on:
 * alpha = min(alpha_max, opacity * G); a pair with alpha < alpha_min is
 * skipped; compositing of a pixel stops before the surfel that would bring
 * the transmittance below t_min.  lowpass = 1 adds the screen-space term
 * G2 = exp(-|x - mu|^2) with G = max(G3, G2).  bg is the background colour
 * added with the final transmittance.  Defaults: 1/255, 0.99, 1e-4, 1, 0. */
typedef struct bgs_raster_params {
    float alpha_min;
    float alpha_max;
    float t_min;
    int32_t lowpass;
    float bg[3];
    int32_t reserved;
} bgs_raster_params;

/* ROI generator settings (Sec. 3.5).  margin m >= 0 pixels (32 in the
 * paper); tile T is the ROI tile size: 16, the rasteriser's native tile
 * the paper aligns ROIs to, or 8 or 32 (an option for tuning): ROI boxes
 * are aligned outward to multiples of T, the tile mask holds T x T tiles,
 * and the patch re-renders exactly the pixels of the masked T-tiles (the
 * rasteriser still bins 16x16 tiles; with T = 8 it composites only the
 * masked 8x8 quadrants of each binned tile); edge_samples N
 * in [1, 65536] per image edge; gap_passes in [0, 64]; center_roi = 1
 * enables Step 2 (connected center holes), 0 fills the remaining holes
 * along their row instead; a_min in (0, 1] is the accumulated weight A
 * below which a source pixel counts as empty background.  edge_bounds
 * selects the valid projection bounds of Eq. 7-8: 0 takes the extrema of
 * Eq. 6 over all projected edge samples (as the paper writes it); 1 takes,
 * for each side, the worst case of that side's own edge over both depth
 * hypotheses (u_min = largest x of the left edge, u_max = smallest x of
 * the right edge, likewise v for top and bottom), which covers the strip a
 * border leaves uncovered at any depth in the range; a side whose edge has
 * no valid projection falls back to Eq. 6. */
typedef struct bgs_roi_params {
    int32_t margin;
    int32_t tile;
    int32_t edge_samples;
    int32_t gap_passes;
    int32_t center_roi;
    float a_min;
    int32_t edge_bounds;
    /* 1: view-colour transfer, an option outside the paper's method (which
     * reprojects the dominant image's colours, 0, the default).  The
     * dominant pass of bgs_render_stereo also composites every surfel's
     * colour seen from the affiliated eye's centre (its SH evaluated
     * towards the surfel from there) with the dominant eye's weights, and
     * the reprojection moves that colour instead, so warped pixels keep the
     * affiliated view's view-dependent colour.  The dominant outputs are
     * unchanged.  A no-op for degree-0 scenes (nothing is added then); the
     * dominant pass then never splits long lists into continuation
     * segments.  bgs_render_stereo only: the batched form rejects it. */
    int32_t view_colour;
} bgs_roi_params;

/* Box kinds. */
enum { BGS_BOX_LEFT = 0, BGS_BOX_RIGHT = 1, BGS_BOX_TOP = 2, BGS_BOX_BOTTOM = 3, BGS_BOX_CENTER = 4 };
/* Per-pixel classes of the affiliated eye. */
enum { BGS_CLS_WARPED = 0, BGS_CLS_HOLE = 1, BGS_CLS_GAP = 2, BGS_CLS_ROI = 3, BGS_CLS_ROWFILL = 4 };

/* An ROI: half-open pixel rectangle [x0,x1)x[y0,y1), aligned outward to the
 * tile grid and clipped to the image; label is the component label (the
 * smallest linear pixel index of the component) of a center box, -1 for an
 * edge box. */
typedef struct bgs_box {
    int32_t x0, y0, x1, y1, kind, label;
} bgs_box;

/* Per-frame statistics; overflow bit 0 = tile-key capacity exceeded, bit 1
 * = box capacity exceeded (the tile mask is still complete).  n_roi_tiles
 * counts the 16x16 rasteriser tiles the ROI pass re-rendered. */
typedef struct bgs_stats {
    int64_t n_keys_dom, n_keys_roi;
    int32_t n_holes, n_gap, n_center, n_rowfill, n_boxes, n_roi_tiles;
    int32_t overflow;
    int32_t reserved;
    /* Only with bgs_ctx_set_count_pairs(ctx, 1): (pixel, surfel) pairs the
     * blend evaluated, and those that contributed to a pixel; and the blend's
     * work shape {records walked summed over waves, records that passed a
     * wave's strip test, longest walk of one wave, longest tile list}. */
    int64_t pairs_eval_dom, pairs_used_dom, pairs_eval_roi, pairs_used_roi;
    int64_t blend_work_dom[4], blend_work_roi[4];
} bgs_stats;

typedef struct bgs_ctx bgs_ctx;

/* Context: a HIP stream (NULL = the null stream) and the last error text.
 * The context is a small host object; it owns no device memory. */
BGS_API int32_t bgs_ctx_create(bgs_ctx** ctx, void* hip_stream);
BGS_API int32_t bgs_ctx_destroy(bgs_ctx* ctx);
BGS_API int32_t bgs_ctx_set_stream(bgs_ctx* ctx, void* hip_stream);
/* sync = 1 (default): render calls wait at their end and report the key
 * count and capacity overflow; sync = 0: nothing waits. */
BGS_API int32_t bgs_ctx_set_sync(bgs_ctx* ctx, int32_t sync);
BGS_API const char* bgs_last_error(const bgs_ctx* ctx);
/* count = 1: the blend kernels also count evaluated and contributing
 * (pixel, surfel) pairs into bgs_stats (slower; for measurement only). */
BGS_API int32_t bgs_ctx_set_count_pairs(bgs_ctx* ctx, int32_t count);

/* Scheduling of long tile lists in the blend; the pixels agree with a
 * single front-to-back walk to fp32 rounding.  A tile composites at most
 * `cap` records of its list in its own workgroup (cap_dom for the dominant
 * eye and full renders, cap_roi for the ROI patch; 0 = the whole list).
 * Where pixels are still compositing after that, at least 2 seg_len records
 * remain, and some pixel, extrapolating the decay of its transmittance
 * over the second half of the capped walk, is expected to composite at
 * least `far` more records (far_dom, far_roi), the rest of the list is
 * split into up to 32 segments of about seg_len records that other
 * workgroups composite speculatively; the segments are chained front to
 * back, and a pixel that stops inside a segment is composited again over
 * that segment, in order, from its exact state (unless the segment's own
 * walk started from that state).  Lists are continued only on images of at
 * most 4096 16x16 tiles (larger ones fill the GPU with their tiles alone).
 * Defaults 1024, 32, 32, 0, 256.  BGS_ERR_INVALID_ARG for a negative cap or far, or seg_len < 1. */
BGS_API int32_t bgs_ctx_set_blend_split(bgs_ctx* ctx, int32_t cap_dom, int32_t cap_roi, int32_t seg_len,
                                        int32_t far_dom, int32_t far_roi);

/* Per-stage GPU timing with HIP events recorded on the context's stream
 * around each stage's launches.  stages is a bit mask over enum bgs_stage
 * (bit i times stage i; -1 times every stage; 0 turns timing off); every
 * call clears the totals.  Each timed stage adds two event records to the
 * stream, so time only the stages you need where the frame rate matters.
 * Frames may be issued back to back: the events of the last 64 frames are
 * kept, and older ones are folded into the totals as new frames start (a
 * frame 64 frames old has long finished).  bgs_timing_collect() waits for
 * the recorded stages, adds them to the totals and copies totals (ms) and
 * counts for the BGS_NUM_STAGES stages, in the order of enum bgs_stage. */
enum bgs_stage {
    BGS_STAGE_PREPROCESS_DOM = 0, BGS_STAGE_DEPTH_SORT_DOM, BGS_STAGE_EMIT_DOM, BGS_STAGE_TILE_SORT_DOM,
    BGS_STAGE_RANGES_DOM, BGS_STAGE_BLEND_DOM, BGS_STAGE_REPROJECT, BGS_STAGE_CLASSIFY,
    BGS_STAGE_PREPROCESS_ROI, BGS_STAGE_DEPTH_SORT_ROI, BGS_STAGE_EMIT_ROI, BGS_STAGE_TILE_SORT_ROI,
    BGS_STAGE_RANGES_ROI, BGS_STAGE_BLEND_ROI, BGS_NUM_STAGES
};
BGS_API int32_t bgs_ctx_set_timing(bgs_ctx* ctx, int32_t stages);
BGS_API int32_t bgs_timing_collect(bgs_ctx* ctx, double* total_ms, int64_t* counts);

/* Workspace bytes for scenes of up to n surfels, images of up to
 * width x height, and up to key_capacity (surfel, tile) keys per render.
 * The render calls derive their key capacity from the size they are given,
 * so a larger workspace simply holds more keys.  Allocate it 256-byte
 * aligned (any torch allocation is). */
BGS_API int32_t bgs_workspace_size(int64_t n, int32_t width, int32_t height, int64_t key_capacity,
                                   size_t* bytes);

/* Status of the last asynchronous render on this context: number of keys
 * of the last dominant and ROI passes and the overflow flags.  The
 * overflow bits are those of ANY frame rendered with this workspace since
 * the previous poll (each frame's reset folds the last frame's bits into a
 * sticky word that only this call clears), so one poll after a run of
 * asynchronous frames tells whether any of them ran out of capacity.
 * Waits for the context's stream. */
BGS_API int32_t bgs_poll_status(bgs_ctx* ctx, void* ws, size_t ws_bytes, bgs_stats* stats);

/* Stage 1 (Sec. 3.1, Sec. 3.3): full tile rasterisation of one eye.
 * Outputs rgb[3][H][W] = sum w_i c_i + T bg, depth_raw[H][W] = D =
 * sum d_i w_i (d_i the ray-surfel intersection depth, or the centre depth
 * where the low-pass term dominates) and alpha[H][W] = A = sum w_i, all
 * from the same weights w_i = alpha_i T_i.  The depth proxy is D/A.
 * n_keys (host, optional) receives the number of (surfel, tile) keys.
 * Returns BGS_ERR_CAPACITY (and the required count in *n_keys) when the
 * workspace holds too few keys. */
BGS_API int32_t bgs_render_dominant(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam,
                                    const bgs_raster_params* raster, void* ws, size_t ws_bytes, float* rgb,
                                    float* depth_raw, float* alpha, int64_t* n_keys);

/* Stage 2 (Sec. 3.4, Eq. 3-5): forward reprojection to the destination
 * camera.  A source pixel with A >= a_min carries depth d = D/A (fp32);
 * it is unprojected, moved to the destination frame with the relative
 * pose in fp64, projected and rounded to the nearest pixel; a z-test keeps
 * the smallest (fp32 depth, source index).  Pixels with A < a_min move as
 * points at infinite depth (rotation only) and lose every z-test.
 * Outputs: rgb_dst/alpha_dst copied from the winning source pixel, z_dst
 * its destination depth (+inf for background), hole_mask 1 where no source
 * pixel landed (rgb 0, z +inf, alpha 0 there), depth_range[2] (device) =
 * min/max of D/A over covered source pixels (z_near/z_far if none).
 * Source and destination images may differ in size.  Asynchronous. */
BGS_API int32_t bgs_reproject(bgs_ctx* ctx, const bgs_camera* src, const bgs_camera* dst,
                              const bgs_roi_params* roi, const float* rgb_src, const float* depth_raw_src,
                              const float* alpha_src, void* ws, size_t ws_bytes, float* rgb_dst, float* z_dst,
                              float* alpha_dst, uint8_t* hole_mask, float* depth_range);

/* bgs_reproject for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, semantics and outputs as bgs_reproject,
 * without the workspace: its scratch (status words, the per-row partials
 * and, for rigs that do not keep rows, the 64-bit z-buffer) lives in a
 * static device array of BGS_REPROJECT_NOALLOC_SCRATCH_BYTES that each GPU
 * the library runs on holds until the process ends.  The destination image
 * may have at most BGS_REPROJECT_NOALLOC_MAX_PIXELS pixels
 * (BGS_ERR_INVALID_ARG beyond, nothing launched).  Every call on one GPU
 * uses that GPU's single array: calls that overlap in time on one GPU
 * (several streams or host threads) race and must be serialised by the
 * caller.  Each call clears what it accumulates, so consecutive calls of
 * any sizes are independent.  Calls no allocator.  Asynchronous. */
#define BGS_REPROJECT_NOALLOC_MAX_PIXELS (1 << 23)
#define BGS_REPROJECT_NOALLOC_SCRATCH_BYTES (512 + 16 * 16384 + 8 * (size_t)BGS_REPROJECT_NOALLOC_MAX_PIXELS)
BGS_API int32_t bgs_reproject_noalloc(bgs_ctx* ctx, const bgs_camera* src, const bgs_camera* dst,
                                      const bgs_roi_params* roi, const float* rgb_src, const float* depth_raw_src,
                                      const float* alpha_src, float* rgb_dst, float* z_dst, float* alpha_dst,
                                      uint8_t* hole_mask, float* depth_range);

/* Stage 3 and the interpolation part of Stage 4 (Sec. 3.1, Sec. 3.5).
 * Step 1: N samples per source-image edge reprojected at the two depths of
 * depth_range give the extrema of Eq. 6, border widths by Eq. 7-8
 * (clamped to half the image), then full-height/width strips aligned
 * outward to 16-pixel tiles.  Gaps: gap_passes Jacobi passes in which a
 * hole outside the edge ROIs with at least one non-hole 8-neighbour takes
 * their fp32 mean (fixed neighbour order) for RGB and alpha and their
 * largest depth.  Step 2 (center_roi = 1): remaining holes outside the edge
 * ROIs -> 8-connected components labelled by their smallest linear index
 * -> bounding box + margin -> clipped, tile-aligned center box; with
 * center_roi = 0 they copy the nearest non-hole pixel of their row (the
 * farther of the two sides, or bg when the row has none).
 *   rgb_dst, z_dst, alpha_dst   in/out warped image
 *   cls        in: hole mask from bgs_reproject; out: per-pixel class
 *   labels     out [H][W] int32, component label or -1
 *   boxes      out: edge boxes (left, right, top, bottom that exist), then
 *              center boxes in increasing label order, up to box_capacity
 *   n_boxes    out (device int32): total box count, even beyond capacity
 *   tile_mask  out [ceil(H/T)][ceil(W/T)] uint8 (T = roi->tile): 1 = the
 *              T x T tile touches a box
 * Asynchronous. */
BGS_API int32_t bgs_classify_holes(bgs_ctx* ctx, const bgs_camera* src, const bgs_camera* dst,
                                   const bgs_roi_params* roi, const bgs_raster_params* raster,
                                   const float* depth_range, void* ws, size_t ws_bytes, float* rgb_dst,
                                   float* z_dst, float* alpha_dst, uint8_t* cls, int32_t* labels, bgs_box* boxes,
                                   int32_t box_capacity, int32_t* n_boxes, uint8_t* tile_mask);

/* Stage 4 (Sec. 3.1): ROI-restricted re-rasterisation.  tile_mask is
 * [ceil(H/T)][ceil(W/T)] with T = roi->tile.  Only the 16x16 rasteriser
 * tiles that overlap a masked T-tile are binned, sorted and blended; every
 * pixel of a masked T-tile
 * is overwritten with the render at dst: rgb, alpha = A, z = D/A (or +inf
 * when A < a_min), cls = BGS_CLS_ROI.  Other pixels are untouched.
 * n_keys (host, optional) receives the number of ROI keys. */
BGS_API int32_t bgs_patch_rois(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* dst,
                               const bgs_raster_params* raster, const bgs_roi_params* roi,
                               const uint8_t* tile_mask, void* ws, size_t ws_bytes, float* rgb_dst, float* z_dst,
                               float* alpha_dst, uint8_t* cls, int64_t* n_keys);

/* The whole binocular frame (Sec. 3.1 Stages 1-4 in order): dominant
 * render -> reprojection -> classification and interpolation -> ROI patch.
 * Dominant outputs as bgs_render_dominant; affiliated outputs as
 * bgs_patch_rois after bgs_classify_holes.  stats (host, optional). */
BGS_API int32_t bgs_render_stereo(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam_dom,
                                  const bgs_camera* cam_aff, const bgs_raster_params* raster,
                                  const bgs_roi_params* roi, void* ws, size_t ws_bytes, float* rgb_dom,
                                  float* depth_raw_dom, float* alpha_dom, float* rgb_aff, float* z_aff,
                                  float* alpha_aff, uint8_t* cls_aff, int32_t* labels, bgs_box* boxes,
                                  int32_t box_capacity, int32_t* n_boxes, uint8_t* tile_mask, bgs_stats* stats);

/* ---- batched form ------------------------------------------------------ */

/* One stereo pair of a batch: its scene, cameras, ROI settings, its own
 * workspace (bgs_workspace_size for its scene and image size) and its
 * outputs, laid out as for bgs_render_stereo. */
typedef struct bgs_batch_pair {
    const bgs_scene* scene; /* host pointer to a scene description (arrays on the device) */
    bgs_camera cam_dom, cam_aff;
    bgs_roi_params roi;
    int32_t box_capacity;
    void* ws;
    size_t ws_bytes;
    float *rgb_dom, *depth_raw_dom, *alpha_dom;
    float *rgb_aff, *z_aff, *alpha_aff;
    uint8_t* cls_aff;
    int32_t* labels;
    bgs_box* boxes;
    int32_t* n_boxes;
    uint8_t* tile_mask;
} bgs_batch_pair;

/* Bytes of the batch workspace for n_pairs pairs (descriptors and queue). */
BGS_API int32_t bgs_batch_workspace_size(int32_t n_pairs, size_t* bytes);

/* Many stereo frames in one call (Sec. 3.1 Stages 1-4 for each pair, with
 * the same results as bgs_render_stereo given the same settings, except
 * that long tile lists are never split into continuation segments).  Every
 * pair's binning runs in turn, then ONE persistent blend launch renders the
 * dominant-eye tiles of all pairs from a shared (pair, tile) work queue;
 * then every pair's reprojection, classification and ROI binning, and one
 * persistent launch for all ROI tiles.  Scenes and image sizes may differ
 * between pairs.  Asynchronous: each pair's key count and overflow flags are
 * read with bgs_poll_status on its workspace.  n_pairs in [1, 4096]. */
BGS_API int32_t bgs_render_stereo_batch(bgs_ctx* ctx, int32_t n_pairs, const bgs_batch_pair* pairs,
                                        const bgs_raster_params* raster, void* batch_ws, size_t batch_ws_bytes);

/* The batch captured once into a HIP graph and replayed: capture records
 * every launch of bgs_render_stereo_batch on the context's stream (which
 * must not be the null stream; stage timing must be off) without running
 * them; bgs_graph_launch replays them on the context's stream, with the
 * pairs, cameras and buffers of the capture. */
typedef struct bgs_graph bgs_graph;
BGS_API int32_t bgs_batch_graph_capture(bgs_ctx* ctx, int32_t n_pairs, const bgs_batch_pair* pairs,
                                        const bgs_raster_params* raster, void* batch_ws, size_t batch_ws_bytes,
                                        bgs_graph** graph);
BGS_API int32_t bgs_graph_launch(bgs_ctx* ctx, bgs_graph* graph);
BGS_API int32_t bgs_graph_destroy(bgs_graph* graph);

/* ---- stage-level exports used by the parity tests ---------------------- */

/* Stable LSD radix sort of (key, value) pairs by the low key_bits bits of
 * the keys (1..32), in place.  Workspace: bgs_sort_workspace_size(n). */
BGS_API int32_t bgs_sort_workspace_size(int64_t n, size_t* bytes);
BGS_API int32_t bgs_sort_pairs(bgs_ctx* ctx, uint32_t* keys, uint32_t* values, int64_t n, int32_t key_bits,
                               void* ws, size_t ws_bytes);

/* Connected components of a uint8 mask (nonzero = set) with 8- (conn = 8)
 * or 4-connectivity (conn = 4); labels[p] = smallest linear index of p's
 * component, -1 off the mask.  Asynchronous. */
BGS_API int32_t bgs_label_components(bgs_ctx* ctx, const uint8_t* mask, int32_t width, int32_t height,
                                     int32_t conn, int32_t* labels);

/* Per-surfel binning data of Stage 1 for one camera: zkey[n] = bits of the
 * fp32 centre depth (the compositing order key; 0xFFFFFFFF when culled),
 * rects[n][4] = inclusive tile rectangle (tx0, ty0, tx1, ty1), or -1s when
 * the surfel touches no tile, counts[n] = tiles in the rectangle. */
BGS_API int32_t bgs_preprocess_debug(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam,
                                     const bgs_raster_params* raster, void* ws, size_t ws_bytes, uint32_t* zkey,
                                     int32_t* rects, uint32_t* counts);

/* Per-tile trace of the last dominant-eye blend run with pair counting on
 * (bgs_ctx_set_count_pairs): for each launched block, 6 int64 {tile, list
 * length, most records one wave evaluated, CU id, start, end (wall
 * clock, 100 MHz)}.
 * n, width, height are those the workspace was laid out for.  Waits for
 * the stream.  Measurement only. */
BGS_API int32_t bgs_blend_trace(bgs_ctx* ctx, int64_t n, int32_t width, int32_t height, void* ws, size_t ws_bytes,
                                int64_t* out);

/* Binned and sorted tile lists of Stage 1: ranges[n_tiles][2] = [start,
 * end) into values, values[key_capacity] = surfel indices in compositing
 * order within each tile.  n_keys (host) receives the key count. */
BGS_API int32_t bgs_tile_lists_debug(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam,
                                     const bgs_raster_params* raster, void* ws, size_t ws_bytes, uint32_t* ranges,
                                     uint32_t* values, int64_t values_capacity, int64_t* n_keys);

#ifdef __cplusplus
}
#endif

#endif /* BGS_H */
