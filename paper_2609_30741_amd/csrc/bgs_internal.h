// Internal declarations of the HIP library behind include/bgs.h.
// gfx950 (CDNA4): wave64, 160 KiB LDS per CU, 256 CUs in 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "bgs.h"

namespace bgs {

constexpr int kTile = 16;            // rasteriser tile edge (pixels)
constexpr int kScanItems = 8;        // elements per thread in a scan block
constexpr int kScanBlock = 256 * kScanItems;    // 2048 elements per block

// Per-surfel record written by the preprocess and staged through LDS by the
// blend kernel.  64 bytes.
//   a = (mu_x, mu_y, C1, C2)    projected centre; u numerator coefficients
//   b = (D1, D2, N1, N2)        v numerator; common denominator
//   c = (lam_num, z_c, opacity, band direction)
//   d = (r, g, b, band interval)
// With dx = i - mu_x, dy = j - mu_y and den = 1 + N1 dx + N2 dy the
// surfel-plane coordinates of pixel (i, j), times sqrt(1/2), are
// u = (C1 dx + C2 dy)/den, v = (D1 dx + D2 dy)/den and the ray meets the
// plane at depth
// lam_num/den (lam_num < 0 marks a surfel seen exactly edge-on).  The
// strip band bounds every pixel x the surfel can reach by
// |n.(x - mu) - c| <= w, with n a pair of snorm16 (x low, y high) and c, w
// a pair of fp16 (c low, w high).
struct alignas(16) SurfelRec {
    float4 a, b, c, d;
};

// Camera constants for the preprocess (fp64 geometry).
struct PreCam {
    double Rt[9];  // world-to-camera rotation R^T, row-major
    double t[3];   // camera centre
    double fx, fy, cx, cy;
    double z_near;
    float zc[4];   // fp32 centre-depth key coefficients (r20, r21, r22, tz)
    int W, H, tiles_x, tiles_y;
};

struct SceneArgs {
    const float* pos;
    const float* quat;
    const float* scale;
    const float* opacity;
    const float* sh;
    int n;
    int sh_degree;
};

// Optional ROI restriction of the binning: only tiles with mask = 1 are
// emitted, under compact ids (row-major rank among masked tiles).
// prefix[t] = number of masked tiles before tile t in row-major order
// (n_tiles + 1 entries), so a tile's compact id is prefix[t] and the masked
// tiles of row ty in columns [a, b] number prefix[ty*tx+b+1] - prefix[ty*tx+a].
struct MaskArgs {
    const uint32_t* prefix;  // masked tiles before each tile (n_tiles + 1)
    const uint32_t* colcum;  // column sums of prefix over rows (tiles_y x (tiles_x + 1))
    int tiles_x;
    int enabled;
};

struct BlendArgs {
    int W, H, tiles_x;
    float alpha_min, alpha_max, t_min;
    int lowpass;
    float bg0, bg1, bg2;
    float a_min;     // patch mode: depth proxy written only when A >= a_min
    float z_near;
    int patch;       // 0: write rgb/depth_raw/alpha; 1: write rgb/z/alpha/cls
    uint32_t vmask;  // surfel index = sorted value & vmask (values that also carry the tile key)
    // ROI patch with 8-pixel ROI tiles: the 8x8 ROI tile mask (qmask_w tiles
    // per row); an 8x8 quadrant of a 16x16 tile that it leaves out is neither
    // composited nor written.  Null otherwise.
    const uint8_t* qmask;
    int qmask_w;
    // View-colour transfer (dominant eye of a stereo frame only; an option
    // outside the paper's method): xrecs are the records of the affiliated
    // eye, whose last float4 holds each surfel's colour seen from that eye;
    // the blend composites them with the dominant eye's weights into
    // xrgb[3][H][W] (plus T bg).  Null otherwise.
    const SurfelRec* xrecs;
    float* xrgb;
};

// Continuation of long tile lists in the blend (k_blend, k_blend_seg,
// k_blend_chain, k_blend_fix in raster.hip).  All arrays live in the
// workspace.  A continued tile takes a slot and a run of consecutive items,
// one per segment of its remaining records.
struct ContArgs {
    uint32_t cap;          // records a tile composites before its rest is continued; 0: never
    uint32_t seg_len;      // records per continuation segment (at most kContMaxSeg segments)
    uint32_t max_slots;    // tiles that may be continued per pass
    uint32_t min_far;      // continue a tile only if some pixel is expected to composite this many more records
    uint32_t* n_slots;     // counters (DevStatus), cleared before each pass
    uint32_t* n_items;
    uint4* slot_desc;      // per slot: compact tile id, first continued record, end record, item base | nseg << kContSegShift
    uint32_t* item_slot;   // per item: its slot
    float4* st1;           // per slot: 256 pixels x 2 float4 after the capped walk
    float4* part;          // per item: 256 pixels x 2 float4, the segment's walk from the slot's transmittance
};
constexpr uint32_t kContMaxSeg = 32;
constexpr uint32_t kContSegShift = 26;  // item base in the low 26 bits, segment count above


// Device status block kept in the workspace.
struct DevStatus {
    uint32_t n_keys;       // keys of the last binning (may exceed capacity)
    uint32_t n_sort;       // min(n_keys, capacity): keys actually sorted
    uint32_t n_masked;     // masked tiles of the last ROI patch
    uint32_t n_keys_dom;
    uint32_t n_keys_roi;
    uint32_t overflow;     // bit 0 key capacity, bit 1 box capacity
    uint32_t n_holes, n_gap, n_center, n_rowfill, n_boxes, n_roi_tiles, n_edge;
    // Overflow bits of every earlier frame since the last bgs_poll_status:
    // the per-frame reset folds the previous frame's overflow into it, and
    // only the poll clears it.
    uint32_t sticky;
    // Depth-range reduction over positive fp32 bits: the complement of the
    // minimum (so that a zeroed block means "none yet") and the maximum.
    uint32_t dmin_inv, dmax_bits;
    uint32_t pad2[2];
    uint32_t n_slots, n_items;  // blend continuation of the current pass
    // Counting mode only, dominant then ROI pass, 6 each: evaluated pairs,
    // contributing pairs, records walked (summed over waves), records past
    // the strip test (summed over waves), longest walk of one wave, longest
    // tile list.
    unsigned long long pairs[12];
    int32_t edge_boxes[4 * 6];
    int32_t widths[4];
};

// ---- status and fills (sort.hip) --------------------------------------------
// Start-of-frame reset of the status block by a kernel (no memset node, so a
// frame can be captured in a graph): full = 1 zeroes every word; full = 0
// keeps the sticky overflow word and ORs the previous frame's overflow bits
// into it.
hipError_t launch_status_reset(DevStatus* st, int full, hipStream_t s);
// dst[i] = value for i < n, by a kernel.
hipError_t launch_fill_u32(uint32_t* dst, int64_t n, uint32_t value, hipStream_t s);

// ---- scan / sort (sort.hip) -------------------------------------------------
size_t scan_tmp_elems(int64_t n);
// out[i] = sum_{j < i} in[idx ? idx[j] : j] for i = 0..n, with n = *n_dev when
// n_dev is given (at most n_cap), else n_cap.  Elements past n count as 0.
hipError_t exclusive_scan(const uint32_t* in, const uint32_t* idx, uint32_t* out, const uint32_t* n_dev,
                          int64_t n_cap, uint32_t* tmp, hipStream_t s);
// Key count of a binning pass, recorded in the status block by the scan of
// the per-surfel key counts (which: 0 dominant, 1 ROI; cap: key capacity).
// It also clears the blend-continuation counters of the pass.
struct KeyCount {
    DevStatus* st;
    uint32_t cap;
    int which;
    uint2* ranges;     // tile ranges to clear to empty (n_tiles of them)
    uint32_t n_tiles;
};
// Exclusive scan of n per-surfel counts (gathered through idx) into out[0..n]
// with the key count recorded, in two launches.  Returns false, launching
// nothing, when n is beyond its size limit (use exclusive_scan and
// launch_status_keys then); *err gets the launch status otherwise.
bool scan_counts(const uint32_t* in, const uint32_t* idx, uint32_t* out, int64_t n, uint32_t* tmp,
                 const KeyCount& kcnt, hipStream_t s, hipError_t* err);
// scan_counts' down-sweep alone, over counts in order whose totals per 256
// consecutive elements are already in partials; false when n needs more
// than the flat form's blocks.
bool scan_counts_presummed(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* partials,
                           const KeyCount& kcnt, hipStream_t s, hipError_t* err);
// Whether the flat, two-launch scan covers n elements.
bool scan_is_flat(int64_t n);
size_t radix_tmp_bytes(int64_t n_cap);
// Stable LSD radix sort of (keys, values) by bits [key_shift, key_shift +
// key_bits) of the keys, with digits of up to 8 bits.  (ka, va) is the
// input, (kb, vb) the ping-pong buffer; iota = true ignores the input
// values and uses the input positions instead; va = vb = null (and iota
// false) sorts the keys alone (keys that carry their value in the bits
// below key_shift).  The element count is *n_dev (<= n_cap), or n_cap when
// n_dev is null.
// Returns in *in_b whether the result is in (kb, vb).  n_hint (optional):
// the expected element count when it is far below n_cap, or -1 when only
// the device knows it (both kernel forms are then launched, each gated on
// *n_dev); it only chooses the kernels' sub-chunk size, never the result.
hipError_t radix_sort(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, const uint32_t* n_dev,
                      int64_t n_cap, int key_bits, bool iota, void* tmp, hipStream_t s, bool* in_b,
                      int64_t n_hint = 0, int key_shift = 0);

// ---- rasteriser (raster.hip) --------------------------------------------------
// cam2 (optional): also the keys, rects and records of a second camera (no
// key counts: see launch_masked_counts).  nseg (optional, per surfel): the
// rows of the surfel's band that hold keys, which the emission lists.
hipError_t launch_preprocess(const SceneArgs& sc, const PreCam& cam, float alpha_min, int lowpass,
                             const MaskArgs& mask, SurfelRec* recs, uint32_t* zkeys, uint2* rects,
                             uint32_t* counts, const PreCam* cam2, SurfelRec* recs2, uint32_t* zkeys2,
                             uint2* rects2, uint32_t* nseg, hipStream_t s);
// Key counts within the mask's tiles from precomputed tile rects and records,
// and the rows that hold them (nseg), per surfel.
hipError_t launch_masked_counts(const uint2* rects, const SurfelRec* recs, int n, int n_tiles, const MaskArgs& mask,
                                uint32_t* counts, uint32_t* nseg, hipStream_t s);
// The same counts in compositing order (counts[i] and nseg[i] for surfel
// order[i]), with the total of every 256 consecutive positions in partials
// (ceil(n / 256) of them): the scan then needs only its down-sweep
// (scan_counts_presummed).
hipError_t launch_masked_counts_ordered(const uint2* rects, const SurfelRec* recs, const uint32_t* order, int n,
                                        int n_tiles, const MaskArgs& mask, uint32_t* counts, uint32_t* partials,
                                        uint32_t* nseg, hipStream_t s);
// Keys of every surfel in compositing order: the tiles of its rect that its
// strip band meets (and the mask holds, when enabled), row by row.
// vbits > 0: one word per key, tile << vbits | surfel (tvals unused);
// vbits = 0: the tile in tkeys and the surfel in tvals.
// nseg (optional): each surfel's rows with keys as its counting pass left
// them, indexed by position in the order (nseg_by_pos) or by surfel; null:
// the emission counts them itself.
hipError_t launch_emit(const uint32_t* order, const uint32_t* offs, const uint2* rects, const SurfelRec* recs, int n,
                       int tiles_x, int n_tiles, const MaskArgs& mask, uint32_t cap, int vbits, uint32_t* tkeys,
                       uint32_t* tvals, const uint32_t* nseg, int nseg_by_pos, hipStream_t s);
// Tile ranges of the sorted keys (tile = key >> key_shift); the ranges must
// have been cleared (by scan_counts, or launch_clear_ranges).
hipError_t launch_ranges(const uint32_t* tkeys, const uint32_t* n_dev, int64_t cap, uint2* ranges,
                         int n_tiles, int key_shift, hipStream_t s);
// dst[i] = src[i] & mask for i < n.
hipError_t launch_mask_copy(const uint32_t* src, uint32_t* dst, int64_t n, uint32_t mask, hipStream_t s);
hipError_t launch_clear_ranges(uint2* ranges, int n_tiles, hipStream_t s);
// Dispatch order of the (compact) tiles for the blend, heaviest first.
hipError_t launch_tile_order(const uint2* ranges, const uint32_t* n_live, int n_tiles, uint32_t* order,
                             hipStream_t s);
// One block per (compact) tile, in `order`; n_live (device, optional) limits
// the blocks that do work when the tile count is only known on the device.
// pair_counts (optional): the six blend counters of DevStatus::pairs.
hipError_t launch_blend(const SurfelRec* recs, const uint32_t* vals, const uint2* ranges,
                        const uint32_t* tile_list, const uint32_t* order, const uint32_t* n_live, int n_blocks,
                        const BlendArgs& a, const ContArgs& ca, float* rgb, float* d_or_z, float* alpha, uint8_t* cls,
                        unsigned long long* pair_counts, long long* trace, hipStream_t s);
// One frame's blend of a batch (one eye of one stereo pair), in device
// memory: a persistent launch renders the tiles of every frame of the batch
// from a shared work queue.
struct BatchBlendDesc {
    const SurfelRec* recs;
    const uint32_t* vals;
    const uint2* ranges;
    const uint32_t* tile_list;  // compact id -> tile id (masked passes); null: identity
    const uint32_t* order;      // dispatch order of the compact tiles, heaviest first
    const uint32_t* n_live;     // live compact tiles (masked passes); null: n_tiles
    uint32_t n_tiles;
    uint32_t reserved;
    BlendArgs a;
    float* rgb;
    float* dz;
    float* alpha;
    uint8_t* cls;
};
// Copy a descriptor (a kernel argument) into device memory.
hipError_t launch_put_desc(const BatchBlendDesc& d, BatchBlendDesc* dst, hipStream_t s);
// Blend every tile of n frames: item prefix over the frames, then one
// persistent launch of `grid` workgroups that take (frame, tile) items from
// a queue counter in turn until all are done (no waits between workgroups).
// scratch: n + 2 words (prefix and counter).  patch: the frames are ROI
// passes (the patch writes).
hipError_t launch_blend_batch(const BatchBlendDesc* descs, int n, uint32_t* scratch, int grid, bool patch,
                              hipStream_t s);

// Tables of an ROI tile mask (n_tiles = tiles_x * tiles_y): prefix[n_tiles +
// 1], the compact list of masked tile ids, the masked count in DevStatus, and
// colcum[tiles_y][tiles_x + 1], the column sums of prefix over rows.
// The 16x16 rasteriser-tile mask of an ROI tile mask with T x T tiles (T =
// 8 or 32) for a W x H image: a 16-tile is set iff it overlaps a set T-tile.
hipError_t launch_mask_to16(const uint8_t* tmask, int T, int W, int H, uint8_t* mask16, hipStream_t s);
hipError_t launch_mask_tables(const uint8_t* tile_mask, int n_tiles, int tiles_x, uint32_t* prefix,
                              uint32_t* tile_list, uint32_t* colcum, DevStatus* st, hipStream_t s);
// Record the key count offs[n] of a binning (which: 0 dominant, 1 ROI).
hipError_t launch_status_keys(const uint32_t* offs, int n, DevStatus* st, uint32_t cap, int which,
                              hipStream_t s);

// ---- reprojection and classification (warp.hip, no fp contraction) -------
struct WarpCam {
    int W, H;
    double fx, fy, cx, cy, z_near, z_far;
};
struct RelPose {
    double M[9], c[3];
};
RelPose rel_pose(const bgs_camera& src, const bgs_camera& dst);

// Per-block partials the reprojection leaves in wpart (row-preserving form:
// one per row; the scatter form reduces with atomics and leaves none).
int warp_parts(const WarpCam& src, const WarpCam& dst, const RelPose& P);
// reset: clear the status fields the reprojection and classification
// accumulate (not needed when the whole status block was zeroed);
// depth_range (optional): fold the partials into the status block and
// write the covered depth-proxy range there; without it the classification
// that follows folds them.
hipError_t launch_reproject(const WarpCam& src, const WarpCam& dst, const RelPose& P, float a_min,
                            const float* rgb, const float* draw, const float* alpha, unsigned long long* zbuf,
                            float* rgb_dst, float* z_dst, float* alpha_dst, uint8_t* hole, float* depth_range,
                            bool reset, uint4* wpart, DevStatus* st, hipStream_t s);
struct ClassifyBufs {
    uint8_t* hole;     // interpolation tags
    uint8_t* hole2;    // center-hole mask
    uint32_t* bcount;  // component roots per 256-pixel block, then their exclusive scan
    uint32_t* rmask;   // per 256-pixel block: bit mask of its component roots (8 words)
    int32_t* bbox;     // per component: box (4) and root pixel (1), 8 words
    uint8_t* pflag;    // block-local piece roots
    int4* pbox;        // piece boxes, indexed by root pixel
    uint4* wpart;      // reprojection partials (warp_parts entries)
    uint2* gpart;      // gap-fill partials, one per gap-fill block
};
// depth_range null: take the range from the reprojection just run (its
// partials in b.wpart and its status fields).
hipError_t launch_classify(const WarpCam& src, const WarpCam& dst, const RelPose& P, const bgs_roi_params& roi,
                           const float bg[3], const float* depth_range, float* rgb, float* z, float* alpha,
                           uint8_t* cls, int32_t* labels, bgs_box* boxes, int32_t box_cap, int32_t* n_boxes,
                           uint8_t* tile_mask, const ClassifyBufs& b, DevStatus* st, hipStream_t s);
hipError_t launch_label_components(const uint8_t* mask, int W, int H, int conn, int32_t* labels,
                                   hipStream_t s);

}  // namespace bgs
