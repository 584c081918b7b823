// C ABI of the binocular 2DGS frame path: argument validation, workspace
// layout and the order of the stages on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bgs_internal.h"

// Scratch of bgs_reproject_noalloc: one copy per GPU, allocated with the
// code object and held until the process ends.  Layout: the status block
// (512 bytes), one uint4 partial per destination row (16384 rows at most),
// then the 64-bit z-buffer.  In host code this name is only a stand-in for
// the symbol; its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[BGS_REPROJECT_NOALLOC_SCRATCH_BYTES];

struct bgs_ctx {
    hipStream_t stream = nullptr;
    int sync = 1;
    int count_pairs = 0;
    uint32_t timing = 0;  // bit i: time stage i
    // Blend continuation: records a tile composites before the rest of its
    // list is split into segments (0: never), per pass, and the segment length.
    uint32_t cap_dom = 1024, cap_roi = 32, seg_len = 32, far_dom = 0, far_roi = 256;
    // Stage timing: a ring of event pairs, one set per frame, so frames can
    // be issued back to back; a set is folded into the totals when the ring
    // comes round to it again (its frame is long done by then) or on collect.
    static constexpr int kRing = 64;
    hipEvent_t ev[kRing][BGS_NUM_STAGES][2] = {};
    bool pending[kRing][BGS_NUM_STAGES] = {};
    int slot = 0;
    hipError_t timing_err = hipSuccess;  // first failure of an event call while timing, reported on collect
    double total_ms[BGS_NUM_STAGES] = {};
    int64_t count[BGS_NUM_STAGES] = {};
    std::string err;
    // The workspace whose status block this context last reset: a new one is
    // zeroed completely (its sticky overflow word included) before first use.
    const void* ws_seen = nullptr;
    // The same for the per-pair workspaces of batched frames.
    std::vector<const void*> batch_seen;
    int n_cu = 0;  // compute units of the device (persistent launches), looked up once
};

// A captured batch: the graph and its executable instance.
struct bgs_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace bgs {
namespace {

constexpr size_t kAlign = 256;
// Tiles per pass whose list tail may be continued by segment workgroups.
constexpr int64_t kContSlots = 512;
// Long tile lists are continued by segment workgroups only on images of at
// most this many 16x16 tiles: on larger ones the tiles of a pass already
// fill the GPU, and the four continuation launches would run (nearly)
// empty.  800x600 (1900 tiles): continuation saves 54 us in the ROI pass;
// 1600x1064 (6700 tiles): without it both passes are 18-20 us shorter.
constexpr int kSplitMaxTiles = 4096;

inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout.  Regions that depend only on the image size come first
// so that stage calls, which do not know the scene size, find them at the
// same offsets; the surfel region follows, then the tile keys, whose count
// is whatever the remaining bytes hold.
struct Layout {
    size_t status;
    size_t zbuf, hole, hole2, bcount, rmask, bbox, pflag, pbox, wpart, gpart;
    size_t ranges, colcum, mprefix, tlist, torder, mask16;
    size_t xrgb;  // view-colour transfer: the dominant pass's affiliated-view colours [3][H][W]
    size_t recs, zkeys, rects, counts, nseg, dkeys_b, dvals_a, dvals_b, offs, surf_scan;
    size_t recs2, zkeys2, rects2;  // the affiliated eye's surfels, from the dominant pass of a stereo frame
    size_t tkeys_a, tkeys_b, tvals_a, tvals_b;
    size_t radix;
    size_t trace;  // per-tile blend trace of the last counting-mode dominant pass
    size_t cdesc, citem, cst1, cpart;  // blend continuation
    uint32_t cslots;
    size_t total;
};

Layout make_layout(int64_t n, int64_t W, int64_t H, int64_t kc) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += up(bytes);
        return at;
    };
    const int64_t np = W * H;
    const int64_t nt = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    L.status = take(sizeof(DevStatus));
    L.zbuf = take(8 * np);
    L.hole = take(np);
    L.hole2 = take(np);
    const int64_t nb = (np + 255) / 256;  // 256-pixel blocks of the component labelling
    L.bcount = take(4 * (nb + 1));
    L.rmask = take(32 * nb);
    L.bbox = take(16 * np);  // 8 words per component; at most np / 2 components
    L.pflag = take(np);
    L.pbox = take(16 * np);
    L.wpart = take(16 * H);                                   // one per row
    L.gpart = take(8 * ((W + 63) / 64) * ((H + 15) / 16));   // one per gap-fill block
    L.ranges = take(8 * nt);
    L.colcum = take(4 * (nt + (H + kTile - 1) / kTile));
    L.mprefix = take(4 * (nt + 1));
    L.tlist = take(4 * nt);
    L.torder = take(4 * nt);
    L.mask16 = take(nt);  // rasteriser-tile mask of an ROI mask with 8- or 32-pixel tiles
    L.xrgb = take(12 * np);
    L.recs = take(sizeof(SurfelRec) * n);
    L.zkeys = take(4 * n);
    L.rects = take(8 * n);
    L.counts = take(4 * n);
    L.nseg = take(4 * n);
    L.dkeys_b = take(4 * n);
    L.dvals_a = take(4 * n);
    L.dvals_b = take(4 * n);
    L.offs = take(4 * (n + 1));
    // Scan scratch: the count scan's block sums, or the per-256 totals of the
    // ROI pass's ordered counts (ceil(n / 256) words), whichever is larger.
    L.surf_scan = take(4 * std::max<size_t>(scan_tmp_elems(n), (size_t)((n + 255) / 256) + 64));
    L.recs2 = take(sizeof(SurfelRec) * n);
    L.zkeys2 = take(4 * n);
    L.rects2 = take(8 * n);
    L.tkeys_a = take(4 * kc);
    L.tkeys_b = take(4 * kc);
    L.tvals_a = take(4 * kc);
    L.tvals_b = take(4 * kc);
    L.radix = take(radix_tmp_bytes(kc > n ? kc : n));
    L.trace = take(6 * 8 * nt);
    L.cslots = (uint32_t)(nt < kContSlots ? nt : kContSlots);
    L.cdesc = take(16 * (size_t)L.cslots);
    L.citem = take(4 * (size_t)L.cslots * kContMaxSeg);
    L.cst1 = take(8192 * (size_t)L.cslots);
    L.cpart = take(8192 * (size_t)L.cslots * kContMaxSeg);
    L.total = o;
    return L;
}

// Largest key capacity whose layout fits in `bytes` (-1 if none does).
int64_t key_capacity_for(int64_t n, int64_t W, int64_t H, size_t bytes) {
    if (make_layout(n, W, H, 0).total > bytes) return -1;
    int64_t lo = 0, hi = 1;
    while (hi < (int64_t)0xFFFFFFF0 && make_layout(n, W, H, hi).total <= bytes) hi *= 2;
    if (hi > (int64_t)0xFFFFFFF0) hi = 0xFFFFFFF0;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (make_layout(n, W, H, mid).total <= bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

int fail(bgs_ctx* ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(bgs_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

int hip_fail(bgs_ctx* ctx, hipError_t e, const char* where) {
    return fail(ctx, BGS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_CHECK(expr, where)                        \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

int check_camera(bgs_ctx* ctx, const bgs_camera* c, const char* name) {
    if (!c) return fail(ctx, BGS_ERR_INVALID_ARG, "%s: null camera", name);
    if (c->width < 1 || c->width > 16384 || c->height < 1 || c->height > 16384)
        return fail(ctx, BGS_ERR_INVALID_ARG, "%s: image size %dx%d outside [1, 16384]", name, c->width, c->height);
    if (!(c->fx > 0.0) || !(c->fy > 0.0) || !std::isfinite(c->fx) || !std::isfinite(c->fy))
        return fail(ctx, BGS_ERR_INVALID_ARG, "%s: focal lengths must be positive", name);
    if (!std::isfinite(c->cx) || !std::isfinite(c->cy))
        return fail(ctx, BGS_ERR_INVALID_ARG, "%s: principal point must be finite", name);
    if (!(c->z_near > 0.0) || !(c->z_far > c->z_near))
        return fail(ctx, BGS_ERR_INVALID_ARG, "%s: need 0 < z_near < z_far", name);
    for (int i = 0; i < 3; ++i) {
        if (!std::isfinite(c->t[i])) return fail(ctx, BGS_ERR_INVALID_ARG, "%s: camera centre not finite", name);
        for (int j = 0; j < 3; ++j) {
            double d = 0.0;
            for (int k = 0; k < 3; ++k) d += c->R[k * 3 + i] * c->R[k * 3 + j];
            if (!(std::fabs(d - (i == j ? 1.0 : 0.0)) <= 1e-6))
                return fail(ctx, BGS_ERR_INVALID_ARG, "%s: R is not orthonormal", name);
        }
    }
    return BGS_OK;
}

int check_scene(bgs_ctx* ctx, const bgs_scene* s) {
    if (!s) return fail(ctx, BGS_ERR_INVALID_ARG, "null scene");
    if (s->n < 0 || s->n >= ((int64_t)1 << 31)) return fail(ctx, BGS_ERR_INVALID_ARG, "scene size %lld out of range", (long long)s->n);
    if (s->sh_degree < 0 || s->sh_degree > 3)
        return fail(ctx, BGS_ERR_INVALID_ARG, "sh_degree %d outside 0..3", s->sh_degree);
    if (s->n > 0 && (!s->pos || !s->quat || !s->scale || !s->opacity || !s->sh))
        return fail(ctx, BGS_ERR_INVALID_ARG, "null scene array");
    return BGS_OK;
}

int check_raster(bgs_ctx* ctx, const bgs_raster_params* r) {
    if (!r) return fail(ctx, BGS_ERR_INVALID_ARG, "null raster params");
    if (!(r->alpha_min > 0.f && r->alpha_min < 1.f) || !(r->alpha_max > r->alpha_min && r->alpha_max <= 1.f) ||
        !(r->t_min > 0.f && r->t_min < 1.f))
        return fail(ctx, BGS_ERR_INVALID_ARG, "raster thresholds out of range");
    return BGS_OK;
}

int check_roi(bgs_ctx* ctx, const bgs_roi_params* r) {
    if (!r) return fail(ctx, BGS_ERR_INVALID_ARG, "null roi params");
    if (r->tile != 8 && r->tile != 16 && r->tile != 32)
        return fail(ctx, BGS_ERR_UNSUPPORTED, "ROI tile %d unsupported (8, 16 or 32)", r->tile);
    if (r->margin < 0 || r->margin > 16384) return fail(ctx, BGS_ERR_INVALID_ARG, "margin %d out of range", r->margin);
    if (r->edge_samples < 1 || r->edge_samples > 65536)
        return fail(ctx, BGS_ERR_INVALID_ARG, "edge_samples %d out of range", r->edge_samples);
    if (r->gap_passes < 0 || r->gap_passes > 64)
        return fail(ctx, BGS_ERR_INVALID_ARG, "gap_passes %d out of range", r->gap_passes);
    if (!(r->a_min > 0.f && r->a_min <= 1.f)) return fail(ctx, BGS_ERR_INVALID_ARG, "a_min out of (0, 1]");
    if (r->edge_bounds != 0 && r->edge_bounds != 1)
        return fail(ctx, BGS_ERR_INVALID_ARG, "edge_bounds %d is neither 0 nor 1", r->edge_bounds);
    if (r->view_colour != 0 && r->view_colour != 1)
        return fail(ctx, BGS_ERR_INVALID_ARG, "view_colour %d is neither 0 nor 1", r->view_colour);
    return BGS_OK;
}

PreCam make_precam(const bgs_camera& c) {
    PreCam p{};
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) p.Rt[r * 3 + q] = c.R[q * 3 + r];
    for (int i = 0; i < 3; ++i) p.t[i] = c.t[i];
    p.fx = c.fx;
    p.fy = c.fy;
    p.cx = c.cx;
    p.cy = c.cy;
    p.z_near = c.z_near;
    // Centre-depth key coefficients: row 2 of R^T and -(R^T t)_2, in fp64
    // with a fixed summation order, then rounded to fp32.
    const double r20 = c.R[0 * 3 + 2], r21 = c.R[1 * 3 + 2], r22 = c.R[2 * 3 + 2];
    const double tz = -(((r20 * c.t[0]) + (r21 * c.t[1])) + (r22 * c.t[2]));
    p.zc[0] = (float)r20;
    p.zc[1] = (float)r21;
    p.zc[2] = (float)r22;
    p.zc[3] = (float)tz;
    p.W = c.width;
    p.H = c.height;
    p.tiles_x = (c.width + kTile - 1) / kTile;
    p.tiles_y = (c.height + kTile - 1) / kTile;
    return p;
}

WarpCam make_warpcam(const bgs_camera& c) {
    WarpCam w;
    w.W = c.width;
    w.H = c.height;
    w.fx = c.fx;
    w.fy = c.fy;
    w.cx = c.cx;
    w.cy = c.cy;
    w.z_near = c.z_near;
    w.z_far = c.z_far;
    return w;
}

int tile_bits(int64_t n_tiles) {
    int b = 1;
    while (((int64_t)1 << b) < n_tiles) ++b;
    return b;
}

// Records the start (end = 0) or end (end = 1) of a stage when timing is on.
// Fold one ring slot's finished stages into the totals.
hipError_t drain_slot(bgs_ctx* ctx, int r) {
    for (int i = 0; i < BGS_NUM_STAGES; ++i) {
        if (!ctx->pending[r][i]) continue;
        hipError_t e = hipEventSynchronize(ctx->ev[r][i][1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev[r][i][0], ctx->ev[r][i][1]);
        if (e != hipSuccess) return e;
        ctx->total_ms[i] += ms;
        ctx->count[i] += 1;
        ctx->pending[r][i] = false;
    }
    return hipSuccess;
}

// Record a stage boundary.  A stage started again in the same slot begins
// a new frame: move to the next slot, folding in what it still holds.
void mark(bgs_ctx* ctx, int stage, int end) {
    if (!((ctx->timing >> stage) & 1u)) return;
    if (!end && ctx->pending[ctx->slot][stage]) {
        ctx->slot = (ctx->slot + 1) % bgs_ctx::kRing;
        const hipError_t e = drain_slot(ctx, ctx->slot);
        if (e != hipSuccess && ctx->timing_err == hipSuccess) ctx->timing_err = e;
    }
    const hipError_t e = hipEventRecord(ctx->ev[ctx->slot][stage][end], ctx->stream);
    if (e != hipSuccess) {
        // Leave the stage out of this frame rather than time an unrecorded event.
        if (ctx->timing_err == hipSuccess) ctx->timing_err = e;
        ctx->pending[ctx->slot][stage] = false;
        return;
    }
    if (end) ctx->pending[ctx->slot][stage] = true;
}

void fill_stats(const DevStatus& h, bgs_stats* s) {
    s->n_keys_dom = h.n_keys_dom;
    s->n_keys_roi = h.n_keys_roi;
    s->n_holes = (int32_t)h.n_holes;
    s->n_gap = (int32_t)h.n_gap;
    s->n_center = (int32_t)h.n_center;
    s->n_rowfill = (int32_t)h.n_rowfill;
    s->n_boxes = (int32_t)h.n_boxes;
    s->n_roi_tiles = (int32_t)h.n_roi_tiles;
    s->overflow = (int32_t)h.overflow;
    s->reserved = 0;
    s->pairs_eval_dom = (int64_t)h.pairs[0];
    s->pairs_used_dom = (int64_t)h.pairs[1];
    s->pairs_eval_roi = (int64_t)h.pairs[6];
    s->pairs_used_roi = (int64_t)h.pairs[7];
    for (int i = 0; i < 4; ++i) {
        s->blend_work_dom[i] = (int64_t)h.pairs[2 + i];
        s->blend_work_roi[i] = (int64_t)h.pairs[8 + i];
    }
}

struct RasterOut {
    float* rgb;
    float* dz;
    float* alpha;
    uint8_t* cls;
};

// Stage 1 for one camera, optionally restricted to the tiles of tile_mask.
// reuse_order: the compositing order of an earlier pass whose centre-depth
// keys are bit-identical to this camera's (null: sort here).  *order_out
// receives the order used.
// cam_next: also preprocess the surfels for this camera (the affiliated eye
// of a stereo frame) into the second record set; precomputed: this pass's
// camera is that one, so it takes those records and only counts the keys
// inside tile_mask.
// The sorted per-tile surfel lists of a pass: surfel = vals[i] & vmask.
struct SortedVals {
    const uint32_t* vals;
    uint32_t vmask;
};

int raster_pass(bgs_ctx* ctx, const Layout& L, void* ws, int64_t kc, const bgs_scene& scene, const bgs_camera& cam,
                const bgs_raster_params& rp, const uint8_t* tile_mask, float a_min, const RasterOut& out, int which,
                const uint32_t* reuse_order = nullptr, const uint32_t** order_out = nullptr,
                const bgs_camera* cam_next = nullptr, bool precomputed = false, SortedVals* vals_out = nullptr,
                const uint8_t* qmask = nullptr, int qmask_w = 0, BatchBlendDesc* defer = nullptr,
                bool xfer = false) {
    hipStream_t s = ctx->stream;
    const int n = (int)scene.n;
    const PreCam pc = make_precam(cam);
    const int n_tiles = pc.tiles_x * pc.tiles_y;
    DevStatus* st = at<DevStatus>(ws, L.status);
    const int sb = which ? BGS_STAGE_PREPROCESS_ROI : BGS_STAGE_PREPROCESS_DOM;
    mark(ctx, sb + 0, 0);
    MaskArgs mask{nullptr, nullptr, pc.tiles_x, 0};
    if (tile_mask) {
        HIP_CHECK(launch_mask_tables(tile_mask, n_tiles, pc.tiles_x, at<uint32_t>(ws, L.mprefix),
                                     at<uint32_t>(ws, L.tlist), at<uint32_t>(ws, L.colcum), st, s),
                  "mask tables");
        mask.prefix = at<uint32_t>(ws, L.mprefix);
        mask.colcum = at<uint32_t>(ws, L.colcum);
        mask.enabled = 1;
    }
    SurfelRec* recs = at<SurfelRec>(ws, precomputed ? L.recs2 : L.recs);
    uint32_t* zkeys = at<uint32_t>(ws, precomputed ? L.zkeys2 : L.zkeys);
    uint2* rects = at<uint2>(ws, precomputed ? L.rects2 : L.rects);
    uint32_t* counts = at<uint32_t>(ws, L.counts);
    uint32_t* nseg = at<uint32_t>(ws, L.nseg);  // rows with keys per surfel, from the counting kernel
    int nseg_by_pos = 0;
    uint32_t* offs = at<uint32_t>(ws, L.offs);
    // Precomputed records: the masked key counts are taken in compositing
    // order together with the first step of their scan, once the order is
    // known (below), when the flat scan covers n.
    const bool fused_counts = precomputed && scan_is_flat(n);
    if (precomputed) {
        if (!tile_mask) return fail(ctx, BGS_ERR_INVALID_ARG, "precomputed records need a tile mask");
        if (!fused_counts)
            HIP_CHECK(launch_masked_counts(rects, recs, n, n_tiles, mask, counts, nseg, s), "masked counts");
    } else {
        const SceneArgs sa{scene.pos, scene.quat, scene.scale, scene.opacity, scene.sh, n, scene.sh_degree};
        PreCam pn{};
        if (cam_next) pn = make_precam(*cam_next);
        HIP_CHECK(launch_preprocess(sa, pc, rp.alpha_min, rp.lowpass, mask, recs, zkeys, rects, counts,
                                    cam_next ? &pn : nullptr, at<SurfelRec>(ws, L.recs2), at<uint32_t>(ws, L.zkeys2),
                                    at<uint2>(ws, L.rects2), nseg, s),
                  "preprocess");
    }
    mark(ctx, sb + 0, 1);
    // Compositing order: surfels sorted by (fp32 centre-depth bits, index).
    mark(ctx, sb + 1, 0);
    bool in_b = false;
    const uint32_t* order = reuse_order;
    if (!order) {
        uint32_t* dva = at<uint32_t>(ws, L.dvals_a);
        uint32_t* dvb = at<uint32_t>(ws, L.dvals_b);
        HIP_CHECK(radix_sort(zkeys, dva, at<uint32_t>(ws, L.dkeys_b), dvb, nullptr, n, 32, true,
                             at<void>(ws, L.radix), s, &in_b),
                  "depth sort");
        order = in_b ? dvb : dva;
    }
    if (order_out) *order_out = order;
    mark(ctx, sb + 1, 1);
    mark(ctx, sb + 2, 0);
    hipError_t se = hipSuccess;
    uint2* ranges = at<uint2>(ws, L.ranges);
    uint32_t* surf_scan = at<uint32_t>(ws, L.surf_scan);
    const KeyCount kcnt{st, (uint32_t)kc, which, ranges, (uint32_t)n_tiles};
    bool scanned;
    if (fused_counts) {
        nseg_by_pos = 1;
        HIP_CHECK(launch_masked_counts_ordered(rects, recs, order, n, n_tiles, mask, counts, surf_scan, nseg, s),
                  "masked counts");
        scanned = scan_counts_presummed(counts, offs, n, surf_scan, kcnt, s, &se);  // the flat form covers n
    } else {
        scanned = scan_counts(counts, order, offs, n, surf_scan, kcnt, s, &se);
    }
    if (scanned) {
        HIP_CHECK(se, "count scan");
    } else {
        HIP_CHECK(exclusive_scan(counts, order, offs, nullptr, n, at<uint32_t>(ws, L.surf_scan), s), "count scan");
        HIP_CHECK(launch_status_keys(offs, n, st, (uint32_t)kc, which, s), "key count");
        HIP_CHECK(launch_clear_ranges(ranges, n_tiles, s), "range clear");
    }
    uint32_t* tka = at<uint32_t>(ws, L.tkeys_a);
    uint32_t* tva = at<uint32_t>(ws, L.tvals_a);
    uint32_t* tkb = at<uint32_t>(ws, L.tkeys_b);
    uint32_t* tvb = at<uint32_t>(ws, L.tvals_b);
    // A key and its surfel share one word (tile << vbits | surfel) when both
    // fit in 32 bits: the sort then moves half the bytes.
    const int tbits = tile_bits(n_tiles), sbits = tile_bits(n);
    const int vbits = tbits + sbits <= 32 ? sbits : 0;
    HIP_CHECK(launch_emit(order, offs, rects, recs, n, pc.tiles_x, n_tiles, mask, (uint32_t)kc, vbits, tka, tva, nseg,
                          nseg_by_pos, s),
              "emit");
    mark(ctx, sb + 2, 1);
    // Stable sort by tile: within a tile the emission (= compositing) order stays.
    mark(ctx, sb + 3, 0);
    // An ROI pass's key count is known only on the device and ranges from a
    // few thousand keys to most of a full pass's: the sort runs both of its
    // forms, each gated on that count.
    HIP_CHECK(radix_sort(tka, vbits ? nullptr : tva, tkb, vbits ? nullptr : tvb, &st->n_sort, kc, tbits, false,
                         at<void>(ws, L.radix), s, &in_b, tile_mask ? -1 : 0, vbits),
              "tile sort");
    const uint32_t* skeys = in_b ? tkb : tka;
    const uint32_t* svals = vbits ? skeys : in_b ? tvb : tva;
    const uint32_t vmask = vbits ? (1u << vbits) - 1u : 0xFFFFFFFFu;
    if (vals_out) *vals_out = SortedVals{svals, vmask};
    mark(ctx, sb + 3, 1);
    mark(ctx, sb + 4, 0);
    HIP_CHECK(launch_ranges(skeys, &st->n_sort, kc, ranges, n_tiles, vbits, s), "ranges");
    uint32_t* torder = at<uint32_t>(ws, L.torder);
    HIP_CHECK(launch_tile_order(ranges, tile_mask ? &st->n_masked : nullptr, n_tiles, torder, s), "tile order");
    mark(ctx, sb + 4, 1);
    BlendArgs ba{};
    ba.W = cam.width;
    ba.H = cam.height;
    ba.tiles_x = pc.tiles_x;
    ba.alpha_min = rp.alpha_min;
    ba.alpha_max = rp.alpha_max;
    ba.t_min = rp.t_min;
    ba.lowpass = rp.lowpass;
    ba.bg0 = rp.bg[0];
    ba.bg1 = rp.bg[1];
    ba.bg2 = rp.bg[2];
    ba.a_min = a_min;
    ba.z_near = (float)cam.z_near;
    ba.patch = tile_mask ? 1 : 0;
    ba.vmask = vmask;
    ba.qmask = qmask;
    ba.qmask_w = qmask_w;
    if (xfer) {
        // The affiliated eye's records hold every binned surfel's colour seen
        // from that eye (written by the two-eye preprocess of this pass).
        ba.xrecs = at<SurfelRec>(ws, L.recs2);
        ba.xrgb = at<float>(ws, L.xrgb);
    }
    const uint32_t cap = n_tiles > kSplitMaxTiles || xfer ? 0u : which ? ctx->cap_roi : ctx->cap_dom;
    const ContArgs ca{cap, ctx->seg_len, L.cslots, which ? ctx->far_roi : ctx->far_dom, &st->n_slots,
                      &st->n_items,
                      at<uint4>(ws, L.cdesc), at<uint32_t>(ws, L.citem), at<float4>(ws, L.cst1),
                      at<float4>(ws, L.cpart)};
    if (defer) {
        // Batched form: the blend of this frame runs later, in one launch with
        // the other frames of the batch (no continuation there).
        BatchBlendDesc d{};
        d.recs = recs;
        d.vals = svals;
        d.ranges = ranges;
        d.tile_list = tile_mask ? at<uint32_t>(ws, L.tlist) : nullptr;
        d.order = torder;
        d.n_live = tile_mask ? &st->n_masked : nullptr;
        d.n_tiles = (uint32_t)n_tiles;
        d.a = ba;
        d.rgb = out.rgb;
        d.dz = out.dz;
        d.alpha = out.alpha;
        d.cls = out.cls;
        HIP_CHECK(launch_put_desc(d, defer, s), "batch descriptor");
        return BGS_OK;
    }
    mark(ctx, sb + 5, 0);
    HIP_CHECK(launch_blend(recs, svals, ranges, tile_mask ? at<uint32_t>(ws, L.tlist) : nullptr, torder,
                           tile_mask ? &st->n_masked : nullptr, n_tiles, ba, ca, out.rgb, out.dz, out.alpha, out.cls,
                           ctx->count_pairs ? &st->pairs[6 * which] : nullptr,
                           (ctx->count_pairs && which == 0) ? at<long long>(ws, L.trace) : nullptr, s),
              "blend");
    mark(ctx, sb + 5, 1);
    return BGS_OK;
}

// The rasteriser-tile (16x16) mask an ROI pass bins, and the 8x8 quadrant
// mask its blend honours, for an ROI tile mask with roi.tile-pixel tiles.
struct PatchMasks {
    const uint8_t* mask16;
    const uint8_t* qmask;
    int qmask_w;
};

hipError_t patch_masks(bgs_ctx* ctx, const Layout& L, void* ws, const bgs_camera& dst, int T, const uint8_t* tile_mask,
                       PatchMasks* pm) {
    if (T == kTile) {
        *pm = PatchMasks{tile_mask, nullptr, 0};
        return hipSuccess;
    }
    uint8_t* m16 = at<uint8_t>(ws, L.mask16);
    *pm = PatchMasks{m16, T == 8 ? tile_mask : nullptr, (dst.width + 7) / 8};
    return launch_mask_to16(tile_mask, T, dst.width, dst.height, m16, ctx->stream);
}

// Start-of-frame status reset: zero the block, keeping the overflow bits of
// earlier frames (sticky until polled) once this context has used the workspace.
hipError_t reset_status(bgs_ctx* ctx, void* ws, DevStatus* st) {
    const int full = ws != ctx->ws_seen;
    ctx->ws_seen = ws;
    return launch_status_reset(st, full, ctx->stream);
}

int finish(bgs_ctx* ctx, void* ws, const Layout& L, DevStatus* host) {
    HIP_CHECK(hipMemcpyAsync(host, at<DevStatus>(ws, L.status), sizeof(DevStatus), hipMemcpyDeviceToHost, ctx->stream),
              "status readback");
    HIP_CHECK(hipStreamSynchronize(ctx->stream), "stream sync");
    return BGS_OK;
}

}  // namespace
}  // namespace bgs

using namespace bgs;

namespace {

// Device address of `scratch` on each GPU, looked up once per device with
// that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_for_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t bgs_ctx_create(bgs_ctx** out, void* stream) {
    if (!out) return BGS_ERR_INVALID_ARG;
    bgs_ctx* c = new (std::nothrow) bgs_ctx();
    if (!c) return BGS_ERR_INVALID_ARG;
    c->stream = (hipStream_t)stream;
    *out = c;
    return BGS_OK;
}

int32_t bgs_ctx_destroy(bgs_ctx* ctx) {
    if (!ctx) return BGS_OK;
    for (int r = 0; r < bgs_ctx::kRing; ++r)
        for (int i = 0; i < BGS_NUM_STAGES; ++i)
            for (int j = 0; j < 2; ++j)
                if (ctx->ev[r][i][j]) (void)hipEventDestroy(ctx->ev[r][i][j]);  // nothing to report on teardown
    delete ctx;
    return BGS_OK;
}

int32_t bgs_ctx_set_stream(bgs_ctx* ctx, void* stream) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)stream;
    return BGS_OK;
}

int32_t bgs_ctx_set_sync(bgs_ctx* ctx, int32_t sync) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    ctx->sync = sync ? 1 : 0;
    return BGS_OK;
}

const char* bgs_last_error(const bgs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t bgs_ctx_set_count_pairs(bgs_ctx* ctx, int32_t count) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    ctx->count_pairs = count ? 1 : 0;
    return BGS_OK;
}

int32_t bgs_ctx_set_blend_split(bgs_ctx* ctx, int32_t cap_dom, int32_t cap_roi, int32_t seg_len, int32_t far_dom,
                                int32_t far_roi) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (cap_dom < 0 || cap_roi < 0 || seg_len < 1 || far_dom < 0 || far_roi < 0)
        return fail(ctx, BGS_ERR_INVALID_ARG, "blend split: need caps >= 0, seg_len >= 1 and far_* >= 0");
    ctx->cap_dom = (uint32_t)cap_dom;
    ctx->cap_roi = (uint32_t)cap_roi;
    ctx->seg_len = (uint32_t)seg_len;
    ctx->far_dom = (uint32_t)far_dom;
    ctx->far_roi = (uint32_t)far_roi;
    return BGS_OK;
}

int32_t bgs_ctx_set_timing(bgs_ctx* ctx, int32_t on) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (on) {
        for (int r = 0; r < bgs_ctx::kRing; ++r)
            for (int i = 0; i < BGS_NUM_STAGES; ++i)
                for (int j = 0; j < 2; ++j)
                    if (!ctx->ev[r][i][j]) {
                        hipError_t e = hipEventCreate(&ctx->ev[r][i][j]);
                        if (e != hipSuccess) return hip_fail(ctx, e, "event create");
                    }
    }
    ctx->timing = on == -1 ? ((1u << BGS_NUM_STAGES) - 1u) : ((uint32_t)on & ((1u << BGS_NUM_STAGES) - 1u));
    ctx->slot = 0;
    for (int i = 0; i < BGS_NUM_STAGES; ++i) {
        for (int r = 0; r < bgs_ctx::kRing; ++r) ctx->pending[r][i] = false;
        ctx->total_ms[i] = 0.0;
        ctx->count[i] = 0;
    }
    return BGS_OK;
}

int32_t bgs_timing_collect(bgs_ctx* ctx, double* total_ms, int64_t* counts) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (ctx->timing_err != hipSuccess) {
        const hipError_t e = ctx->timing_err;
        ctx->timing_err = hipSuccess;
        return hip_fail(ctx, e, "stage timing (event record)");
    }
    for (int k = 1; k <= bgs_ctx::kRing; ++k) {
        const hipError_t e = drain_slot(ctx, (ctx->slot + k) % bgs_ctx::kRing);
        if (e != hipSuccess) return hip_fail(ctx, e, "stage timing");
    }
    for (int i = 0; i < BGS_NUM_STAGES; ++i) {
        if (total_ms) total_ms[i] = ctx->total_ms[i];
        if (counts) counts[i] = ctx->count[i];
    }
    return BGS_OK;
}

int32_t bgs_workspace_size(int64_t n, int32_t width, int32_t height, int64_t key_capacity, size_t* bytes) {
    if (!bytes || n < 0 || n >= ((int64_t)1 << 31) || width < 1 || height < 1 || width > 16384 || height > 16384 ||
        key_capacity < 0 || key_capacity > (int64_t)0xFFFFFFF0)
        return BGS_ERR_INVALID_ARG;
    *bytes = make_layout(n, width, height, key_capacity).total;
    return BGS_OK;
}

int32_t bgs_poll_status(bgs_ctx* ctx, void* ws, size_t ws_bytes, bgs_stats* stats) {
    if (!ctx || !ws || !stats) return fail(ctx, BGS_ERR_INVALID_ARG, "null argument");
    if (ws_bytes < sizeof(DevStatus)) return fail(ctx, BGS_ERR_WORKSPACE, "workspace too small");
    Layout L{};
    L.status = 0;
    DevStatus h{};
    int rc = finish(ctx, ws, L, &h);
    if (rc) return rc;
    fill_stats(h, stats);
    // Overflow of any frame since the last poll, not only of the last one.
    stats->overflow = (int32_t)(h.overflow | h.sticky);
    if (ws == ctx->ws_seen) {
        HIP_CHECK(launch_fill_u32(&at<DevStatus>(ws, 0)->sticky, 1, 0u, ctx->stream), "sticky clear");
        HIP_CHECK(hipStreamSynchronize(ctx->stream), "stream sync");
    }
    return BGS_OK;
}

int32_t bgs_render_dominant(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam,
                            const bgs_raster_params* raster, void* ws, size_t ws_bytes, float* rgb, float* depth_raw,
                            float* alpha, int64_t* n_keys) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_scene(ctx, scene)) || (rc = check_camera(ctx, cam, "camera")) || (rc = check_raster(ctx, raster)))
        return rc;
    if (!ws || !rgb || !depth_raw || !alpha) return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    const int64_t kc = key_capacity_for(scene->n, cam->width, cam->height, ws_bytes);
    if (kc < 0) return fail(ctx, BGS_ERR_WORKSPACE, "workspace of %zu bytes is too small", ws_bytes);
    const Layout L = make_layout(scene->n, cam->width, cam->height, kc);
    DevStatus* st = at<DevStatus>(ws, L.status);
    HIP_CHECK(reset_status(ctx, ws, st), "status reset");
    rc = raster_pass(ctx, L, ws, kc, *scene, *cam, *raster, nullptr, 0.f, RasterOut{rgb, depth_raw, alpha, nullptr}, 0);
    if (rc) return rc;
    if (!ctx->sync) return BGS_OK;
    DevStatus h{};
    if ((rc = finish(ctx, ws, L, &h))) return rc;
    if (n_keys) *n_keys = h.n_keys_dom;
    if (h.overflow & 1u)
        return fail(ctx, BGS_ERR_CAPACITY, "%u tile keys exceed the workspace capacity of %lld", h.n_keys_dom,
                    (long long)kc);
    return BGS_OK;
}

int32_t bgs_reproject(bgs_ctx* ctx, const bgs_camera* src, const bgs_camera* dst, const bgs_roi_params* roi,
                      const float* rgb_src, const float* depth_raw_src, const float* alpha_src, void* ws,
                      size_t ws_bytes, float* rgb_dst, float* z_dst, float* alpha_dst, uint8_t* hole_mask,
                      float* depth_range) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_camera(ctx, src, "src")) || (rc = check_camera(ctx, dst, "dst")) || (rc = check_roi(ctx, roi)))
        return rc;
    if (!rgb_src || !depth_raw_src || !alpha_src || !ws || !rgb_dst || !z_dst || !alpha_dst || !hole_mask ||
        !depth_range)
        return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    if ((int64_t)src->width * src->height > ((int64_t)1 << 32))
        return fail(ctx, BGS_ERR_INVALID_ARG, "source image too large");
    const Layout L = make_layout(0, dst->width, dst->height, 0);
    if (L.total > ws_bytes) return fail(ctx, BGS_ERR_WORKSPACE, "workspace of %zu bytes is too small", ws_bytes);
    DevStatus* st = at<DevStatus>(ws, L.status);
    HIP_CHECK(launch_reproject(make_warpcam(*src), make_warpcam(*dst), rel_pose(*src, *dst), roi->a_min, rgb_src,
                               depth_raw_src, alpha_src, at<unsigned long long>(ws, L.zbuf), rgb_dst, z_dst, alpha_dst,
                               hole_mask, depth_range, true, at<uint4>(ws, L.wpart), st, ctx->stream),
              "reproject");
    return BGS_OK;
}

int32_t bgs_reproject_noalloc(bgs_ctx* ctx, const bgs_camera* src, const bgs_camera* dst, const bgs_roi_params* roi,
                              const float* rgb_src, const float* depth_raw_src, const float* alpha_src, float* rgb_dst,
                              float* z_dst, float* alpha_dst, uint8_t* hole_mask, float* depth_range) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_camera(ctx, src, "src")) || (rc = check_camera(ctx, dst, "dst")) || (rc = check_roi(ctx, roi)))
        return rc;
    if (!rgb_src || !depth_raw_src || !alpha_src || !rgb_dst || !z_dst || !alpha_dst || !hole_mask || !depth_range)
        return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    if ((int64_t)src->width * src->height > ((int64_t)1 << 32))
        return fail(ctx, BGS_ERR_INVALID_ARG, "source image too large");
    const int64_t nd = (int64_t)dst->width * dst->height;
    if (nd > (int64_t)BGS_REPROJECT_NOALLOC_MAX_PIXELS)
        return fail(ctx, BGS_ERR_INVALID_ARG,
                    "destination of %dx%d pixels exceeds the %d pixels of the static scratch; use bgs_reproject",
                    dst->width, dst->height, (int)BGS_REPROJECT_NOALLOC_MAX_PIXELS);
    static_assert(sizeof(DevStatus) <= 512, "status block fits its scratch slot");
    void* base = nullptr;
    HIP_CHECK(scratch_for_current_device(&base), "scratch address");
    char* sp = static_cast<char*>(base);
    DevStatus* st = reinterpret_cast<DevStatus*>(sp);
    uint4* wpart = reinterpret_cast<uint4*>(sp + 512);
    unsigned long long* zbuf = reinterpret_cast<unsigned long long*>(sp + 512 + 16 * 16384);
    // reset = true clears the status fields the reprojection accumulates; the
    // z-buffer is refilled and every row partial rewritten by each call.
    HIP_CHECK(launch_reproject(make_warpcam(*src), make_warpcam(*dst), rel_pose(*src, *dst), roi->a_min, rgb_src,
                               depth_raw_src, alpha_src, zbuf, rgb_dst, z_dst, alpha_dst, hole_mask, depth_range, true,
                               wpart, st, ctx->stream),
              "reproject");
    return BGS_OK;
}

int32_t bgs_classify_holes(bgs_ctx* ctx, const bgs_camera* src, const bgs_camera* dst, const bgs_roi_params* roi,
                           const bgs_raster_params* raster, const float* depth_range, void* ws, size_t ws_bytes,
                           float* rgb_dst, float* z_dst, float* alpha_dst, uint8_t* cls, int32_t* labels,
                           bgs_box* boxes, int32_t box_capacity, int32_t* n_boxes, uint8_t* tile_mask) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_camera(ctx, src, "src")) || (rc = check_camera(ctx, dst, "dst")) || (rc = check_roi(ctx, roi)) ||
        (rc = check_raster(ctx, raster)))
        return rc;
    if (!depth_range || !ws || !rgb_dst || !z_dst || !alpha_dst || !cls || !labels || !n_boxes || !tile_mask ||
        (box_capacity > 0 && !boxes) || box_capacity < 0)
        return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer or negative box capacity");
    const Layout L = make_layout(0, dst->width, dst->height, 0);
    if (L.total > ws_bytes) return fail(ctx, BGS_ERR_WORKSPACE, "workspace of %zu bytes is too small", ws_bytes);
    ClassifyBufs b{at<uint8_t>(ws, L.hole), at<uint8_t>(ws, L.hole2), at<uint32_t>(ws, L.bcount),
                   at<uint32_t>(ws, L.rmask), at<int32_t>(ws, L.bbox), at<uint8_t>(ws, L.pflag),
                   at<int4>(ws, L.pbox), at<uint4>(ws, L.wpart), at<uint2>(ws, L.gpart)};
    HIP_CHECK(launch_classify(make_warpcam(*src), make_warpcam(*dst), rel_pose(*src, *dst), *roi, raster->bg,
                              depth_range, rgb_dst, z_dst, alpha_dst, cls, labels, boxes, box_capacity, n_boxes,
                              tile_mask, b, at<DevStatus>(ws, L.status), ctx->stream),
              "classify");
    return BGS_OK;
}

int32_t bgs_patch_rois(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* dst, const bgs_raster_params* raster,
                       const bgs_roi_params* roi, const uint8_t* tile_mask, void* ws, size_t ws_bytes, float* rgb_dst,
                       float* z_dst, float* alpha_dst, uint8_t* cls, int64_t* n_keys) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_scene(ctx, scene)) || (rc = check_camera(ctx, dst, "dst")) || (rc = check_raster(ctx, raster)) ||
        (rc = check_roi(ctx, roi)))
        return rc;
    if (!tile_mask || !ws || !rgb_dst || !z_dst || !alpha_dst || !cls) return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    const int64_t kc = key_capacity_for(scene->n, dst->width, dst->height, ws_bytes);
    if (kc < 0) return fail(ctx, BGS_ERR_WORKSPACE, "workspace of %zu bytes is too small", ws_bytes);
    const Layout L = make_layout(scene->n, dst->width, dst->height, kc);
    DevStatus* st = at<DevStatus>(ws, L.status);
    HIP_CHECK(reset_status(ctx, ws, st), "status reset");
    PatchMasks pm{};
    HIP_CHECK(patch_masks(ctx, L, ws, *dst, roi->tile, tile_mask, &pm), "ROI tile mask");
    rc = raster_pass(ctx, L, ws, kc, *scene, *dst, *raster, pm.mask16, roi->a_min,
                     RasterOut{rgb_dst, z_dst, alpha_dst, cls}, 1, nullptr, nullptr, nullptr, false, nullptr, pm.qmask,
                     pm.qmask_w);
    if (rc) return rc;
    if (!ctx->sync) return BGS_OK;
    DevStatus h{};
    if ((rc = finish(ctx, ws, L, &h))) return rc;
    if (n_keys) *n_keys = h.n_keys_roi;
    if (h.overflow & 1u)
        return fail(ctx, BGS_ERR_CAPACITY, "%u ROI keys exceed the workspace capacity of %lld", h.n_keys_roi,
                    (long long)kc);
    return BGS_OK;
}

int32_t bgs_render_stereo(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam_dom, const bgs_camera* cam_aff,
                          const bgs_raster_params* raster, const bgs_roi_params* roi, void* ws, size_t ws_bytes,
                          float* rgb_dom, float* depth_raw_dom, float* alpha_dom, float* rgb_aff, float* z_aff,
                          float* alpha_aff, uint8_t* cls_aff, int32_t* labels, bgs_box* boxes, int32_t box_capacity,
                          int32_t* n_boxes, uint8_t* tile_mask, bgs_stats* stats) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_scene(ctx, scene)) || (rc = check_camera(ctx, cam_dom, "dominant camera")) ||
        (rc = check_camera(ctx, cam_aff, "affiliated camera")) || (rc = check_raster(ctx, raster)) ||
        (rc = check_roi(ctx, roi)))
        return rc;
    if (!ws || !rgb_dom || !depth_raw_dom || !alpha_dom || !rgb_aff || !z_aff || !alpha_aff || !cls_aff || !labels ||
        !n_boxes || !tile_mask || box_capacity < 0 || (box_capacity > 0 && !boxes))
        return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer or negative box capacity");
    const int W = cam_dom->width > cam_aff->width ? cam_dom->width : cam_aff->width;
    const int H = cam_dom->height > cam_aff->height ? cam_dom->height : cam_aff->height;
    const int64_t kc = key_capacity_for(scene->n, W, H, ws_bytes);
    if (kc < 0) return fail(ctx, BGS_ERR_WORKSPACE, "workspace of %zu bytes is too small", ws_bytes);
    const Layout L = make_layout(scene->n, W, H, kc);
    hipStream_t s = ctx->stream;
    DevStatus* st = at<DevStatus>(ws, L.status);
    HIP_CHECK(reset_status(ctx, ws, st), "status reset");
    // Stage 1: dominant eye with the depth proxy (and, with the view-colour
    // transfer on a scene whose colours depend on the view, the affiliated
    // view's colours under the same weights).
    const uint32_t* dom_order = nullptr;
    const bool xfer = roi->view_colour != 0 && scene->sh_degree > 0;
    rc = raster_pass(ctx, L, ws, kc, *scene, *cam_dom, *raster, nullptr, 0.f,
                     RasterOut{rgb_dom, depth_raw_dom, alpha_dom, nullptr}, 0, nullptr, &dom_order, cam_aff, false,
                     nullptr, nullptr, 0, nullptr, xfer);
    if (rc) return rc;
    const float* rgb_src = xfer ? at<float>(ws, L.xrgb) : rgb_dom;
    // The affiliated eye's compositing order equals the dominant one when
    // their fp32 centre-depth key coefficients and near planes coincide bit
    // for bit (same orientation, offset perpendicular to the optical axis):
    // every surfel then gets the same key, so the depth sort is reused.
    const PreCam pd = make_precam(*cam_dom), pa = make_precam(*cam_aff);
    const bool same_keys = std::memcmp(pd.zc, pa.zc, sizeof pd.zc) == 0 && pd.z_near == pa.z_near;
    // Stage 2: reprojection.  The hole mask is written straight into cls.
    const WarpCam wd = make_warpcam(*cam_dom), wa = make_warpcam(*cam_aff);
    const RelPose P = rel_pose(*cam_dom, *cam_aff);
    // The status block was zeroed at the start of the frame, so the
    // reprojection needs no reset, and classification reads the depth range
    // straight from it.
    mark(ctx, BGS_STAGE_REPROJECT, 0);
    HIP_CHECK(launch_reproject(wd, wa, P, roi->a_min, rgb_src, depth_raw_dom, alpha_dom,
                               at<unsigned long long>(ws, L.zbuf), rgb_aff, z_aff, alpha_aff, cls_aff, nullptr, false,
                               at<uint4>(ws, L.wpart), st, s),
              "reproject");
    mark(ctx, BGS_STAGE_REPROJECT, 1);
    // Stage 3: hole classification and interpolation.
    ClassifyBufs b{at<uint8_t>(ws, L.hole), at<uint8_t>(ws, L.hole2), at<uint32_t>(ws, L.bcount),
                   at<uint32_t>(ws, L.rmask), at<int32_t>(ws, L.bbox), at<uint8_t>(ws, L.pflag),
                   at<int4>(ws, L.pbox), at<uint4>(ws, L.wpart), at<uint2>(ws, L.gpart)};
    mark(ctx, BGS_STAGE_CLASSIFY, 0);
    HIP_CHECK(launch_classify(wd, wa, P, *roi, raster->bg, nullptr, rgb_aff, z_aff, alpha_aff, cls_aff, labels, boxes,
                              box_capacity, n_boxes, tile_mask, b, st, s),
              "classify");
    mark(ctx, BGS_STAGE_CLASSIFY, 1);
    // Stage 4: ROI re-rasterisation of the affiliated eye.
    PatchMasks pm{};
    HIP_CHECK(patch_masks(ctx, L, ws, *cam_aff, roi->tile, tile_mask, &pm), "ROI tile mask");
    rc = raster_pass(ctx, L, ws, kc, *scene, *cam_aff, *raster, pm.mask16, roi->a_min,
                     RasterOut{rgb_aff, z_aff, alpha_aff, cls_aff}, 1, same_keys ? dom_order : nullptr, nullptr,
                     nullptr, true, nullptr, pm.qmask, pm.qmask_w);
    if (rc) return rc;
    if (!ctx->sync && !stats) return BGS_OK;
    DevStatus h{};
    if ((rc = finish(ctx, ws, L, &h))) return rc;
    if (stats) fill_stats(h, stats);
    if (h.overflow & 1u)
        return fail(ctx, BGS_ERR_CAPACITY, "tile keys (%u dominant, %u ROI) exceed the capacity of %lld", h.n_keys_dom,
                    h.n_keys_roi, (long long)kc);
    return BGS_OK;
}

}  // extern "C"

namespace {

constexpr int32_t kMaxBatch = 4096;

size_t batch_desc_bytes(int32_t n) { return up(sizeof(BatchBlendDesc) * (size_t)n); }

size_t batch_ws_bytes_for(int32_t n) { return 2 * batch_desc_bytes(n) + 2 * up(4 * ((size_t)n + 2)); }

// Start-of-frame status reset of a batched pair's workspace (sticky overflow
// kept once this context has reset that workspace before).
hipError_t reset_status_batch(bgs_ctx* ctx, void* ws, DevStatus* st) {
    bool seen = false;
    for (const void* w : ctx->batch_seen) seen = seen || w == ws;
    if (!seen) ctx->batch_seen.push_back(ws);
    return launch_status_reset(st, seen ? 0 : 1, ctx->stream);
}

// Validate the batch (host only, nothing launched), then issue it.
int batch_issue(bgs_ctx* ctx, int32_t n, const bgs_batch_pair* pairs, const bgs_raster_params* raster, void* bws,
                size_t bws_bytes) {
    int rc;
    if (n < 1 || n > kMaxBatch) return fail(ctx, BGS_ERR_INVALID_ARG, "batch of %d pairs outside [1, %d]", n, kMaxBatch);
    if (!pairs || !bws) return fail(ctx, BGS_ERR_INVALID_ARG, "null batch");
    if ((rc = check_raster(ctx, raster))) return rc;
    if (bws_bytes < batch_ws_bytes_for(n)) return fail(ctx, BGS_ERR_WORKSPACE, "batch workspace too small");
    if (ctx->timing) return fail(ctx, BGS_ERR_INVALID_ARG, "stage timing must be off for batched frames");
    std::vector<Layout> lays((size_t)n);
    std::vector<int64_t> kcs((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const bgs_batch_pair& q = pairs[i];
        if ((rc = check_scene(ctx, q.scene)) || (rc = check_camera(ctx, &q.cam_dom, "dominant camera")) ||
            (rc = check_camera(ctx, &q.cam_aff, "affiliated camera")) || (rc = check_roi(ctx, &q.roi)))
            return rc;
        if (q.roi.view_colour)
            return fail(ctx, BGS_ERR_UNSUPPORTED, "pair %d: the view-colour transfer is not supported in batches", i);
        if (!q.ws || !q.rgb_dom || !q.depth_raw_dom || !q.alpha_dom || !q.rgb_aff || !q.z_aff || !q.alpha_aff ||
            !q.cls_aff || !q.labels || !q.n_boxes || !q.tile_mask || q.box_capacity < 0 ||
            (q.box_capacity > 0 && !q.boxes))
            return fail(ctx, BGS_ERR_INVALID_ARG, "pair %d: null buffer or negative box capacity", i);
        const int W = std::max(q.cam_dom.width, q.cam_aff.width), H = std::max(q.cam_dom.height, q.cam_aff.height);
        kcs[i] = key_capacity_for(q.scene->n, W, H, q.ws_bytes);
        if (kcs[i] < 0) return fail(ctx, BGS_ERR_WORKSPACE, "pair %d: workspace of %zu bytes is too small", i, q.ws_bytes);
        lays[i] = make_layout(q.scene->n, W, H, kcs[i]);
    }
    if (ctx->n_cu <= 0) {
        int dev = 0, cus = 0;
        HIP_CHECK(hipGetDevice(&dev), "device");
        HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
        ctx->n_cu = cus > 0 ? cus : 256;
    }
    const int grid = ctx->n_cu * 8;  // 8 blend workgroups fit a CU (LDS)
    hipStream_t s = ctx->stream;
    BatchBlendDesc* dd = at<BatchBlendDesc>(bws, 0);
    BatchBlendDesc* dr = at<BatchBlendDesc>(bws, batch_desc_bytes(n));
    uint32_t* qd = at<uint32_t>(bws, 2 * batch_desc_bytes(n));
    uint32_t* qr = at<uint32_t>(bws, 2 * batch_desc_bytes(n) + up(4 * ((size_t)n + 2)));
    std::vector<const uint32_t*> dom_order((size_t)n);
    // Stage 1 of every pair up to its sorted tile lists; the blends follow in
    // one launch.
    for (int32_t i = 0; i < n; ++i) {
        const bgs_batch_pair& q = pairs[i];
        void* ws = q.ws;
        HIP_CHECK(reset_status_batch(ctx, ws, at<DevStatus>(ws, lays[i].status)), "status reset");
        rc = raster_pass(ctx, lays[i], ws, kcs[i], *q.scene, q.cam_dom, *raster, nullptr, 0.f,
                         RasterOut{q.rgb_dom, q.depth_raw_dom, q.alpha_dom, nullptr}, 0, nullptr, &dom_order[i],
                         &q.cam_aff, false, nullptr, nullptr, 0, dd + i);
        if (rc) return rc;
    }
    HIP_CHECK(launch_blend_batch(dd, n, qd, grid, false, s), "batched blend");
    // Stages 2-3 and the ROI binning of every pair, then one launch for all
    // ROI tiles.
    for (int32_t i = 0; i < n; ++i) {
        const bgs_batch_pair& q = pairs[i];
        void* ws = q.ws;
        const Layout& L = lays[i];
        DevStatus* st = at<DevStatus>(ws, L.status);
        const PreCam pd = make_precam(q.cam_dom), pa = make_precam(q.cam_aff);
        const bool same_keys = std::memcmp(pd.zc, pa.zc, sizeof pd.zc) == 0 && pd.z_near == pa.z_near;
        const WarpCam wd = make_warpcam(q.cam_dom), wa = make_warpcam(q.cam_aff);
        const RelPose P = rel_pose(q.cam_dom, q.cam_aff);
        HIP_CHECK(launch_reproject(wd, wa, P, q.roi.a_min, q.rgb_dom, q.depth_raw_dom, q.alpha_dom,
                                   at<unsigned long long>(ws, L.zbuf), q.rgb_aff, q.z_aff, q.alpha_aff, q.cls_aff, nullptr,
                                   false, at<uint4>(ws, L.wpart), st, s),
                  "reproject");
        ClassifyBufs b{at<uint8_t>(ws, L.hole), at<uint8_t>(ws, L.hole2), at<uint32_t>(ws, L.bcount),
                       at<uint32_t>(ws, L.rmask), at<int32_t>(ws, L.bbox), at<uint8_t>(ws, L.pflag),
                       at<int4>(ws, L.pbox), at<uint4>(ws, L.wpart), at<uint2>(ws, L.gpart)};
        HIP_CHECK(launch_classify(wd, wa, P, q.roi, raster->bg, nullptr, q.rgb_aff, q.z_aff, q.alpha_aff, q.cls_aff,
                                  q.labels, q.boxes, q.box_capacity, q.n_boxes, q.tile_mask, b, st, s),
                  "classify");
        PatchMasks pm{};
        HIP_CHECK(patch_masks(ctx, L, ws, q.cam_aff, q.roi.tile, q.tile_mask, &pm), "ROI tile mask");
        rc = raster_pass(ctx, L, ws, kcs[i], *q.scene, q.cam_aff, *raster, pm.mask16, q.roi.a_min,
                         RasterOut{q.rgb_aff, q.z_aff, q.alpha_aff, q.cls_aff}, 1, same_keys ? dom_order[i] : nullptr,
                         nullptr, nullptr, true, nullptr, pm.qmask, pm.qmask_w, dr + i);
        if (rc) return rc;
    }
    HIP_CHECK(launch_blend_batch(dr, n, qr, grid, true, s), "batched ROI blend");
    return BGS_OK;
}

}  // namespace

extern "C" {

int32_t bgs_batch_workspace_size(int32_t n_pairs, size_t* bytes) {
    if (!bytes || n_pairs < 1 || n_pairs > kMaxBatch) return BGS_ERR_INVALID_ARG;
    *bytes = batch_ws_bytes_for(n_pairs);
    return BGS_OK;
}

int32_t bgs_render_stereo_batch(bgs_ctx* ctx, int32_t n_pairs, const bgs_batch_pair* pairs,
                                const bgs_raster_params* raster, void* batch_ws, size_t batch_ws_bytes) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    return batch_issue(ctx, n_pairs, pairs, raster, batch_ws, batch_ws_bytes);
}

int32_t bgs_batch_graph_capture(bgs_ctx* ctx, int32_t n_pairs, const bgs_batch_pair* pairs,
                                const bgs_raster_params* raster, void* batch_ws, size_t batch_ws_bytes,
                                bgs_graph** graph) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (!graph) return fail(ctx, BGS_ERR_INVALID_ARG, "null graph");
    if (!ctx->stream) return fail(ctx, BGS_ERR_INVALID_ARG, "graph capture needs a stream other than the null stream");
    HIP_CHECK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    const int rc = batch_issue(ctx, n_pairs, pairs, raster, batch_ws, batch_ws_bytes);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->stream, &g);  // ends the capture whatever happened
    if (rc) {
        if (g) (void)hipGraphDestroy(g);  // the error of the issue is the one reported
        return rc;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(ctx, ei, "graph instantiate");
    }
    bgs_graph* out = new (std::nothrow) bgs_graph();
    if (!out) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return fail(ctx, BGS_ERR_INVALID_ARG, "out of host memory");
    }
    out->graph = g;
    out->exec = ex;
    *graph = out;
    return BGS_OK;
}

int32_t bgs_graph_launch(bgs_ctx* ctx, bgs_graph* graph) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (!graph || !graph->exec) return fail(ctx, BGS_ERR_INVALID_ARG, "null graph");
    HIP_CHECK(hipGraphLaunch(graph->exec, ctx->stream), "graph launch");
    return BGS_OK;
}

int32_t bgs_graph_destroy(bgs_graph* graph) {
    if (!graph) return BGS_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);  // nothing to report on teardown
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return BGS_OK;
}

int32_t bgs_blend_trace(bgs_ctx* ctx, int64_t n, int32_t width, int32_t height, void* ws, size_t ws_bytes,
                        int64_t* out) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (!ws || !out || width < 1 || height < 1 || n < 0) return fail(ctx, BGS_ERR_INVALID_ARG, "bad argument");
    const int64_t kc = key_capacity_for(n, width, height, ws_bytes);
    if (kc < 0) return fail(ctx, BGS_ERR_WORKSPACE, "workspace too small");
    const Layout L = make_layout(n, width, height, kc);
    const int64_t nt = ((width + kTile - 1) / kTile) * (int64_t)((height + kTile - 1) / kTile);
    HIP_CHECK(hipMemcpyAsync(out, at<long long>(ws, L.trace), 6 * 8 * (size_t)nt, hipMemcpyDeviceToHost, ctx->stream),
              "trace copy");
    HIP_CHECK(hipStreamSynchronize(ctx->stream), "sync");
    return BGS_OK;
}

int32_t bgs_sort_workspace_size(int64_t n, size_t* bytes) {
    if (!bytes || n < 0 || n > (int64_t)0xFFFFFFF0) return BGS_ERR_INVALID_ARG;
    *bytes = up(sizeof(DevStatus)) + 2 * up(4 * (size_t)n) + up(radix_tmp_bytes(n));
    return BGS_OK;
}

int32_t bgs_sort_pairs(bgs_ctx* ctx, uint32_t* keys, uint32_t* values, int64_t n, int32_t key_bits, void* ws,
                       size_t ws_bytes) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (n < 0 || n > (int64_t)0xFFFFFFF0) return fail(ctx, BGS_ERR_INVALID_ARG, "n out of range");
    if (key_bits < 1 || key_bits > 32) return fail(ctx, BGS_ERR_INVALID_ARG, "key_bits %d outside 1..32", key_bits);
    if (n == 0) return BGS_OK;
    if (!keys || !values || !ws) return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    size_t need = 0;
    bgs_sort_workspace_size(n, &need);
    if (ws_bytes < need) return fail(ctx, BGS_ERR_WORKSPACE, "sort workspace needs %zu bytes", need);
    uint32_t* kb = at<uint32_t>(ws, up(sizeof(DevStatus)));
    uint32_t* vb = at<uint32_t>(ws, up(sizeof(DevStatus)) + up(4 * (size_t)n));
    void* tmp = at<void>(ws, up(sizeof(DevStatus)) + 2 * up(4 * (size_t)n));
    bool in_b = false;
    HIP_CHECK(radix_sort(keys, values, kb, vb, nullptr, n, key_bits, false, tmp, ctx->stream, &in_b), "sort");
    if (in_b) {
        HIP_CHECK(hipMemcpyAsync(keys, kb, 4 * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream), "copy");
        HIP_CHECK(hipMemcpyAsync(values, vb, 4 * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream), "copy");
    }
    return BGS_OK;
}

int32_t bgs_label_components(bgs_ctx* ctx, const uint8_t* mask, int32_t width, int32_t height, int32_t conn,
                             int32_t* labels) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    if (width < 1 || height < 1 || width > 16384 || height > 16384)
        return fail(ctx, BGS_ERR_INVALID_ARG, "image size out of range");
    if (conn != 4 && conn != 8) return fail(ctx, BGS_ERR_INVALID_ARG, "conn must be 4 or 8");
    if (!mask || !labels) return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    HIP_CHECK(launch_label_components(mask, width, height, conn, labels, ctx->stream), "label components");
    return BGS_OK;
}

int32_t bgs_preprocess_debug(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam,
                             const bgs_raster_params* raster, void* ws, size_t ws_bytes, uint32_t* zkey, int32_t* rects,
                             uint32_t* counts) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_scene(ctx, scene)) || (rc = check_camera(ctx, cam, "camera")) || (rc = check_raster(ctx, raster)))
        return rc;
    if (!ws || !zkey || !rects || !counts) return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    const int64_t kc = key_capacity_for(scene->n, cam->width, cam->height, ws_bytes);
    if (kc < 0) return fail(ctx, BGS_ERR_WORKSPACE, "workspace too small");
    const Layout L = make_layout(scene->n, cam->width, cam->height, kc);
    const PreCam pc = make_precam(*cam);
    const SceneArgs sa{scene->pos, scene->quat, scene->scale, scene->opacity, scene->sh, (int)scene->n,
                       scene->sh_degree};
    const int n = (int)scene->n;
    const MaskArgs no_mask{nullptr, nullptr, pc.tiles_x, 0};
    HIP_CHECK(launch_preprocess(sa, pc, raster->alpha_min, raster->lowpass, no_mask, at<SurfelRec>(ws, L.recs), zkey,
                                at<uint2>(ws, L.rects), counts, nullptr, nullptr, nullptr, nullptr, nullptr,
                                ctx->stream),
              "preprocess");
    // Unpack the tile rectangles for the caller.
    if (n > 0) {
        std::vector<uint2> hr(n);
        HIP_CHECK(hipMemcpyAsync(hr.data(), at<uint2>(ws, L.rects), 8 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream),
                  "rect readback");
        HIP_CHECK(hipStreamSynchronize(ctx->stream), "sync");
        std::vector<int32_t> out(4 * (size_t)n);
        for (int k = 0; k < n; ++k) {
            if (hr[k].x == 0xFFFFFFFFu) {
                out[4 * k] = out[4 * k + 1] = out[4 * k + 2] = out[4 * k + 3] = -1;
            } else {
                out[4 * k] = (int32_t)(hr[k].x & 0xFFFF);
                out[4 * k + 1] = (int32_t)(hr[k].x >> 16);
                out[4 * k + 2] = (int32_t)(hr[k].y & 0xFFFF);
                out[4 * k + 3] = (int32_t)(hr[k].y >> 16);
            }
        }
        HIP_CHECK(hipMemcpyAsync(rects, out.data(), 16 * (size_t)n, hipMemcpyHostToDevice, ctx->stream), "rect copy");
        HIP_CHECK(hipStreamSynchronize(ctx->stream), "sync");
    }
    return BGS_OK;
}

int32_t bgs_tile_lists_debug(bgs_ctx* ctx, const bgs_scene* scene, const bgs_camera* cam,
                             const bgs_raster_params* raster, void* ws, size_t ws_bytes, uint32_t* ranges,
                             uint32_t* values, int64_t values_capacity, int64_t* n_keys) {
    if (!ctx) return BGS_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_scene(ctx, scene)) || (rc = check_camera(ctx, cam, "camera")) || (rc = check_raster(ctx, raster)))
        return rc;
    if (!ws || !ranges || !values || !n_keys) return fail(ctx, BGS_ERR_INVALID_ARG, "null buffer");
    const int64_t kc = key_capacity_for(scene->n, cam->width, cam->height, ws_bytes);
    if (kc < 0) return fail(ctx, BGS_ERR_WORKSPACE, "workspace too small");
    const Layout L = make_layout(scene->n, cam->width, cam->height, kc);
    DevStatus* st = at<DevStatus>(ws, L.status);
    HIP_CHECK(reset_status(ctx, ws, st), "status reset");
    // A render whose outputs go to scratch pixel buffers; the binning it
    // leaves in the workspace is what is copied out.
    const int64_t np = (int64_t)cam->width * cam->height;
    // Scratch outputs: rgb in the piece-box region (16 B/px), depth and
    // alpha in the z-buffer (8 B/px).
    float* scratch = at<float>(ws, L.pbox);
    SortedVals sv{};
    rc = raster_pass(ctx, L, ws, kc, *scene, *cam, *raster, nullptr, 0.f,
                     RasterOut{scratch, at<float>(ws, L.zbuf), at<float>(ws, L.zbuf) + np, nullptr}, 0, nullptr,
                     nullptr, nullptr, false, &sv);
    if (rc) return rc;
    DevStatus h{};
    if ((rc = finish(ctx, ws, L, &h))) return rc;
    *n_keys = h.n_keys_dom;
    if (h.overflow & 1u) return fail(ctx, BGS_ERR_CAPACITY, "key capacity exceeded");
    if ((int64_t)h.n_sort > values_capacity) return fail(ctx, BGS_ERR_CAPACITY, "values_capacity too small");
    const PreCam pc = make_precam(*cam);
    const int n_tiles = pc.tiles_x * pc.tiles_y;
    HIP_CHECK(hipMemcpyAsync(ranges, at<uint2>(ws, L.ranges), 8 * (size_t)n_tiles, hipMemcpyDeviceToDevice, ctx->stream),
              "copy");
    HIP_CHECK(launch_mask_copy(sv.vals, values, (int64_t)h.n_sort, sv.vmask, ctx->stream), "copy");
    HIP_CHECK(hipStreamSynchronize(ctx->stream), "sync");
    return BGS_OK;
}

}  // extern "C"
