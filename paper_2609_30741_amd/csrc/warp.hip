// Reprojection (Sec. 3.4, Eq. 3-5) and hole classification (Sec. 3.1
// Stage 3, Sec. 3.5 Steps 1-2) for gfx950.
//
// This file is compiled without floating-point contraction: the fp64
// reprojection, the Eq. 6-8 extrema and the fp32 interpolation sums are
// evaluated operation by operation in a fixed order, so that their integer
// outcomes (target pixels, hole masks, widths, labels, boxes) are exactly
// reproducible.
#include <algorithm>
#include <cfloat>
#include <climits>

#include "bgs_internal.h"

namespace bgs {

RelPose rel_pose(const bgs_camera& src, const bgs_camera& dst) {
    RelPose P;
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            double p0 = dst.R[0 * 3 + r] * src.R[0 * 3 + q];
            double p1 = dst.R[1 * 3 + r] * src.R[1 * 3 + q];
            double p2 = dst.R[2 * 3 + r] * src.R[2 * 3 + q];
            P.M[r * 3 + q] = (p0 + p1) + p2;
        }
    double d0 = src.t[0] - dst.t[0], d1 = src.t[1] - dst.t[1], d2 = src.t[2] - dst.t[2];
    for (int r = 0; r < 3; ++r) {
        double p0 = dst.R[0 * 3 + r] * d0;
        double p1 = dst.R[1 * 3 + r] * d1;
        double p2 = dst.R[2 * 3 + r] * d2;
        P.c[r] = (p0 + p1) + p2;
    }
    return P;
}

namespace {

// X' = M X (+ c): a source-frame point in the destination frame.
__device__ inline void map_point(const RelPose& P, bool with_t, double X, double Y, double Z, double out[3]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double p0 = P.M[r * 3 + 0] * X;
        double p1 = P.M[r * 3 + 1] * Y;
        double p2 = P.M[r * 3 + 2] * Z;
        double s = (p0 + p1) + p2;
        out[r] = with_t ? s + P.c[r] : s;
    }
}

// Pinhole projection (Eq. 3) in pixels, unrounded.
__device__ inline void project(const WarpCam& c, const double X[3], double* u, double* v) {
    double qx = X[0] / X[2];
    double qy = X[1] / X[2];
    double sx = c.fx * qx;
    double sy = c.fy * qy;
    *u = sx + c.cx;
    *v = sy + c.cy;
}

__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
    return v;
}

// Block-wide reductions for 256-thread blocks; every thread gets the result.
// s4 is a 4-entry LDS scratch that the caller does not touch in between.
__device__ inline uint32_t block_sum_u32(uint32_t v, uint32_t* s4) {
    v = wave_sum_u32(v);
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
    __syncthreads();
    const uint32_t r = s4[0] + s4[1] + s4[2] + s4[3];
    __syncthreads();
    return r;
}
__device__ inline uint32_t block_min_u32(uint32_t v, uint32_t* s4) {
    v = wave_min_u32(v);
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
    __syncthreads();
    const uint32_t r = min(min(s4[0], s4[1]), min(s4[2], s4[3]));
    __syncthreads();
    return r;
}
__device__ inline uint32_t block_max_u32(uint32_t v, uint32_t* s4) {
    v = wave_max_u32(v);
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
    __syncthreads();
    const uint32_t r = max(max(s4[0], s4[1]), max(s4[2], s4[3]));
    __syncthreads();
    return r;
}

// Image kernels in 2D: a 256-thread block covers 64 columns x kBandRows
// rows, a wave per row at a time (coalesced), so no pixel index is divided.
constexpr int kBandRows = 16;
inline dim3 band_grid(int W, int H) { return dim3((unsigned)((W + 63) / 64), (unsigned)((H + kBandRows - 1) / kBandRows)); }

__global__ void k_warp_reset(DevStatus* st) {
    st->n_holes = 0;
    st->n_gap = 0;
    st->n_center = 0;
    st->n_rowfill = 0;
    st->n_boxes = 0;
    st->n_edge = 0;
    st->dmin_inv = 0u;
    st->dmax_bits = 0u;
    st->overflow &= ~2u;
}

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// Where source pixel (i, j) with alpha A and raw depth Dr lands: the
// fixed-order fp64 recipe of Eq. 4-5.  Returns false when it lands nowhere;
// *df gets the fp32 depth proxy of a covered source pixel (else stays
// untouched).
__device__ inline bool splat_target_v(const WarpCam& src, const WarpCam& dst, const RelPose& P, float a_min, float A,
                                      float Dr, int i, int j, int64_t* fu_out, int64_t* fv_out,
                                      unsigned long long* key, float* df_out) {
    const int64_t s = (int64_t)j * src.W + i;
    const double xn = ((double)i - src.cx) / src.fx;
    const double yn = ((double)j - src.cy) / src.fy;
    double Xp[3];
    bool ok;
    float zf;
    if (A >= a_min) {
        const float df = Dr / A;
        *df_out = df;
        const double d = (double)df;
        map_point(P, true, d * xn, d * yn, d, Xp);
        ok = Xp[2] > dst.z_near;
        zf = (float)Xp[2];
    } else {
        map_point(P, false, xn, yn, 1.0, Xp);
        ok = Xp[2] > 0.0;
        zf = INFINITY;
    }
    if (!ok) return false;
    double u, v;
    project(dst, Xp, &u, &v);
    const double fu = floor(u + 0.5), fv = floor(v + 0.5);
    if (!(fu >= 0.0 && fu <= (double)(dst.W - 1) && fv >= 0.0 && fv <= (double)(dst.H - 1))) return false;
    *fu_out = (int64_t)fu;
    *fv_out = (int64_t)fv;
    *key = ((unsigned long long)__float_as_uint(zf) << 32) | (unsigned long long)(uint32_t)s;
    return true;
}
__device__ inline bool splat_target(const WarpCam& src, const WarpCam& dst, const RelPose& P, float a_min,
                                    const float* __restrict__ draw, const float* __restrict__ alpha, int i, int j,
                                    int64_t* fu_out, int64_t* fv_out, unsigned long long* key, float* df_out) {
    const int64_t s = (int64_t)j * src.W + i;
    return splat_target_v(src, dst, P, a_min, alpha[s], draw[s], i, j, fu_out, fv_out, key, df_out);
}

// Forward splat of every source pixel into the destination z-buffer.
__global__ __launch_bounds__(256) void k_reproject_scatter(WarpCam src, WarpCam dst, RelPose P, float a_min,
                                                           const float* __restrict__ draw,
                                                           const float* __restrict__ alpha,
                                                           unsigned long long* __restrict__ zbuf, DevStatus* st) {
    __shared__ uint32_t s4[4];
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    uint32_t dmin = 0xFFFFFFFFu, dmax = 0u;
    for (int r = threadIdx.x >> 6; r < kBandRows; r += 4) {
        const int j = blockIdx.y * kBandRows + r;
        if (i >= src.W || j >= src.H) continue;
        int64_t fu, fv;
        unsigned long long key;
        float df = -1.f;
        const bool hit = splat_target(src, dst, P, a_min, draw, alpha, i, j, &fu, &fv, &key, &df);
        if (df >= 0.f) {
            dmin = min(dmin, __float_as_uint(df));
            dmax = max(dmax, __float_as_uint(df));
        }
        if (hit) atomicMin(&zbuf[fv * dst.W + fu], key);
    }
    dmin = block_min_u32(dmin, s4);
    dmax = block_max_u32(dmax, s4);
    if (threadIdx.x == 0) {
        if (dmin != 0xFFFFFFFFu) atomicMax(&st->dmin_inv, ~dmin);
        if (dmax != 0u) atomicMax(&st->dmax_bits, dmax);
    }
}

// Resolve one destination pixel t from its z-buffer key.
__device__ inline uint32_t resolve_pixel(unsigned long long key, int64_t t, int64_t nd, int64_t ns,
                                         const float* __restrict__ rgb, const float* __restrict__ alpha,
                                         float* __restrict__ rgb_dst, float* __restrict__ z_dst,
                                         float* __restrict__ a_dst, uint8_t* __restrict__ hole) {
    if (key == ~0ull) {
        rgb_dst[t] = 0.f;
        rgb_dst[nd + t] = 0.f;
        rgb_dst[2 * nd + t] = 0.f;
        z_dst[t] = INFINITY;
        a_dst[t] = 0.f;
        hole[t] = 1;
        return 1;
    }
    const uint32_t s = (uint32_t)(key & 0xFFFFFFFFull);
    rgb_dst[t] = rgb[s];
    rgb_dst[nd + t] = rgb[ns + s];
    rgb_dst[2 * nd + t] = rgb[2 * ns + s];
    z_dst[t] = __uint_as_float((uint32_t)(key >> 32));
    a_dst[t] = alpha[s];
    hole[t] = 0;
    return 0;
}

// Row-preserving form (the host has proven that every splat stays on its
// source row, as for a rig that keeps the orientation and moves along x):
// one block of NT threads per row, the row's z-buffer in LDS (64-bit LDS
// atomicMin), the z-test and the resolve in one kernel.  Same recipe, same
// result as the scatter/resolve pair.  Each thread takes kRowPix pixels of a
// chunk of NT * kRowPix and issues all of their loads before any arithmetic,
// so the row's memory latency is paid once per chunk rather than once per
// pixel; the row's four counters are reduced in one LDS exchange.
// kStage: the source row's colour and alpha are loaded with its alpha and
// depth (coalesced, in the same burst) and kept in LDS, so the resolve
// reads them there instead of gathering them from memory after the z-test.
constexpr int kRowThreads = 512, kRowItems = 2;  // threads per row block, pixels per thread per chunk
constexpr int kRowStageLds = 48 * 1024;         // LDS bytes of a staged row block (z row + source row)
constexpr int kRowStageMinW = 1024;             // source rows at least this long are staged
template <int NT, int kRowPix, bool kStage>
__global__ __launch_bounds__(NT) void k_reproject_rows(WarpCam src, WarpCam dst, RelPose P, float a_min,
                                                       const float* __restrict__ draw,
                                                       const float* __restrict__ alpha,
                                                       const float* __restrict__ rgb, float* __restrict__ rgb_dst,
                                                       float* __restrict__ z_dst, float* __restrict__ a_dst,
                                                       uint8_t* __restrict__ hole, uint4* __restrict__ wpart) {
    extern __shared__ unsigned long long zrow[];
    __shared__ uint4 s_red[NT / 64];
    // Staged: the source row's r, g, b and alpha planes follow the z row.
    float* s_src = reinterpret_cast<float*>(zrow + dst.W);
    const int j = blockIdx.x;
    const int64_t ns = (int64_t)src.W * src.H;
    for (int t = threadIdx.x; t < dst.W; t += NT) zrow[t] = ~0ull;
    __syncthreads();
    uint32_t dmin = 0xFFFFFFFFu, dmax = 0u, off_row = 0;
    const int64_t srow = (int64_t)j * src.W;
    for (int base = 0; base < src.W; base += NT * kRowPix) {
        float Av[kRowPix], Dv[kRowPix], Rv[kRowPix], Gv[kRowPix], Bv[kRowPix];
#pragma unroll
        for (int k = 0; k < kRowPix; ++k) {
            const int i = base + threadIdx.x + NT * k;
            Av[k] = i < src.W ? alpha[srow + i] : 0.f;
            Dv[k] = i < src.W ? draw[srow + i] : 0.f;
            if (kStage) {
                Rv[k] = i < src.W ? rgb[srow + i] : 0.f;
                Gv[k] = i < src.W ? rgb[ns + srow + i] : 0.f;
                Bv[k] = i < src.W ? rgb[2 * ns + srow + i] : 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < kRowPix; ++k) {
            const int i = base + threadIdx.x + NT * k;
            if (i >= src.W) continue;
            if (kStage) {
                s_src[i] = Rv[k];
                s_src[src.W + i] = Gv[k];
                s_src[2 * src.W + i] = Bv[k];
                s_src[3 * src.W + i] = Av[k];
            }
            int64_t fu, fv;
            unsigned long long key;
            float df = -1.f;
            const bool hit = splat_target_v(src, dst, P, a_min, Av[k], Dv[k], i, j, &fu, &fv, &key, &df);
            if (df >= 0.f) {
                dmin = min(dmin, __float_as_uint(df));
                dmax = max(dmax, __float_as_uint(df));
            }
            if (hit) {
                if (fv == j) atomicMin(&zrow[fu], key);
                else off_row = 1;
            }
        }
    }
    __syncthreads();
    const int64_t nd = (int64_t)dst.W * dst.H;
    const int64_t drow = (int64_t)j * dst.W;
    uint32_t holes = 0;
    for (int base = 0; base < dst.W; base += NT * kRowPix) {
        unsigned long long kv[kRowPix];
        float c0[kRowPix], c1[kRowPix], c2[kRowPix], av[kRowPix];
#pragma unroll
        for (int k = 0; k < kRowPix; ++k) {
            const int t = base + threadIdx.x + NT * k;
            kv[k] = t < dst.W ? zrow[t] : ~0ull;
            const uint32_t sidx = (uint32_t)(kv[k] & 0xFFFFFFFFull);
            const bool have = kv[k] != ~0ull;
            if (kStage) {
                // A splat of this row comes from this row of the source.
                const int i = have ? (int)((int64_t)sidx - srow) : 0;
                c0[k] = have ? s_src[i] : 0.f;
                c1[k] = have ? s_src[src.W + i] : 0.f;
                c2[k] = have ? s_src[2 * src.W + i] : 0.f;
                av[k] = have ? s_src[3 * src.W + i] : 0.f;
            } else {
                c0[k] = have ? rgb[sidx] : 0.f;
                c1[k] = have ? rgb[ns + sidx] : 0.f;
                c2[k] = have ? rgb[2 * ns + sidx] : 0.f;
                av[k] = have ? alpha[sidx] : 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < kRowPix; ++k) {
            const int t = base + threadIdx.x + NT * k;
            if (t >= dst.W) continue;
            const int64_t g = drow + t;
            const bool have = kv[k] != ~0ull;
            rgb_dst[g] = c0[k];
            rgb_dst[nd + g] = c1[k];
            rgb_dst[2 * nd + g] = c2[k];
            z_dst[g] = have ? __uint_as_float((uint32_t)(kv[k] >> 32)) : INFINITY;
            a_dst[g] = av[k];
            hole[g] = have ? 0 : 1;
            holes += have ? 0u : 1u;
        }
    }
    // The row's partial: max of ~dmin, max of dmax, hole count, off-row flag.
    uint32_t x = wave_max_u32(~dmin), y = wave_max_u32(dmax), h = wave_sum_u32(holes), f = wave_max_u32(off_row);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = make_uint4(x, y, h, f);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint4 r = s_red[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) {
            const uint4 q = s_red[w];
            r.x = max(r.x, q.x);
            r.y = max(r.y, q.y);
            r.z += q.z;
            r.w = max(r.w, q.w);
        }
        // off_row cannot be set when the host's bound holds (overflow bit 2).
        wpart[j] = make_uint4(r.x, r.y, r.z, r.w ? 4u : 0u);
    }
}

// Fold the per-row partials of k_reproject_rows (n of them; none for the
// scatter form, which reduces with atomics) into the status block, from
// every thread of a 256-thread block.  Returns the depth-proxy range of the
// covered pixels, or [z_near, z_far] when none was covered, to every thread.
// The kernel is a single workgroup on the critical path, so its latency is
// what counts: the status words and four partials per thread are loaded
// together, and the four reductions share one barrier.
__device__ inline void fold_warp_parts(const uint4* __restrict__ wpart, int n, DevStatus* st, float z_near,
                                       float z_far, float* r0, float* r1) {
    __shared__ uint4 s_w[4];
    const uint32_t a0 = st->dmin_inv, b0 = st->dmax_bits, h0 = st->n_holes, f0 = st->overflow;
    uint32_t a = 0u, b = 0u, h = 0u, f = 0u;  // 0 is the identity of each fold
    for (int i0 = threadIdx.x; i0 < n; i0 += 1024) {
        uint4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = i0 + 256 * u < n ? wpart[i0 + 256 * u] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a = max(a, q[u].x);
            b = max(b, q[u].y);
            h += q[u].z;
            f |= q[u].w;
        }
    }
    a = wave_max_u32(a);
    b = wave_max_u32(b);
    h = wave_sum_u32(h);
    f = wave_max_u32(f);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = make_uint4(a, b, h, f);
    __syncthreads();
    a = a0;
    b = b0;
    h = 0u;
    f = 0u;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint4 q = s_w[w];
        a = max(a, q.x);
        b = max(b, q.y);
        h += q.z;
        f = max(f, q.w);
    }
    if (threadIdx.x == 0) {
        st->dmin_inv = a;
        st->dmax_bits = b;
        st->n_holes = h0 + h;
        if (f) st->overflow = f0 | f;
    }
    if (a == 0u) {
        *r0 = z_near;
        *r1 = z_far;
    } else {
        *r0 = __uint_as_float(~a);
        *r1 = __uint_as_float(b);
    }
}

__global__ __launch_bounds__(256) void k_reproject_resolve(int64_t nd, int64_t ns,
                                                           const unsigned long long* __restrict__ zbuf,
                                                           const float* __restrict__ rgb,
                                                           const float* __restrict__ alpha,
                                                           float* __restrict__ rgb_dst, float* __restrict__ z_dst,
                                                           float* __restrict__ a_dst, uint8_t* __restrict__ hole,
                                                           DevStatus* st) {
    __shared__ uint32_t s4[4];
    uint32_t h = 0;
    for (int64_t t = (int64_t)blockIdx.x * 1024 + threadIdx.x, e = min(nd, (int64_t)blockIdx.x * 1024 + 1024); t < e;
         t += 256)
        h += resolve_pixel(zbuf[t], t, nd, ns, rgb, alpha, rgb_dst, z_dst, a_dst, hole);
    h = block_sum_u32(h, s4);
    if (threadIdx.x == 0 && h) atomicAdd(&st->n_holes, h);
}

// Standalone reprojection: fold the partials and write the depth range.
__global__ __launch_bounds__(256) void k_warp_finish(const uint4* __restrict__ wpart, int n, DevStatus* st,
                                                     float z_near, float z_far, float* range) {
    float r0, r1;
    fold_warp_parts(wpart, n, st, z_near, z_far, &r0, &r1);
    if (threadIdx.x == 0) {
        range[0] = r0;
        range[1] = r1;
    }
}

// ---------------------------------------------------------------------------
// Step 1: edge ROIs (Eq. 6-8).  One block.
// ---------------------------------------------------------------------------
// Sample k of N along an edge of L pixels: the nearest pixel to
// k (L - 1) / (N - 1), halves rounded down, i.e. floor((2k(L-1) + N-1) /
// (2(N-1))).  The quotient is taken in double (exact operands below 2^53,
// so within one of the floor) and corrected in integers, which costs far
// less than a 64-bit integer division.
__device__ inline int edge_pos(int k, int N, int L) {
    if (N <= 1) return 0;
    const int64_t a = 2 * (int64_t)k * (L - 1) + (N - 1), b = 2 * (int64_t)(N - 1);
    int64_t q = (int64_t)((double)a / (double)b);
    if (q * b > a) --q;
    else if ((q + 1) * b <= a) ++q;
    return (int)q;
}
__device__ inline double snap(double x) {
    double r = rint(x);
    return fabs(x - r) <= 1e-6 ? r : x;
}
__device__ inline double clampd(double x, double a, double b) { return x < a ? a : (x > b ? b : x); }
__device__ inline int64_t align_down(int64_t x, int64_t T) { return (x / T) * T; }
__device__ inline int64_t align_up(int64_t x, int64_t T) { return ((x + T - 1) / T) * T; }

// With tm set, also writes the edge boxes' tiles into the ROI tile mask
// (every tile covered by an edge box is 1, all others 0); k_gap_fill does
// that instead when it runs, over its many workgroups.  depth_range null: the range
// comes from the reprojection just run, whose partials (n_wpart, possibly
// none) it folds into the status block first.
__global__ __launch_bounds__(256) void k_edge_rois(WarpCam src, WarpCam dst, RelPose P, int N, int margin, int T,
                                                   int edge_bounds, const float* __restrict__ depth_range,
                                                   const uint4* __restrict__ wpart, int n_wpart, DevStatus* st,
                                                   bgs_box* boxes, int box_cap, uint8_t* __restrict__ tm) {
    __shared__ double red[8][4];
    __shared__ int32_t sbx[4][6];
    __shared__ int snb;
    float r0, r1;
    if (depth_range) {
        r0 = depth_range[0];
        r1 = depth_range[1];
    } else {
        fold_warp_parts(wpart, n_wpart, st, (float)src.z_near, (float)src.z_far, &r0, &r1);
    }
    const double hyp0 = (double)r0, hyp1 = (double)r1;
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    // Per side, the worst case of its own edge (edge_bounds = 1): largest x
    // of the left edge, smallest x of the right, largest y of the top,
    // smallest y of the bottom.
    double lmax = -INFINITY, rmin = INFINITY, tmax = -INFINITY, bmin = INFINITY;
    const int total = 4 * N;  // N <= 65536
    for (int q = threadIdx.x; q < total; q += 256) {
        const int edge = q / N;
        const int k = q - edge * N;
        int i, j;
        if (edge == 0) { i = edge_pos(k, N, src.W); j = 0; }
        else if (edge == 1) { i = edge_pos(k, N, src.W); j = src.H - 1; }
        else if (edge == 2) { i = 0; j = edge_pos(k, N, src.H); }
        else { i = src.W - 1; j = edge_pos(k, N, src.H); }
        const double xn = ((double)i - src.cx) / src.fx;
        const double yn = ((double)j - src.cy) / src.fy;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double d = h ? hyp1 : hyp0;
            double Xp[3];
            map_point(P, true, d * xn, d * yn, d, Xp);
            if (!(Xp[2] > dst.z_near)) continue;
            double u, v;
            project(dst, Xp, &u, &v);
            xmin = fmin(xmin, u);
            xmax = fmax(xmax, u);
            ymin = fmin(ymin, v);
            ymax = fmax(ymax, v);
            if (edge == 0) tmax = fmax(tmax, v);
            else if (edge == 1) bmin = fmin(bmin, v);
            else if (edge == 2) lmax = fmax(lmax, u);
            else rmin = fmin(rmin, u);
        }
    }
    // min / max are exact in any order: wave shuffles, then the four waves.
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        xmin = fmin(xmin, __shfl_xor(xmin, off, 64));
        xmax = fmax(xmax, __shfl_xor(xmax, off, 64));
        ymin = fmin(ymin, __shfl_xor(ymin, off, 64));
        ymax = fmax(ymax, __shfl_xor(ymax, off, 64));
        lmax = fmax(lmax, __shfl_xor(lmax, off, 64));
        rmin = fmin(rmin, __shfl_xor(rmin, off, 64));
        tmax = fmax(tmax, __shfl_xor(tmax, off, 64));
        bmin = fmin(bmin, __shfl_xor(bmin, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        red[0][w] = xmin;
        red[1][w] = xmax;
        red[2][w] = ymin;
        red[3][w] = ymax;
        red[4][w] = lmax;
        red[5][w] = rmin;
        red[6][w] = tmax;
        red[7][w] = bmin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double rx0 = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
        const double rx1 = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        const double ry0 = fmin(fmin(red[2][0], red[2][1]), fmin(red[2][2], red[2][3]));
        const double ry1 = fmax(fmax(red[3][0], red[3][1]), fmax(red[3][2], red[3][3]));
        const double el = fmax(fmax(red[4][0], red[4][1]), fmax(red[4][2], red[4][3]));
        const double er = fmin(fmin(red[5][0], red[5][1]), fmin(red[5][2], red[5][3]));
        const double et = fmax(fmax(red[6][0], red[6][1]), fmax(red[6][2], red[6][3]));
        const double eb = fmin(fmin(red[7][0], red[7][1]), fmin(red[7][2], red[7][3]));
        const bool pe = edge_bounds != 0;
        const double W = dst.W, H = dst.H, m = margin;
        const double hw = floor(W / 2.0), hh = floor(H / 2.0);
        // A side whose own edge has no valid projection keeps Eq. 6.
        const double umin = snap(pe && el > -INFINITY ? el : rx0), umax = snap(pe && er < INFINITY ? er : rx1);
        const double vmin = snap(pe && et > -INFINITY ? et : ry0), vmax = snap(pe && eb < INFINITY ? eb : ry1);
        const double lw = umin > 0.0 ? clampd(ceil(umin) + m, 0.0, hw) : 0.0;
        const double rw = umax < W - 1.0 ? clampd((W - 1.0) - floor(umax) + m, 0.0, hw) : 0.0;
        const double th = vmin > 0.0 ? clampd(ceil(vmin) + m, 0.0, hh) : 0.0;
        const double bh = vmax < H - 1.0 ? clampd((H - 1.0) - floor(vmax) + m, 0.0, hh) : 0.0;
        const int w4[4] = {(int)lw, (int)rw, (int)th, (int)bh};
        const int64_t Wi = dst.W, Hi = dst.H;
        int nb = 0;
        int32_t (*bx)[6] = sbx;  // LDS: indexed by the running box count
        if (w4[0] > 0) {
            int64_t x1 = align_up(w4[0], T);
            int32_t b[6] = {0, 0, (int32_t)(x1 < Wi ? x1 : Wi), (int32_t)Hi, BGS_BOX_LEFT, -1};
            for (int q = 0; q < 6; ++q) bx[nb][q] = b[q];
            ++nb;
        }
        if (w4[1] > 0) {
            int32_t b[6] = {(int32_t)align_down(Wi - w4[1], T), 0, (int32_t)Wi, (int32_t)Hi, BGS_BOX_RIGHT, -1};
            for (int q = 0; q < 6; ++q) bx[nb][q] = b[q];
            ++nb;
        }
        if (w4[2] > 0) {
            int64_t y1 = align_up(w4[2], T);
            int32_t b[6] = {0, 0, (int32_t)Wi, (int32_t)(y1 < Hi ? y1 : Hi), BGS_BOX_TOP, -1};
            for (int q = 0; q < 6; ++q) bx[nb][q] = b[q];
            ++nb;
        }
        if (w4[3] > 0) {
            int32_t b[6] = {0, (int32_t)align_down(Hi - w4[3], T), (int32_t)Wi, (int32_t)Hi, BGS_BOX_BOTTOM, -1};
            for (int q = 0; q < 6; ++q) bx[nb][q] = b[q];
            ++nb;
        }
        for (int q = 0; q < 4; ++q) st->widths[q] = w4[q];
        st->n_edge = (uint32_t)nb;
        snb = nb;
        for (int b = 0; b < nb; ++b) {
            for (int q = 0; q < 6; ++q) st->edge_boxes[b * 6 + q] = bx[b][q];
            if (b < box_cap) {
                boxes[b].x0 = bx[b][0];
                boxes[b].y0 = bx[b][1];
                boxes[b].x1 = bx[b][2];
                boxes[b].y1 = bx[b][3];
                boxes[b].kind = bx[b][4];
                boxes[b].label = bx[b][5];
            }
        }
    }
    __syncthreads();
    if (!tm) return;  // the gap fill writes the mask
    // The mask: box b covers tile columns [x0 / T, ceil(x1 / T)) and rows
    // [y0 / T, ceil(y1 / T)).  The tile ranges sit in registers (the byte
    // stores could alias LDS through a generic pointer, which would reload
    // them per tile), and a thread takes four consecutive tiles per step,
    // so that one division places them all.
    const int tiles_x = (dst.W + T - 1) / T, n_tiles = tiles_x * ((dst.H + T - 1) / T);
    const int nbx = snb;
    int tr[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const bool on = b < nbx;
        tr[b][0] = on ? sbx[b][0] / T : 0;
        tr[b][1] = on ? sbx[b][1] / T : 0;
        tr[b][2] = on ? (sbx[b][2] + T - 1) / T : 0;
        tr[b][3] = on ? (sbx[b][3] + T - 1) / T : 0;
    }
    for (int t0 = 4 * threadIdx.x; t0 < n_tiles; t0 += 4 * 256) {
        int ty = t0 / tiles_x, tx = t0 - ty * tiles_x;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (t0 + u < n_tiles) {
                bool hit = false;
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    hit = hit || (tx >= tr[b][0] && tx < tr[b][2] && ty >= tr[b][1] && ty < tr[b][3]);
                tm[t0 + u] = hit ? 1 : 0;
            }
            if (++tx == tiles_x) {
                tx = 0;
                ++ty;
            }
        }
    }
}

__device__ inline bool in_edge(const DevStatus* st, int x, int y) {
    const int ne = (int)st->n_edge;
    for (int b = 0; b < ne; ++b) {
        const int32_t* e = st->edge_boxes + b * 6;
        if (x >= e[0] && x < e[2] && y >= e[1] && y < e[3]) return true;
    }
    return false;
}

// The (at most four) edge boxes, read once into registers.
struct EdgeBoxes {
    int n;
    int b[4][4];  // x0, y0, x1, y1
    __device__ explicit EdgeBoxes(const DevStatus* st) {
        n = (int)st->n_edge;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) b[k][q] = st->edge_boxes[k * 6 + q];
    }
    __device__ bool contains(int x, int y) const {
        bool in = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) in = in || (k < n && x >= b[k][0] && x < b[k][2] && y >= b[k][1] && y < b[k][3]);
        return in;
    }
    // Does a box overlap the T x T tile whose first pixel is (x0, y0)?
    __device__ bool overlaps(int x0, int y0, int T) const {
        bool in = false;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            in = in || (k < n && x0 < b[k][2] && b[k][0] < x0 + T && y0 < b[k][3] && b[k][1] < y0 + T);
        return in;
    }
};

// ---------------------------------------------------------------------------
// Gap interpolation, Jacobi passes done in place.  tag[p] = 0 for a pixel
// that was never a hole, k for a hole filled in pass k, 255 for a hole.  In
// pass k a neighbour counts as valid iff its tag is below k, which is the
// state before the pass; a pixel filled in pass k is written only where no
// other pixel of pass k reads it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tag_init(int64_t n, const uint8_t* __restrict__ cls, uint8_t* __restrict__ tag) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) tag[p] = cls[p] ? 255 : 0;
}

__global__ __launch_bounds__(256) void k_gap_pass(int W, int H, int pass, float* rgb, float* z, float* alpha,
                                                  uint8_t* tag, uint8_t* __restrict__ cls, DevStatus* st) {
    __shared__ uint32_t s4[4];
    const int64_t n = (int64_t)W * H;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    uint32_t filled = 0;
    for (int r = threadIdx.x >> 6; r < kBandRows; r += 4) {
        const int y = blockIdx.y * kBandRows + r;
        if (x >= W || y >= H) continue;
        const int64_t p = (int64_t)y * W + x;
        if (tag[p] != 255 || in_edge(st, x, y)) continue;
        {
            const int NX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
            const int NY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
            int cnt = 0;
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, sa = 0.f, zm = -INFINITY;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int xx = x + NX[q], yy = y + NY[q];
                if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                const int64_t r = (int64_t)yy * W + xx;
                if ((int)tag[r] >= pass) continue;  // a hole, or filled in this pass
                s0 = s0 + rgb[r];
                s1 = s1 + rgb[n + r];
                s2 = s2 + rgb[2 * n + r];
                sa = sa + alpha[r];
                const float zr = z[r];
                if (zr > zm) zm = zr;
                ++cnt;
            }
            if (cnt > 0) {
                const float fc = (float)cnt;
                rgb[p] = s0 / fc;
                rgb[n + p] = s1 / fc;
                rgb[2 * n + p] = s2 / fc;
                alpha[p] = sa / fc;
                z[p] = zm;
                tag[p] = (uint8_t)pass;
                cls[p] = (uint8_t)BGS_CLS_GAP;
                ++filled;
            }
        }
    }
    filled = block_sum_u32(filled, s4);
    if (threadIdx.x == 0 && filled) atomicAdd(&st->n_gap, filled);
}

// The same gap passes and the center mask in one kernel: a block loads its
// 64 x kBandRows tile plus a halo of kH >= passes pixels into LDS, runs the
// passes there (pass j is final for pixels at least j from the halo's
// edge, which after all passes includes the tile), and writes the tile's filled
// pixels, tags and center mask.  Per pixel it computes exactly what
// k_tag_init, k_gap_pass and k_center_mask compute.  It also writes the
// ROI tile mask's edge-box tiles (the center boxes are added after it).
// Its filled and center counts go to gpart (one entry per block) rather
// than to shared counters, so that hundreds of blocks do not serialise on
// one cache line; the component-box kernels add them up.
constexpr int kGapMaxHalo = 4;
constexpr uint8_t kTagEdge = 253, kTagOut = 254;

// Workgroups are dispatched to the 8 XCDs in turn (block b to XCD b % 8),
// and each XCD has its own L2.  Tile t of an image's gx * gy tiles is
// given to a block of the XCD that owns its row-major eighth of the tiles,
// so neighbouring tiles, which read each other's edge pixels as halo, are
// mostly read through the same L2.  A bijection of [0, gx * gy).
__device__ inline void xcd_tile(uint32_t b, uint32_t gx, uint32_t gy, int* tx, int* ty) {
    const uint32_t n = gx * gy, q = n / 8, r = n % 8;
    const uint32_t xcd = b % 8, k = b / 8;
    const uint32_t t = xcd * q + min(xcd, r) + k;
    *tx = (int)(t % gx);
    *ty = (int)(t / gx);
}

// kH: the halo the LDS region is sized for (passes <= kH).  1D grid of
// ceil(W / 64) * ceil(H / kBandRows) blocks.
template <int kH>
__global__ __launch_bounds__(256) void k_gap_fill(int W, int H, int passes, float* __restrict__ rgb,
                                                  float* __restrict__ z, float* __restrict__ alpha,
                                                  uint8_t* __restrict__ tag_out, uint8_t* __restrict__ cls,
                                                  uint8_t* __restrict__ center, const DevStatus* st,
                                                  uint2* __restrict__ gpart, int T, int tiles_x, int tiles_y,
                                                  uint8_t* __restrict__ tm) {
    constexpr int RW = 64 + 2 * kH, RH = kBandRows + 2 * kH;
    __shared__ float s_c[3][RH * RW];
    __shared__ float s_a[RH * RW], s_z[RH * RW];
    // Tag per pixel: 0 no hole, k a hole filled in pass k, 255 a hole still
    // open, kTagEdge a hole inside an edge ROI (never filled), kTagOut
    // outside the image.  In pass k a neighbour is valid iff its tag is
    // below k.
    __shared__ uint8_t s_tag[RH * RW];
    __shared__ uint16_t s_hl[RH * RW];  // the open holes one pixel or more inside the region
    __shared__ uint32_t s_nh;
    __shared__ uint32_t s4[4];
    const uint32_t gx = (uint32_t)(W + 63) / 64, gy = (uint32_t)(H + kBandRows - 1) / kBandRows;
    int bx, by;
    xcd_tile(blockIdx.x, gx, gy, &bx, &by);
    const uint32_t gb = (uint32_t)by * gx + (uint32_t)bx;
    const int64_t n = (int64_t)W * H;
    // The halo is kH pixels whatever the number of passes: a wider halo
    // changes nothing inside the tile (pass j is final for the pixels j or
    // more from the region's edge).
    const int x0 = bx * 64 - kH, y0 = by * kBandRows - kH;
    const EdgeBoxes eb(st);
    if (threadIdx.x == 0) s_nh = 0;
    {
        // The edge ROIs in the tile mask: the tiles whose first pixel lies
        // in this block's region (so each tile is written by one block).
        const int rx = bx * 64, ry = by * kBandRows;
        const int tx0 = (rx + T - 1) / T, tx1 = min(tiles_x, (rx + 64 + T - 1) / T);
        const int ty0 = (ry + T - 1) / T, ty1 = min(tiles_y, (ry + kBandRows + T - 1) / T);
        const int ntx = tx1 - tx0, nty = ty1 - ty0;
        for (int k = threadIdx.x; ntx > 0 && k < ntx * nty; k += 256) {
            const int ty = ty0 + k / ntx, tx = tx0 + k % ntx;
            tm[(int64_t)ty * tiles_x + tx] = eb.overlaps(tx * T, ty * T, T) ? 1 : 0;
        }
    }
    {
        // Holes are sparse: a tile without one has nothing to fill and no
        // center pixel, and needs none of its neighbours' values.  (The
        // loads are issued together: unrolled, none waits on another.)
        const int cx = bx * 64 + (threadIdx.x & 63);
        uint8_t hv[kBandRows / 4];
#pragma unroll
        for (int q = 0; q < kBandRows / 4; ++q) {
            const int cy = by * kBandRows + (threadIdx.x >> 6) + 4 * q;
            hv[q] = (cx < W && cy < H) ? cls[(int64_t)cy * W + cx] : 0;
        }
        bool any = false;
#pragma unroll
        for (int q = 0; q < kBandRows / 4; ++q) any = any || hv[q] != 0;
        if (!__syncthreads_or(any)) {
            for (int r = threadIdx.x >> 6; r < kBandRows; r += 4) {
                const int cy = by * kBandRows + r;
                if (cx < W && cy < H) {
                    tag_out[(int64_t)cy * W + cx] = 0;
                    center[(int64_t)cy * W + cx] = 0;
                }
            }
            if (threadIdx.x == 0) gpart[gb] = make_uint2(0u, 0u);
            return;
        }
    }
    // The tile and its halo: all loads first (unrolled, so none waits on
    // another), then the LDS stores.
    constexpr int kLoads = (RW * RH + 255) / 256;
    float lc0[kLoads], lc1[kLoads], lc2[kLoads], la[kLoads], lz[kLoads];
    uint8_t lh[kLoads];
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int lx = i % RW, ly = i / RW, x = x0 + lx, y = y0 + ly;
        const bool ok = i < RW * RH && x >= 0 && y >= 0 && x < W && y < H;
        const int64_t p = ok ? (int64_t)y * W + x : 0;
        lh[q] = ok ? cls[p] : 0;
        lc0[q] = ok ? rgb[p] : 0.f;
        lc1[q] = ok ? rgb[n + p] : 0.f;
        lc2[q] = ok ? rgb[2 * n + p] : 0.f;
        la[q] = ok ? alpha[p] : 0.f;
        lz[q] = ok ? z[p] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
        const int i = threadIdx.x + 256 * q;
        if (i >= RW * RH) continue;
        const int lx = i % RW, ly = i / RW, x = x0 + lx, y = y0 + ly;
        if (x < 0 || y < 0 || x >= W || y >= H) {
            s_tag[i] = kTagOut;
            continue;
        }
        s_tag[i] = lh[q] == 0 ? 0 : eb.contains(x, y) ? kTagEdge : 255;
        s_c[0][i] = lc0[q];
        s_c[1][i] = lc1[q];
        s_c[2][i] = lc2[q];
        s_a[i] = la[q];
        s_z[i] = lz[q];
    }
    __syncthreads();
    // The open holes, listed once (in no particular order: a pass reads
    // only tags below its own number, so its pixels are independent), so
    // that the passes visit nothing else.
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int lx = i % RW, ly = i / RW;
        const bool open = i < RW * RH && lx >= 1 && lx < RW - 1 && ly >= 1 && ly < RH - 1 && s_tag[i] == 255;
        const unsigned long long bal = __ballot(open);
        const int lane = threadIdx.x & 63;
        uint32_t base = 0;
        if (lane == 0 && bal) base = atomicAdd(&s_nh, (uint32_t)__popcll(bal));
        base = __shfl(base, 0, 64);
        if (open) s_hl[base + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)i;
    }
    __syncthreads();
    const int nh = (int)s_nh;
    for (int pass = 1; pass <= passes; ++pass) {
        for (int e = threadIdx.x; e < nh; e += 256) {
            const int li = s_hl[e];
            const int ly = li / RW, lx = li - ly * RW;
            // pixels at least `pass` from the region's edge, not yet filled
            if (lx < pass || lx >= RW - pass || ly < pass || ly >= RH - pass || s_tag[li] != 255) continue;
            const int NX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
            const int NY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
            // All eight neighbours' values are read together (no read waits
            // on another), then the valid ones are summed in neighbour order.
            bool ok[8];
            float v0[8], v1[8], v2[8], va[8], vz[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int r = (ly + NY[q]) * RW + lx + NX[q];
                ok[q] = (int)s_tag[r] < pass;  // not outside, not a hole, not filled in this pass
                v0[q] = s_c[0][r];
                v1[q] = s_c[1][r];
                v2[q] = s_c[2][r];
                va[q] = s_a[r];
                vz[q] = s_z[r];
            }
            int cnt = 0;
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, sa = 0.f, zm = -INFINITY;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (!ok[q]) continue;
                s0 = s0 + v0[q];
                s1 = s1 + v1[q];
                s2 = s2 + v2[q];
                sa = sa + va[q];
                if (vz[q] > zm) zm = vz[q];
                ++cnt;
            }
            if (cnt > 0) {
                const float fc = (float)cnt;
                s_c[0][li] = s0 / fc;
                s_c[1][li] = s1 / fc;
                s_c[2][li] = s2 / fc;
                s_a[li] = sa / fc;
                s_z[li] = zm;
                s_tag[li] = (uint8_t)pass;
            }
        }
        __syncthreads();
    }
    uint32_t filled = 0, centers = 0;
    for (int i = threadIdx.x; i < 64 * kBandRows; i += 256) {
        const int lx = kH + (i & 63), ly = kH + (i >> 6), x = x0 + lx, y = y0 + ly;
        if (x >= W || y >= H) continue;
        const int li = ly * RW + lx;
        const int64_t p = (int64_t)y * W + x;
        const uint8_t t = s_tag[li];
        tag_out[p] = t >= kTagEdge ? 255 : t;
        if (t != 0 && t < kTagEdge) {
            rgb[p] = s_c[0][li];
            rgb[n + p] = s_c[1][li];
            rgb[2 * n + p] = s_c[2][li];
            alpha[p] = s_a[li];
            z[p] = s_z[li];
            cls[p] = (uint8_t)BGS_CLS_GAP;
            ++filled;
        }
        const uint32_t c = t == 255 ? 1u : 0u;
        center[p] = (uint8_t)c;
        centers += c;
    }
    filled = block_sum_u32(filled, s4);
    centers = block_sum_u32(centers, s4);
    if (threadIdx.x == 0) gpart[gb] = make_uint2(filled, centers);
}

// Holes left after interpolation and outside the edge ROIs.
__global__ __launch_bounds__(256) void k_center_mask(int W, int H, const uint8_t* __restrict__ tag,
                                                     uint8_t* __restrict__ center, DevStatus* st) {
    __shared__ uint32_t s4[4];
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    uint32_t count = 0;
    for (int r = threadIdx.x >> 6; r < kBandRows; r += 4) {
        const int y = blockIdx.y * kBandRows + r;
        if (x >= W || y >= H) continue;
        const int64_t p = (int64_t)y * W + x;
        const uint32_t c = (tag[p] == 255 && !in_edge(st, x, y)) ? 1u : 0u;
        center[p] = (uint8_t)c;
        count += c;
    }
    count = block_sum_u32(count, s4);
    if (threadIdx.x == 0 && count) atomicAdd(&st->n_center, count);
}

// ---------------------------------------------------------------------------
// Row fill (center step off): nearest non-hole pixel left and right on the
// row via block max/min scans; the farther candidate wins.  One block/row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_row_fill(int W, int H, const uint8_t* __restrict__ tag,
                                                  const uint8_t* __restrict__ center, float bg0, float bg1, float bg2,
                                                  float* __restrict__ rgb, float* __restrict__ z,
                                                  float* __restrict__ alpha, uint8_t* __restrict__ cls,
                                                  DevStatus* st) {
    __shared__ int s_left[256], s_right[256];
    const int y = blockIdx.x;
    const int64_t n = (int64_t)W * H;
    const int64_t row = (int64_t)y * W;
    const int chunk = (W + 255) / 256;
    const int xa = threadIdx.x * chunk, xb = min(xa + chunk, W);
    int last = -1, first = INT_MAX;
    for (int x = xa; x < xb; ++x)
        if (tag[row + x] != 255) {
            last = x;
            if (first == INT_MAX) first = x;
        }
    s_left[threadIdx.x] = last;
    s_right[threadIdx.x] = first;
    __syncthreads();
    // Inclusive scans: max from the left, min from the right.
    for (int off = 1; off < 256; off <<= 1) {
        int l = (int)threadIdx.x >= off ? s_left[threadIdx.x - off] : -1;
        int r = (int)threadIdx.x + off < 256 ? s_right[threadIdx.x + off] : INT_MAX;
        __syncthreads();
        s_left[threadIdx.x] = max(s_left[threadIdx.x], l);
        s_right[threadIdx.x] = min(s_right[threadIdx.x], r);
        __syncthreads();
    }
    int left = threadIdx.x > 0 ? s_left[threadIdx.x - 1] : -1;
    const int right_after = threadIdx.x < 255 ? s_right[threadIdx.x + 1] : INT_MAX;
    uint32_t filled = 0;
    // Nearest valid to the right of x inside the chunk, else right_after.
    for (int x = xa; x < xb; ++x) {
        const int64_t p = row + x;
        if (center[p]) {
            int right = right_after;
            for (int xx = x + 1; xx < xb; ++xx)
                if (tag[row + xx] != 255) {
                    right = xx;
                    break;
                }
            int pick = -1;
            if (left >= 0 && right != INT_MAX) pick = z[row + right] > z[row + left] ? right : left;
            else if (left >= 0) pick = left;
            else if (right != INT_MAX) pick = right;
            if (pick >= 0) {
                const int64_t r = row + pick;
                rgb[p] = rgb[r];
                rgb[n + p] = rgb[n + r];
                rgb[2 * n + p] = rgb[2 * n + r];
                z[p] = z[r];
                alpha[p] = alpha[r];
            } else {
                rgb[p] = bg0;
                rgb[n + p] = bg1;
                rgb[2 * n + p] = bg2;
                z[p] = INFINITY;
                alpha[p] = 0.f;
            }
            cls[p] = (uint8_t)BGS_CLS_ROWFILL;
            ++filled;
        }
        if (tag[p] != 255) left = x;
    }
    __shared__ uint32_t s4[4];
    filled = block_sum_u32(filled, s4);
    if (threadIdx.x == 0 && filled) atomicAdd(&st->n_rowfill, filled);
}

// ---------------------------------------------------------------------------
// Connected components: block-local union-find in LDS over 16x16 pixel
// blocks, then unions across block borders with global atomicMin, then
// flattening.  Links always go from the larger to the smaller index, so the
// root of every component is its smallest linear index.
// ---------------------------------------------------------------------------
__device__ inline int find_root_lds(int* L, int x) {
    int p = __atomic_load_n(&L[x], __ATOMIC_RELAXED);
    while (p != x) {
        x = p;
        p = __atomic_load_n(&L[x], __ATOMIC_RELAXED);
    }
    return x;
}

__device__ inline int find_root_g(int* L, int x) {
    int p = __atomic_load_n(&L[x], __ATOMIC_RELAXED);
    while (p != x) {
        x = p;
        p = __atomic_load_n(&L[x], __ATOMIC_RELAXED);
    }
    return x;
}

__device__ inline void unite_g(int* L, int a, int b) {
    while (true) {
        a = find_root_g(L, a);
        b = find_root_g(L, b);
        if (a == b) return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(&L[a], b);
        if (old == a) return;
        a = old;  // a had gained a parent meanwhile; unite that one with b
    }
}

__device__ inline void unite_lds(int* L, int a, int b) {
    while (true) {
        a = find_root_lds(L, a);
        b = find_root_lds(L, b);
        if (a == b) return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(&L[a], b);
        if (old == a) return;
        a = old;
    }
}

// Block-local labelling of a 16x16 pixel block.  With pflag/pbox given, it
// also records every block-local piece (its root pixel gets pflag = 1 and
// the piece's half-open bounding box in pbox), so that component boxes can
// be formed from pieces instead of pixels.
__global__ __launch_bounds__(256) void k_ccl_local(int W, int H, int conn, const uint8_t* __restrict__ mask,
                                                   int* __restrict__ labels, uint8_t* __restrict__ pflag,
                                                   int4* __restrict__ pbox) {
    __shared__ int L[256];
    __shared__ uint8_t m[256];
    __shared__ int bx0[256], by0[256], bx1[256], by1[256];
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = blockIdx.x * 16 + lx, y = blockIdx.y * 16 + ly;
    const bool in = x < W && y < H;
    const int li = threadIdx.x;
    const bool set = in && mask[(int64_t)y * W + x];
    if (!__syncthreads_or(set)) {  // an empty block (the usual case for a sparse mask)
        if (in) {
            labels[(int64_t)y * W + x] = -1;
            if (pflag) pflag[(int64_t)y * W + x] = 0;
        }
        return;
    }
    m[li] = set ? 1 : 0;
    L[li] = li;
    bx0[li] = INT_MAX;
    by0[li] = INT_MAX;
    bx1[li] = -1;
    by1[li] = -1;
    __syncthreads();
    if (set) {
        // Backward neighbours inside the block: left, up-left, up, up-right.
        if (lx > 0 && m[li - 1]) unite_lds(L, li, li - 1);
        if (ly > 0) {
            if (m[li - 16]) unite_lds(L, li, li - 16);
            if (conn == 8) {
                if (lx > 0 && m[li - 17]) unite_lds(L, li, li - 17);
                if (lx < 15 && m[li - 15]) unite_lds(L, li, li - 15);
            }
        }
    }
    __syncthreads();
    int r = -1;
    if (set) {
        r = find_root_lds(L, li);
        if (pbox) {
            atomicMin(&bx0[r], x);
            atomicMin(&by0[r], y);
            atomicMax(&bx1[r], x + 1);
            atomicMax(&by1[r], y + 1);
        }
    }
    __syncthreads();
    if (!in) return;
    const int64_t g = (int64_t)y * W + x;
    if (set) {
        const int rx = blockIdx.x * 16 + (r & 15), ry = blockIdx.y * 16 + (r >> 4);
        labels[g] = ry * W + rx;
    } else {
        labels[g] = -1;
    }
    if (pflag) {
        const bool root = set && r == li;
        pflag[g] = root ? 1 : 0;
        if (root) pbox[g] = make_int4(bx0[li], by0[li], bx1[li], by1[li]);
    }
}

__global__ __launch_bounds__(256) void k_ccl_border(int W, int H, int conn, const uint8_t* __restrict__ mask,
                                                    int* labels) {
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = blockIdx.x * 16 + lx, y = blockIdx.y * 16 + ly;
    if (x >= W || y >= H) return;
    if (!(lx == 0 || ly == 0 || lx == 15)) return;
    const int64_t p = (int64_t)y * W + x;
    if (!mask[p]) return;
    const int me = (int)p;
    // Neighbours in another block (the rest were joined in LDS).
    if (lx == 0 && x > 0 && mask[p - 1]) unite_g(labels, me, me - 1);
    if (y > 0) {
        if (ly == 0 && mask[p - W]) unite_g(labels, me, me - W);
        if (conn == 8) {
            if (x > 0 && (lx == 0 || ly == 0) && mask[p - W - 1]) unite_g(labels, me, me - W - 1);
            if (x + 1 < W && (lx == 15 || ly == 0) && mask[p - W + 1]) unite_g(labels, me, me - W + 1);
        }
    }
}

__global__ __launch_bounds__(256) void k_ccl_flatten(int64_t n, int* labels) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const int l = labels[p];
    if (l < 0) return;
    labels[p] = find_root_g(labels, l);
}

// ---------------------------------------------------------------------------
// Center boxes.  Component c (in order of root pixel) gets box slot
// n_edge + c.  A component's root is its smallest pixel index, so the
// component roots are the pixels with labels[p] == p; slot_of() ranks a
// root among them from per-block root counts (scanned) and per-block root
// masks, so no per-pixel slot map is needed.
// ---------------------------------------------------------------------------
constexpr int kBoxWords = 8;  // per component: x0, y0, x1, y1, root pixel, pad

// Flatten every label to its root (as k_ccl_flatten) and record, per
// 256-pixel block of the flatten grid, the mask of component roots and its
// population.
__global__ __launch_bounds__(256) void k_ccl_flatten_roots(int64_t n, int* labels, uint32_t* __restrict__ bcount,
                                                           uint32_t* __restrict__ rmask) {
    __shared__ uint32_t cnt[4];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool root = false;
    if (p < n) {
        const int l = labels[p];
        if (l >= 0) {
            root = l == (int)p;
            if (!root) labels[p] = find_root_g(labels, l);
        }
    }
    const unsigned long long m = __ballot(root);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        rmask[(size_t)blockIdx.x * 8 + 2 * w] = (uint32_t)m;
        rmask[(size_t)blockIdx.x * 8 + 2 * w + 1] = (uint32_t)(m >> 32);
        cnt[w] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// One workgroup: the gap-fill counts, an exclusive scan of the nb block
// counts in place (bcount[nb] gets the component count), the box count and
// capacity flag, and the initial (empty) box of every component.
// Adds the gap-fill block counts (n_gpart entries) to the status block.  The
// status words are read first and up to four partials per thread are
// loaded together: this runs on one workgroup, where load latency is most
// of the time.
__device__ inline void fold_gap_parts(const uint2* __restrict__ gpart, int n_gpart, DevStatus* st) {
    __shared__ uint32_t s_g[2][16];
    const uint32_t g0 = st->n_gap, c0 = st->n_center;
    uint32_t f = 0u, c = 0u;
    const int nt = (int)blockDim.x;
    for (int i0 = threadIdx.x; i0 < n_gpart; i0 += 4 * nt) {
        uint2 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = i0 + u * nt < n_gpart ? gpart[i0 + u * nt] : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            f += q[u].x;
            c += q[u].y;
        }
    }
    f = wave_sum_u32(f);
    c = wave_sum_u32(c);
    if ((threadIdx.x & 63) == 0) {
        s_g[0][threadIdx.x >> 6] = f;
        s_g[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tf = 0u, tc = 0u;
        for (int w = 0; w < nt / 64; ++w) {
            tf += s_g[0][w];
            tc += s_g[1][w];
        }
        st->n_gap = g0 + tf;
        st->n_center = c0 + tc;
    }
}

// Block counts up to kRootLds are staged in LDS with coalesced loads (all
// issued together), scanned there and written back coalesced; larger
// images walk per-thread chunks in global memory.
constexpr int kRootLds = 16384;

__global__ __launch_bounds__(1024) void k_root_scan(int64_t nb, uint32_t* bcount, int32_t* __restrict__ bbox,
                                                    int box_cap, int32_t* __restrict__ n_boxes,
                                                    const uint2* __restrict__ gpart, int n_gpart, DevStatus* st) {
    __shared__ uint32_t s_cnt[kRootLds];
    __shared__ uint32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t n_edge = st->n_edge;
    const bool staged = nb <= kRootLds;
    if (staged) {
        constexpr int kU = kRootLds / 1024;
        uint32_t v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = tid + 1024 * u < nb ? bcount[tid + 1024 * u] : 0u;
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (tid + 1024 * u < nb) s_cnt[tid + 1024 * u] = v[u];
    }
    fold_gap_parts(gpart, n_gpart, st);  // its barrier also publishes s_cnt
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = min(nb, (int64_t)tid * per), b1 = min(nb, b0 + per);
    uint32_t sum = 0;
    if (staged)
        for (int64_t b = b0; b < b1; ++b) sum += s_cnt[b];
    else
        for (int64_t b = b0; b < b1; ++b) sum += bcount[b];
    // Exclusive scan of the 1024 chunk sums: within each wave by shuffles,
    // then over the 16 wave totals.
    uint32_t x = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t run = x - sum, total = 0;
    for (int w = 0; w < 16; ++w) {
        const uint32_t ws = wsum[w];
        if (w < wave) run += ws;
        total += ws;
    }
    if (staged) {
        for (int64_t b = b0; b < b1; ++b) {
            const uint32_t c = s_cnt[b];
            s_cnt[b] = run;
            run += c;
        }
        __syncthreads();
        for (int64_t b = tid; b < nb; b += 1024) bcount[b] = s_cnt[b];
    } else {
        for (int64_t b = b0; b < b1; ++b) {
            const uint32_t c = bcount[b];
            bcount[b] = run;
            run += c;
        }
    }
    if (tid == 0) {
        bcount[nb] = total;
        const uint32_t tot = n_edge + total;
        st->n_boxes = tot;
        if ((int64_t)tot > box_cap) atomicOr(&st->overflow, 2u);
        *n_boxes = (int32_t)tot;
    }
    for (uint32_t c = tid; c < total; c += 1024) {
        int32_t* e = bbox + (size_t)c * kBoxWords;
        e[0] = INT_MAX;
        e[1] = INT_MAX;
        e[2] = -1;
        e[3] = -1;
        e[4] = -1;
    }
}

// Rank of component root r among all roots, in pixel order.
__device__ inline uint32_t slot_of(int r, const uint32_t* __restrict__ boff, const uint32_t* __restrict__ rmask) {
    const uint32_t blk = (uint32_t)r >> 8, bit = (uint32_t)r & 255u;
    const uint32_t* m = rmask + (size_t)blk * 8;
    uint32_t rank = boff[blk];
    for (uint32_t q = 0; q < (bit >> 5); ++q) rank += __popc(m[q]);
    const uint32_t low = bit & 31u;
    if (low) rank += __popc(m[bit >> 5] & ((1u << low) - 1u));
    return rank;
}

// Component boxes from the block-local pieces: 4 atomics per piece; the
// piece that holds the component root records it.
__global__ __launch_bounds__(256) void k_bbox_acc(int64_t n, const int* __restrict__ labels,
                                                  const uint8_t* __restrict__ pflag, const int4* __restrict__ pbox,
                                                  const uint32_t* __restrict__ boff, const uint32_t* __restrict__ rmask,
                                                  int32_t* bbox) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n || !pflag[p]) return;
    const int r = labels[p];
    int32_t* e = bbox + (size_t)slot_of(r, boff, rmask) * kBoxWords;
    const int4 b = pbox[p];
    atomicMin(&e[0], b.x);
    atomicMin(&e[1], b.y);
    atomicMax(&e[2], b.z);
    atomicMax(&e[3], b.w);
    if (r == (int)p) e[4] = r;
}

// One workgroup per component (grid-stride over the component count):
// margin, clip, tile alignment, the box record, and its tiles in the mask.
__global__ __launch_bounds__(256) void k_center_boxes(int W, int H, int margin, int T, int tiles_x,
                                                      const uint32_t* __restrict__ ncomp,
                                                      const int32_t* __restrict__ bbox, bgs_box* __restrict__ boxes,
                                                      int box_cap, uint8_t* tm, const DevStatus* st) {
    const uint32_t total = *ncomp;
    for (uint32_t c = blockIdx.x; c < total; c += gridDim.x) {
        const int32_t* e = bbox + (size_t)c * kBoxWords;
        int64_t x0 = e[0] - margin, y0 = e[1] - margin;
        int64_t x1 = e[2] + margin, y1 = e[3] + margin;
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > W) x1 = W;
        if (y1 > H) y1 = H;
        x0 = align_down(x0, T);
        y0 = align_down(y0, T);
        x1 = align_up(x1, T);
        y1 = align_up(y1, T);
        if (x1 > W) x1 = W;
        if (y1 > H) y1 = H;
        if (threadIdx.x == 0) {
            const int64_t slot = (int64_t)st->n_edge + c;
            if (slot < box_cap) {
                boxes[slot].x0 = (int32_t)x0;
                boxes[slot].y0 = (int32_t)y0;
                boxes[slot].x1 = (int32_t)x1;
                boxes[slot].y1 = (int32_t)y1;
                boxes[slot].kind = BGS_BOX_CENTER;
                boxes[slot].label = e[4];
            }
        }
        const int64_t tx0 = x0 / T, ty0 = y0 / T;
        const int64_t bw = (x1 + T - 1) / T - tx0, bh = (y1 + T - 1) / T - ty0;
        for (int64_t q = threadIdx.x; q < bw * bh; q += 256) tm[(ty0 + q / bw) * tiles_x + tx0 + q % bw] = 1;
    }
}

// Box count without center ROIs: the edge boxes only.  256 threads.
__global__ __launch_bounds__(256) void k_box_count(int box_cap, int32_t* n_boxes, const uint2* __restrict__ gpart,
                                                   int n_gpart, DevStatus* st) {
    fold_gap_parts(gpart, n_gpart, st);
    if (threadIdx.x != 0) return;
    const uint32_t tot = st->n_edge;
    st->n_boxes = tot;
    if ((int64_t)tot > box_cap) st->overflow |= 2u;
    *n_boxes = (int32_t)tot;
}

__global__ __launch_bounds__(256) void k_fill_i32(int64_t n, int32_t* p, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned grid(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// True when every splat provably stays on its source row: same row count,
// same fy and cy, and the fp64 bound on |v - j| over the image for any valid
// depth is below a quarter pixel.  With M = I + E (|E| <= eps) and a point
// at depth d >= d_lo, v - j = fy (num / den) with
// |num| <= g + |c1|/d_lo + |yn| (g + |c2|/d_lo), den >= 1 - g - |c2|/d_lo,
// g = eps (|xn| + |yn| + 1); valid splats need Z' > z_near, hence d_lo.
static bool rows_preserved(const WarpCam& src, const WarpCam& dst, const RelPose& P) {
    if (src.H != dst.H || src.fy != dst.fy || src.cy != dst.cy || dst.W > 8192) return false;
    double eps = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) eps = fmax(eps, fabs(P.M[r * 3 + q] - (r == q ? 1.0 : 0.0)));
    const double xn = fmax(fabs(0.0 - src.cx), fabs((src.W - 1.0) - src.cx)) / src.fx;
    const double yn = fmax(fabs(0.0 - src.cy), fabs((src.H - 1.0) - src.cy)) / src.fy;
    const double g = eps * (xn + yn + 1.0);
    const double d_lo = (dst.z_near - fabs(P.c[2])) / (1.0 + g);
    if (!(d_lo > 0.0)) return false;
    const double c1 = fabs(P.c[1]) / d_lo, c2 = fabs(P.c[2]) / d_lo;
    const double den = 1.0 - g - c2;
    if (!(den > 0.5)) return false;
    const double bound = dst.fy * (g + c1 + yn * (g + c2)) / den + 1e-9 * (dst.H + 1.0);
    return bound < 0.25;
}

int warp_parts(const WarpCam& src, const WarpCam& dst, const RelPose& P) {
    return rows_preserved(src, dst, P) ? dst.H : 0;
}

hipError_t launch_reproject(const WarpCam& src, const WarpCam& dst, const RelPose& P, float a_min, const float* rgb,
                            const float* draw, const float* alpha, unsigned long long* zbuf, float* rgb_dst,
                            float* z_dst, float* alpha_dst, uint8_t* hole, float* depth_range, bool reset,
                            uint4* wpart, DevStatus* st, hipStream_t s) {
    const int64_t ns = (int64_t)src.W * src.H, nd = (int64_t)dst.W * dst.H;
    if (reset) hipLaunchKernelGGL(k_warp_reset, dim3(1), dim3(1), 0, s, st);
    if (rows_preserved(src, dst, P)) {
        // Staging pays on long rows (1600 pixels: 20.6 -> 19.5 us); on short
        // ones the larger LDS footprint costs more than the gathers it saves
        // (800 pixels: 8.2 -> 9.0 us).
        const size_t zb = sizeof(unsigned long long) * dst.W, sb = zb + 4 * sizeof(float) * src.W;
        if (src.W >= kRowStageMinW && sb <= (size_t)kRowStageLds)
            hipLaunchKernelGGL((k_reproject_rows<kRowThreads, kRowItems, true>), dim3(dst.H), dim3(kRowThreads), sb, s,
                               src, dst, P, a_min, draw, alpha, rgb, rgb_dst, z_dst, alpha_dst, hole, wpart);
        else
            hipLaunchKernelGGL((k_reproject_rows<kRowThreads, kRowItems, false>), dim3(dst.H), dim3(kRowThreads), zb,
                               s, src, dst, P, a_min, draw, alpha, rgb, rgb_dst, z_dst, alpha_dst, hole, wpart);
    } else {
        hipLaunchKernelGGL(k_fill_u64, dim3(grid(nd)), dim3(256), 0, s, zbuf, nd, ~0ull);
        hipLaunchKernelGGL(k_reproject_scatter, band_grid(src.W, src.H), dim3(256), 0, s, src, dst, P, a_min, draw,
                           alpha, zbuf, st);
        hipLaunchKernelGGL(k_reproject_resolve, dim3((unsigned)((nd + 1023) / 1024)), dim3(256), 0, s, nd, ns, zbuf, rgb,
                           alpha, rgb_dst, z_dst, alpha_dst, hole, st);
    }
    if (depth_range)
        hipLaunchKernelGGL(k_warp_finish, dim3(1), dim3(256), 0, s, wpart, warp_parts(src, dst, P), st,
                           (float)src.z_near, (float)src.z_far, depth_range);
    return hipGetLastError();
}

static hipError_t label_components(const uint8_t* mask, int W, int H, int conn, int32_t* labels, uint8_t* pflag,
                                   int4* pbox, hipStream_t s) {
    const int64_t n = (int64_t)W * H;
    if (n == 0) return hipSuccess;
    dim3 g((W + 15) / 16, (H + 15) / 16);
    hipLaunchKernelGGL(k_ccl_local, g, dim3(256), 0, s, W, H, conn, mask, labels, pflag, pbox);
    hipLaunchKernelGGL(k_ccl_border, g, dim3(256), 0, s, W, H, conn, mask, labels);
    hipLaunchKernelGGL(k_ccl_flatten, dim3(grid(n)), dim3(256), 0, s, n, labels);
    return hipGetLastError();
}

hipError_t launch_label_components(const uint8_t* mask, int W, int H, int conn, int32_t* labels, hipStream_t s) {
    return label_components(mask, W, H, conn, labels, nullptr, nullptr, s);
}

hipError_t launch_classify(const WarpCam& src, const WarpCam& dst, const RelPose& P, const bgs_roi_params& roi,
                           const float bg[3], const float* depth_range, float* rgb, float* z, float* alpha,
                           uint8_t* cls, int32_t* labels, bgs_box* boxes, int32_t box_cap, int32_t* n_boxes,
                           uint8_t* tile_mask, const ClassifyBufs& b, DevStatus* st, hipStream_t s) {
    const int W = dst.W, H = dst.H, T = roi.tile;
    const int64_t n = (int64_t)W * H;
    const int tiles_x = (W + T - 1) / T, tiles_y = (H + T - 1) / T;
    const bool fused = roi.gap_passes <= kGapMaxHalo;  // k_gap_fill writes the edge tiles of the mask
    hipLaunchKernelGGL(k_edge_rois, dim3(1), dim3(256), 0, s, src, dst, P, roi.edge_samples, roi.margin, T,
                       roi.edge_bounds, depth_range, b.wpart, depth_range ? 0 : warp_parts(src, dst, P), st, boxes, box_cap,
                       fused ? nullptr : tile_mask);
    const dim3 gg = band_grid(W, H);
    int n_gpart = 0;
    uint8_t* tag = b.hole;
    uint8_t* center = b.hole2;
    if (fused) {
        const dim3 g1(gg.x * gg.y);
        if (roi.gap_passes <= 2)
            hipLaunchKernelGGL(k_gap_fill<2>, g1, dim3(256), 0, s, W, H, roi.gap_passes, rgb, z, alpha, tag, cls,
                               center, st, b.gpart, T, tiles_x, tiles_y, tile_mask);
        else
            hipLaunchKernelGGL(k_gap_fill<kGapMaxHalo>, g1, dim3(256), 0, s, W, H, roi.gap_passes, rgb, z, alpha, tag,
                               cls, center, st, b.gpart, T, tiles_x, tiles_y, tile_mask);
        n_gpart = (int)(gg.x * gg.y);
    } else {
        hipLaunchKernelGGL(k_tag_init, dim3(grid(n)), dim3(256), 0, s, n, cls, tag);
        for (int pass = 1; pass <= roi.gap_passes; ++pass)
            hipLaunchKernelGGL(k_gap_pass, band_grid(W, H), dim3(256), 0, s, W, H, pass, rgb, z, alpha, tag, cls, st);
        hipLaunchKernelGGL(k_center_mask, band_grid(W, H), dim3(256), 0, s, W, H, tag, center, st);
    }
    if (roi.center_roi) {
        const int64_t nb = (n + 255) / 256;
        dim3 g((W + 15) / 16, (H + 15) / 16);
        hipLaunchKernelGGL(k_ccl_local, g, dim3(256), 0, s, W, H, 8, center, labels, b.pflag, b.pbox);
        hipLaunchKernelGGL(k_ccl_border, g, dim3(256), 0, s, W, H, 8, center, labels);
        hipLaunchKernelGGL(k_ccl_flatten_roots, dim3((unsigned)nb), dim3(256), 0, s, n, labels, b.bcount, b.rmask);
        hipLaunchKernelGGL(k_root_scan, dim3(1), dim3(1024), 0, s, nb, b.bcount, b.bbox, box_cap, n_boxes, b.gpart,
                           n_gpart, st);
        hipLaunchKernelGGL(k_bbox_acc, dim3((unsigned)nb), dim3(256), 0, s, n, labels, b.pflag, b.pbox, b.bcount,
                           b.rmask, b.bbox);
        const unsigned gcb = (unsigned)std::min<int64_t>(256, nb);
        hipLaunchKernelGGL(k_center_boxes, dim3(gcb), dim3(256), 0, s, W, H, roi.margin, T, tiles_x, b.bcount + nb,
                           b.bbox, boxes, box_cap, tile_mask, st);
    } else {
        hipLaunchKernelGGL(k_fill_i32, dim3(grid(n)), dim3(256), 0, s, n, labels, -1);
        hipLaunchKernelGGL(k_row_fill, dim3(H), dim3(256), 0, s, W, H, tag, center, bg[0], bg[1], bg[2], rgb, z, alpha,
                           cls, st);
        hipLaunchKernelGGL(k_box_count, dim3(1), dim3(256), 0, s, box_cap, n_boxes, b.gpart, n_gpart, st);
    }
    return hipGetLastError();
}

}  // namespace bgs
