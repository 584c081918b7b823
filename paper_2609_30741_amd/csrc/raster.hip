// 2DGS tile rasteriser for gfx950: per-surfel preprocess, load-balanced
// (surfel, tile) key emission, tile ranges and front-to-back blending with
// the joint depth proxy (Sec. 3.1 Stage 1, Sec. 3.3 Eq. 1-2).
#include <cmath>

#include <algorithm>

#include "bgs_internal.h"

namespace bgs {

namespace {

// ---------------------------------------------------------------------------
// Preprocess: one thread per surfel.
// ---------------------------------------------------------------------------

// Compositing-order key: fp32 centre depth with one fixed operation order,
// ((r20*px + r21*py) + r22*pz) + tz, every operation rounded separately.
__device__ inline float centre_depth_key(const float zc[4], float px, float py, float pz) {
#pragma clang fp contract(off)
    float a = zc[0] * px;
    float b = zc[1] * py;
    float s = a + b;
    float c = zc[2] * pz;
    s = s + c;
    return s + zc[3];
}

// Real spherical harmonics (Condon-Shortley phase) in Cartesian form for a
// unit direction; the constants are sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
// (times sqrt(2) for m != 0) folded with the polynomial normalisation.
__device__ inline void sh_basis(int deg, float x, float y, float z, float* Y) {
    Y[0] = 0.28209479177387814f;
    if (deg < 1) return;
    const float c1 = 0.4886025119029199f;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = -1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (2.f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * x * z;
    Y[8] = 0.5462742152960396f * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.5900435899266435f * y * (3.f * xx - yy);
    Y[10] = 2.890611442640554f * x * y * z;
    Y[11] = -0.4570457994644658f * y * (4.f * zz - xx - yy);
    Y[12] = 0.3731763325901154f * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -0.4570457994644658f * x * (4.f * zz - xx - yy);
    Y[14] = 1.445305721320277f * z * (xx - yy);
    Y[15] = -0.5900435899266435f * x * (xx - 3.f * yy);
}

// Masked tiles of the rect's rows ty0..ty of columns tx0..tx1, from the
// column sums of the mask prefix: colcum[ty][x] = sum over rows <= ty of
// prefix[row * tiles_x + x].
__device__ inline uint32_t masked_rows(const MaskArgs& m, int tx0, int ty0, int tx1, int ty) {
    const int w = m.tiles_x + 1;
    const uint32_t* c = m.colcum;
    uint32_t s = c[(int64_t)ty * w + tx1 + 1] - c[(int64_t)ty * w + tx0];
    if (ty0 > 0) s -= c[(int64_t)(ty0 - 1) * w + tx1 + 1] - c[(int64_t)(ty0 - 1) * w + tx0];
    return s;
}

__device__ inline uint32_t masked_count(const MaskArgs& m, int tx0, int ty0, int tx1, int ty1) {
    return masked_rows(m, tx0, ty0, tx1, ty1);
}

// ---------------------------------------------------------------------------
// Strip band of a surfel: a direction n (snorm16 pair) and an interval
// [n.mu + c - w, n.mu + c + w] (fp16 c, w) of n.x that holds every pixel x
// the surfel can reach with alpha >= alpha_min.  The blend skips a record
// for a wave's 8x8 pixel region that lies outside the band, which is exact:
// such a record is a no-op on every pixel of the region.  n is the
// footprint's narrowest direction when that confines the regions of a tile
// column better than the y extent, else the y axis.  The band is computed
// for the quantised n the blend decodes, and padded for the fp16 rounding
// and for the blend's fp32 arithmetic.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float snorm16_value(int q) { return (float)q * (1.0f / 32767.0f); }

__device__ __forceinline__ uint32_t half_bits(float x) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
}

__device__ __forceinline__ float half_value(uint32_t bits) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(bits & 0xFFFFu));
}

// Smallest fp16 value >= x (x >= 0), +inf beyond the fp16 range.
__device__ __forceinline__ uint32_t half_bits_up(double x) {
    if (!(x <= 65504.0)) return 0x7C00u;
    uint32_t h = half_bits((float)x);
    while ((double)half_value(h) < x) ++h;
    return h;
}

// Interval of n.x over the conic's outline (dual conic C in normalised
// camera coordinates) for a pixel-space direction n: the tangent lines
// n.x = s solve m^T C2 m - 2 s' m.c3 + s'^2 c22 = 0 with m = (fx nx, fy ny)
// and s = s' + n.(cx, cy).
__device__ __forceinline__ void conic_extent(double nx, double ny, double c00, double c01, double c02, double c11,
                                             double c12, double c22, const PreCam& cam, double& lo, double& hi) {
    const double mx = cam.fx * nx, my = cam.fy * ny;
    const double mc = mx * c02 + my * c12;
    const double mm = mx * mx * c00 + 2.0 * mx * my * c01 + my * my * c11;
    const double d = sqrt(fmax(mc * mc - c22 * mm, 0.0));
    const double s0 = (mc - d) / c22, s1 = (mc + d) / c22;
    const double off = nx * cam.cx + ny * cam.cy;
    lo = fmin(s0, s1) + off;
    hi = fmax(s0, s1) + off;
}

__device__ uint2 strip_band(bool bounded, double c00, double c01, double c02, double c11, double c12, double c22,
                            const PreCam& cam, double mux, double muy, double r_lowpass, double xmin, double xmax,
                            double ymin, double ymax) {
    int qx = 0, qy = 32767;
    if (bounded) {
        // Narrowest direction: smallest eigenvector of F (c3 c3^T - c22 C2) F.
        const double s00 = cam.fx * cam.fx * (c02 * c02 - c22 * c00);
        const double s11 = cam.fy * cam.fy * (c12 * c12 - c22 * c11);
        const double s01 = cam.fx * cam.fy * (c02 * c12 - c22 * c01);
        const double h = 0.5 * (s00 - s11);
        const double lmin = 0.5 * (s00 + s11) - sqrt(h * h + s01 * s01);
        double ex = s01, ey = lmin - s00;
        const double fx2 = lmin - s11, fy2 = s01;
        if (fx2 * fx2 + fy2 * fy2 > ex * ex + ey * ey) {
            ex = fx2;
            ey = fy2;
        }
        const double en = sqrt(ex * ex + ey * ey);
        if (en > 0.0 && isfinite(en)) {
            ex /= en;
            ey /= en;
            if (ey < 0.0) {
                ex = -ex;
                ey = -ey;
            }
            const int cx = (int)rint(ex * 32767.0), cy = (int)rint(ey * 32767.0);
            const double nx = snorm16_value(cx), ny = snorm16_value(cy);
            double lo, hi;
            conic_extent(nx, ny, c00, c01, c02, c11, c12, c22, cam, lo, hi);
            const double nmu = nx * mux + ny * muy, rn = r_lowpass * sqrt(nx * nx + ny * ny);
            lo = fmin(lo, nmu - rn);
            hi = fmax(hi, nmu + rn);
            // Half-length of the rows of one tile column whose 8x8 regions
            // pass, along n and along y.
            const double pass_n = ny > 1e-6 ? (0.5 * (hi - lo) + 3.5 * fabs(nx) + 3.5 * ny) / ny : INFINITY;
            const double pass_y = 0.5 * (ymax - ymin) + 3.5;
            if (pass_n < pass_y) {
                qx = cx;
                qy = cy;
            }
        }
    }
    const double nx = snorm16_value(qx), ny = snorm16_value(qy);
    double lo, hi;
    if (!bounded) {
        lo = -INFINITY;
        hi = INFINITY;
    } else if (qx == 0 && qy == 32767) {
        lo = ny * ymin;  // ymin/ymax already hold the low-pass disc
        hi = ny * ymax;
    } else {
        conic_extent(nx, ny, c00, c01, c02, c11, c12, c22, cam, lo, hi);
        const double nmu = nx * mux + ny * muy, rn = r_lowpass * sqrt(nx * nx + ny * ny);
        lo = fmin(lo, nmu - rn);
        hi = fmax(hi, nmu + rn);
    }
    const uint32_t nbits = ((uint32_t)qx & 0xFFFFu) | ((uint32_t)qy << 16);
    if (!(isfinite(lo) && isfinite(hi))) return make_uint2(nbits, 0u | (0x7C00u << 16));
    const double nmu = nx * (double)(float)mux + ny * (double)(float)muy;
    const double c = 0.5 * (lo + hi) - nmu;
    const uint32_t cb = half_bits((float)c);
    const double rx = fmax(fabs(xmin - mux), fabs(xmax - mux)), ry = fmax(fabs(ymin - muy), fabs(ymax - muy));
    const double pad = 0.05 + 1e-6 * (fabs(mux) + fabs(muy) + sqrt(rx * rx + ry * ry) + cam.W + cam.H) +
                       fabs(nmu - (nx * mux + ny * muy));
    const double w = 0.5 * (hi - lo) + fabs(c - (double)half_value(cb)) + pad;
    return make_uint2(nbits, cb | (half_bits_up(w) << 16));
}


// ---------------------------------------------------------------------------
// Tile binning by band: of row ty of a surfel's tile rect, the columns
// [*a, *b] (empty when *b < *a) whose 16x16 tile meets the record's strip
// band.  A tile that misses the band is missed by every pixel region in it,
// so the record is a no-op there and needs no key.  fp64, from the record's
// own (fp32 centre, snorm16 direction, fp16 interval) values, with half a
// pixel of margin: the preprocess, the masked counts and the emission call
// this one function on the same values, so counts and keys agree exactly.
// ---------------------------------------------------------------------------
struct BandRows {
    double k0, k16, r, inv;  // k(ty) = k0 + k16 ty; columns where |16 nx tx + k| <= r
    bool vertical;           // nx = 0 (or no direction): whole rows in or out
    __device__ BandRows() : k0(0.0), k16(0.0), r(-1.0), inv(0.0), vertical(true) {}  // no tile
    __device__ explicit BandRows(const SurfelRec& rec) {
#pragma clang fp contract(off)
        const uint32_t nq = __float_as_uint(rec.c.w), bq = __float_as_uint(rec.d.w);
        const double nx = (double)snorm16_value((int)(int16_t)(nq & 0xFFFFu));
        const double ny = (double)snorm16_value((int)(int16_t)(nq >> 16));
        const double c = (double)half_value(bq);
        r = (double)half_value(bq >> 16) + 7.5 * (fabs(nx) + fabs(ny)) + 0.5;
        k0 = nx * (7.5 - (double)rec.a.x) + ny * (7.5 - (double)rec.a.y) - c;
        k16 = 16.0 * ny;
        vertical = !(fabs(nx) > 1e-9);
        inv = vertical ? 0.0 : 1.0 / (16.0 * nx);
    }
    __device__ void row(int ty, int tx0, int tx1, int* a, int* b) const {
#pragma clang fp contract(off)
        const double k = fma(k16, (double)ty, k0);
        if (vertical) {  // also an infinite band (r = inf): every column
            const bool in = !(fabs(k) > r);
            *a = in ? tx0 : 1;
            *b = in ? tx1 : 0;
            return;
        }
        double lo = (-r - k) * inv, hi = (r - k) * inv;
        if (lo > hi) {
            const double t = lo;
            lo = hi;
            hi = t;
        }
        lo = ceil(lo);
        hi = floor(hi);
        *a = lo > (double)tx0 ? (lo > (double)tx1 ? tx1 + 1 : (int)lo) : tx0;
        *b = hi < (double)tx1 ? (hi < (double)tx0 ? tx0 - 1 : (int)hi) : tx1;
    }
};

// The rows ty0..ty1 of a surfel's rect, in order: for each row whose band
// interval [a, b] is not empty, f(c, first) gets its key count c (masked
// tiles of [a, b] with the mask enabled, else b - a + 1) and the key of its
// first tile (the compact id with the mask, else the tile id); f returns
// false to stop.  Rows go four at a time, so their mask-prefix loads are in
// flight together: a surfel across a whole image's rows otherwise waits on
// two dependent loads per row.
template <typename F>
__device__ inline void for_band_rows(const BandRows& br, const MaskArgs& m, const uint32_t* pref, int tx0, int ty0,
                                     int tx1, int ty1, F&& f) {
    for (int y0 = ty0; y0 <= ty1; y0 += 4) {
        int a[4], b[4];
        uint32_t lo[4], hi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = 1;
            b[u] = 0;
            if (y0 + u <= ty1) br.row(y0 + u, tx0, tx1, &a[u], &b[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t rb = (int64_t)(y0 + u) * m.tiles_x;
            const bool load = m.enabled && b[u] >= a[u];
            lo[u] = load ? pref[rb + a[u]] : 0u;
            hi[u] = load ? pref[rb + b[u] + 1] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (b[u] < a[u]) continue;
            const int64_t rb = (int64_t)(y0 + u) * m.tiles_x;
            const uint32_t c = m.enabled ? hi[u] - lo[u] : (uint32_t)(b[u] - a[u] + 1);
            const uint32_t first = m.enabled ? lo[u] : (uint32_t)(rb + a[u]);
            if (!f(c, first)) return;
        }
    }
}

// Keys of a surfel: the band's tiles of its rect, only masked ones when the
// mask is enabled.
// segs (optional) receives the number of rows with keys: the segments the
// emission lists for this surfel.
__device__ inline uint32_t band_count(const BandRows& br, const MaskArgs& m, int tx0, int ty0, int tx1, int ty1,
                                      uint32_t* segs = nullptr) {
    uint32_t cnt = 0, ns = 0;
    for_band_rows(br, m, m.prefix, tx0, ty0, tx1, ty1, [&](uint32_t c, uint32_t) {
        cnt += c;
        ns += c ? 1u : 0u;
        return true;
    });
    if (segs) *segs = ns;
    return cnt;
}

// A surfel seen from one camera: its tile rect and every record word but
// the colour (geometry in fp64, Sec. 3.3).  drawn = false: no pixel of this
// camera can get alpha >= alpha_min from it.
struct SurfelView {
    bool drawn;
    int tx0, ty0, tx1, ty1;
    SurfelRec rec;  // rec.d.xyz (colour) left for the caller
};

__device__ __forceinline__ void surfel_view(const PreCam& cam, float px, float py, float pz, float op,
                                            const double tu[3], const double tv[3], double su, double sv,
                                            float alpha_min, int lowpass, SurfelView& v) {
    v.drawn = false;
    // ---- geometry in fp64 ----
    const double d0 = (double)px - cam.t[0], d1 = (double)py - cam.t[1], d2 = (double)pz - cam.t[2];
    double pc[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) pc[r] = cam.Rt[r * 3 + 0] * d0 + cam.Rt[r * 3 + 1] * d1 + cam.Rt[r * 3 + 2] * d2;
    double a[3], b[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        a[r] = cam.Rt[r * 3 + 0] * tu[0] + cam.Rt[r * 3 + 1] * tu[1] + cam.Rt[r * 3 + 2] * tu[2];
        b[r] = cam.Rt[r * 3 + 0] * tv[0] + cam.Rt[r * 3 + 1] * tv[1] + cam.Rt[r * 3 + 2] * tv[2];
    }
    const double nv[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double pzc = pc[2];
    const double mux = cam.fx * pc[0] / pzc + cam.cx;
    const double muy = cam.fy * pc[1] / pzc + cam.cy;

    // ---- conservative pixel bounds of {alpha >= alpha_min} ----
    // Surfel term: the disc u^2+v^2 <= 2 ln(o/alpha_min) of the surfel plane;
    // its outline E(t) = p + cos t A + sin t B projects to a conic whose
    // dual is A A^T + B B^T - p p^T, giving the extreme tangent lines
    // directly.  If the disc reaches z <= 0 the bound is the whole screen.
    const double lr = log((double)op / (double)alpha_min);
    const double rho = sqrt(2.0 * lr) * (1.0 + 1e-5);
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    bool bounded = false;
    double c00 = 0, c01 = 0, c02 = 0, c11 = 0, c12 = 0, c22 = -1;
    {
        const double A[3] = {rho * su * a[0], rho * su * a[1], rho * su * a[2]};
        const double B[3] = {rho * sv * b[0], rho * sv * b[1], rho * sv * b[2]};
        const double zr2 = A[2] * A[2] + B[2] * B[2];
        if (pzc > 0.0 && pzc * pzc > zr2 * (1.0 + 1e-6) + 1e-12) {
            bounded = true;
            c22 = zr2 - pzc * pzc;
            c00 = A[0] * A[0] + B[0] * B[0] - pc[0] * pc[0];
            c01 = A[0] * A[1] + B[0] * B[1] - pc[0] * pc[1];
            c02 = A[0] * A[2] + B[0] * B[2] - pc[0] * pzc;
            c11 = A[1] * A[1] + B[1] * B[1] - pc[1] * pc[1];
            c12 = A[1] * A[2] + B[1] * B[2] - pc[1] * pzc;
            const double dx = sqrt(fmax(c02 * c02 - c00 * c22, 0.0));
            const double dy = sqrt(fmax(c12 * c12 - c11 * c22, 0.0));
            const double kx0 = (c02 - dx) / c22, kx1 = (c02 + dx) / c22;
            const double ky0 = (c12 - dy) / c22, ky1 = (c12 + dy) / c22;
            xmin = cam.fx * fmin(kx0, kx1) + cam.cx;
            xmax = cam.fx * fmax(kx0, kx1) + cam.cx;
            ymin = cam.fy * fmin(ky0, ky1) + cam.cy;
            ymax = cam.fy * fmax(ky0, ky1) + cam.cy;
        } else {
            xmin = -INFINITY;
            xmax = INFINITY;
            ymin = -INFINITY;
            ymax = INFINITY;
        }
    }
    // Low-pass term: exp(-|x - mu|^2) >= alpha_min / o on a disc around mu.
    if (lowpass) {
        const double r2 = sqrt(lr) * (1.0 + 1e-5);
        xmin = fmin(xmin, mux - r2);
        xmax = fmax(xmax, mux + r2);
        ymin = fmin(ymin, muy - r2);
        ymax = fmax(ymax, muy + r2);
    }
    const double padx = 0.02 + 1e-7 * (fabs(xmin) + fabs(xmax));
    const double pady = 0.02 + 1e-7 * (fabs(ymin) + fabs(ymax));
    const double fx0 = fmax(ceil(xmin - padx), 0.0), fx1 = fmin(floor(xmax + padx), (double)(cam.W - 1));
    const double fy0 = fmax(ceil(ymin - pady), 0.0), fy1 = fmin(floor(ymax + pady), (double)(cam.H - 1));
    if (!(fx0 <= fx1 && fy0 <= fy1)) return;
    const int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
    const uint2 band = strip_band(bounded, c00, c01, c02, c11, c12, c22, cam, mux, muy,
                                  lowpass ? sqrt(lr) * (1.0 + 1e-5) : 0.0, xmin, xmax, ymin, ymax);
    v.tx0 = x0 / kTile;
    v.tx1 = x1 / kTile;
    v.ty0 = y0 / kTile;
    v.ty1 = y1 / kTile;
    v.drawn = true;

    // ---- plane-to-screen homography centred at the projected centre ----
    // With r_c = p/p_z and delta = ((i-mu_x)/fx, (j-mu_y)/fy, 0) the pixel
    // ray is r = r_c + delta; the plane n.X = n.p meets it at
    // lambda = p_z / (1 + n.delta / n.r_c), and the in-plane coordinates
    // u = (lambda r - p).t_u / s_u, v likewise, reduce to ratios of linear
    // forms in (dx, dy): the form stays well conditioned near the centre.
    float C1 = 0.f, C2 = 0.f, D1 = 0.f, D2 = 0.f, N1 = 0.f, N2 = 0.f, lam_num = -1.f;
    {
        const double np = nv[0] * pc[0] + nv[1] * pc[1] + nv[2] * pc[2];
        const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        const double pn = sqrt(pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2]);
        if (fabs(np) > 1e-12 * nn * pn) {
            const double nrc = np / pzc;
            const double as[3] = {a[0] / su, a[1] / su, a[2] / su};
            const double bs[3] = {b[0] / sv, b[1] / sv, b[2] / sv};
            const double pa = pc[0] * as[0] + pc[1] * as[1] + pc[2] * as[2];
            const double pb = pc[0] * bs[0] + pc[1] * bs[1] + pc[2] * bs[2];
            const double n1 = nv[0] / (cam.fx * nrc), n2 = nv[1] / (cam.fy * nrc);
            // u and v are stored scaled by sqrt(1/2): the blend then takes
            // -(u^2 + v^2) as the exponent of G3 = exp(-(u^2 + v^2) / 2).
            constexpr double kRootHalf = 0.70710678118654752440;
            C1 = (float)(kRootHalf * (pzc * as[0] / cam.fx - n1 * pa));
            C2 = (float)(kRootHalf * (pzc * as[1] / cam.fy - n2 * pa));
            D1 = (float)(kRootHalf * (pzc * bs[0] / cam.fx - n1 * pb));
            D2 = (float)(kRootHalf * (pzc * bs[1] / cam.fy - n2 * pb));
            N1 = (float)n1;
            N2 = (float)n2;
            lam_num = (float)pzc;
        }
    }
    v.rec.a = make_float4((float)mux, (float)muy, C1, C2);
    v.rec.b = make_float4(D1, D2, N1, N2);
    v.rec.c = make_float4(lam_num, (float)pzc, op, __uint_as_float(band.x));
    v.rec.d = make_float4(0.f, 0.f, 0.f, __uint_as_float(band.y));
}

__device__ __forceinline__ void sh_dir(const PreCam& cam, float px, float py, float pz, float* d) {
    float dirx = (float)((double)px - cam.t[0]), diry = (float)((double)py - cam.t[1]),
          dirz = (float)((double)pz - cam.t[2]);
    const float inv = rsqrtf(dirx * dirx + diry * diry + dirz * dirz);
    d[0] = dirx * inv;
    d[1] = diry * inv;
    d[2] = dirz * inv;
}

// Per surfel: the centre-depth key, tile rect, key count and record for
// `cam`; with kTwo also the key, rect and record for cam2 (the other eye of
// a stereo frame, whose key counts depend on a tile mask known only later).
// The scene is read once; the colours of both eyes come from one pass over
// the SH coefficients, each toward its own camera centre.
template <bool kTwo>
__global__ __launch_bounds__(256) void k_preprocess(SceneArgs sc, PreCam cam, PreCam cam2, float alpha_min,
                                                    int lowpass, MaskArgs mask, SurfelRec* __restrict__ recs,
                                                    uint32_t* __restrict__ zkeys, uint2* __restrict__ rects,
                                                    uint32_t* __restrict__ counts, SurfelRec* __restrict__ recs2,
                                                    uint32_t* __restrict__ zkeys2, uint2* __restrict__ rects2,
                                                    uint32_t* __restrict__ nseg) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= sc.n) return;
    const int n = sc.n;
    const float px = sc.pos[k], py = sc.pos[n + k], pz = sc.pos[2 * n + k];
    const float op = sc.opacity[k];
    const uint2 empty = make_uint2(0xFFFFFFFFu, 0u);
    const float zf = centre_depth_key(cam.zc, px, py, pz);
    const bool in1 = (double)zf > cam.z_near;
    float zf2 = 0.f;
    bool in2 = false;
    if (kTwo) {
        zf2 = centre_depth_key(cam2.zc, px, py, pz);
        in2 = (double)zf2 > cam2.z_near;
        zkeys2[k] = in2 ? __float_as_uint(zf2) : 0xFFFFFFFFu;
    }
    zkeys[k] = in1 ? __float_as_uint(zf) : 0xFFFFFFFFu;
    // alpha = min(0.99, o G) <= o can never reach alpha_min below it.
    const bool live = op >= alpha_min;
    SurfelView v1, v2;
    v1.drawn = v2.drawn = false;
    if (live && (in1 || in2)) {
        double qw = sc.quat[k], qx = sc.quat[n + k], qy = sc.quat[2 * n + k], qz = sc.quat[3 * n + k];
        const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= qn; qx *= qn; qy *= qn; qz *= qn;
        // Columns t_u, t_v of the quaternion's rotation matrix (Sec. 3.3).
        const double tu[3] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy + qw * qz), 2.0 * (qx * qz - qw * qy)};
        const double tv[3] = {2.0 * (qx * qy - qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz + qw * qx)};
        const double su = sc.scale[k], sv = sc.scale[n + k];
        if (in1) surfel_view(cam, px, py, pz, op, tu, tv, su, sv, alpha_min, lowpass, v1);
        if (kTwo && in2) surfel_view(cam2, px, py, pz, op, tu, tv, su, sv, alpha_min, lowpass, v2);
    }
    uint32_t cnt = 0, segs = 0;
    if (v1.drawn) {
        cnt = band_count(BandRows(v1.rec), mask, v1.tx0, v1.ty0, v1.tx1, v1.ty1, &segs);
        rects[k] = make_uint2((uint32_t)v1.tx0 | ((uint32_t)v1.ty0 << 16), (uint32_t)v1.tx1 | ((uint32_t)v1.ty1 << 16));
    } else {
        rects[k] = empty;
    }
    counts[k] = cnt;
    if (nseg) nseg[k] = segs;
    if (kTwo)
        rects2[k] = v2.drawn ? make_uint2((uint32_t)v2.tx0 | ((uint32_t)v2.ty0 << 16),
                                          (uint32_t)v2.tx1 | ((uint32_t)v2.ty1 << 16))
                             : empty;
    const bool col1 = cnt > 0, col2 = kTwo && v2.drawn;
    if (!col1 && !col2) return;
    // ---- colour: SH towards the surfel from each camera's centre ----
    // (With two eyes, the second eye's colour is also kept for every surfel
    // the first eye bins, drawn in the second eye or not: the view-colour
    // transfer composites it with the first eye's weights.)
    float d1[3] = {0.f, 0.f, 1.f}, d2[3] = {0.f, 0.f, 1.f};
    if (col1) sh_dir(cam, px, py, pz, d1);
    if (kTwo && (col1 || col2)) sh_dir(cam2, px, py, pz, d2);
    float Y1[16], Y2[16];
    sh_basis(sc.sh_degree, d1[0], d1[1], d1[2], Y1);
    if (kTwo) sh_basis(sc.sh_degree, d2[0], d2[1], d2[2], Y2);
    const int nc = (sc.sh_degree + 1) * (sc.sh_degree + 1);
    float acc1[3] = {0.f, 0.f, 0.f}, acc2[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < nc; ++c) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float q = sc.sh[(int64_t)(c * 3 + ch) * n + k];
            acc1[ch] += Y1[c] * q;
            if (kTwo) acc2[ch] += Y2[c] * q;
        }
    }
    if (col1) {
        v1.rec.d.x = fmaxf(acc1[0] + 0.5f, 0.f);
        v1.rec.d.y = fmaxf(acc1[1] + 0.5f, 0.f);
        v1.rec.d.z = fmaxf(acc1[2] + 0.5f, 0.f);
        recs[k] = v1.rec;
    }
    if (col2) {
        v2.rec.d.x = fmaxf(acc2[0] + 0.5f, 0.f);
        v2.rec.d.y = fmaxf(acc2[1] + 0.5f, 0.f);
        v2.rec.d.z = fmaxf(acc2[2] + 0.5f, 0.f);
        recs2[k] = v2.rec;
    } else if (kTwo && col1) {
        // Not drawn in the second eye: only the colour part, for the transfer.
        recs2[k].d = make_float4(fmaxf(acc2[0] + 0.5f, 0.f), fmaxf(acc2[1] + 0.5f, 0.f), fmaxf(acc2[2] + 0.5f, 0.f),
                                 0.f);
    }
}

// Surfels whose rect spans more than kCoopRows tile rows are counted (ROI
// pass) and have their segments listed (emission, up to kCoopMax per
// workgroup) by a whole wave, a row per lane: the nearest surfels span the
// image's rows, and one thread walking them set these kernels' tails.
constexpr int kCoopRows = 16;
constexpr int kCoopMax = 32;

// Key counts of surfels whose tile rects and records were computed
// earlier, restricted to the tiles of a mask.
// The mask prefix is staged in LDS (dynamic shared memory, mask_lds words)
// when it fits: the band rows read it twice a row.
__global__ __launch_bounds__(256) void k_masked_counts(const uint2* __restrict__ rects,
                                                       const SurfelRec* __restrict__ recs, int n, MaskArgs mask,
                                                       int mask_lds, uint32_t* __restrict__ counts,
                                                       uint32_t* __restrict__ nseg) {
    extern __shared__ uint32_t s_mpre[];
    if (mask_lds > 0) {  // uniform over the grid
        for (int i = threadIdx.x; i < mask_lds; i += 256) s_mpre[i] = mask.prefix[i];
        __syncthreads();
        mask.prefix = s_mpre;
    }
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const uint2 r = rects[k];
    if (r.x > r.y || masked_count(mask, (int)(r.x & 0xFFFFu), (int)(r.x >> 16), (int)(r.y & 0xFFFFu),
                                  (int)(r.y >> 16)) == 0) {
        counts[k] = 0;
        nseg[k] = 0;
        return;
    }
    uint32_t segs = 0;
    counts[k] = band_count(BandRows(recs[k]), mask, (int)(r.x & 0xFFFFu), (int)(r.x >> 16), (int)(r.y & 0xFFFFu),
                           (int)(r.y >> 16), &segs);
    nseg[k] = segs;
}

// The ROI pass's key counts in compositing order, fused with the first step
// of their scan: one thread per position i of the order writes the masked
// key count of surfel order[i] at i, and each block of 256 positions writes
// its total to partials[block], so only the scan's down-sweep remains (it
// adds kScanItems of these partials per block of its own).
__global__ __launch_bounds__(256) void k_masked_counts_ordered(const uint2* __restrict__ rects,
                                                               const SurfelRec* __restrict__ recs,
                                                               const uint32_t* __restrict__ order, int n,
                                                               MaskArgs mask, int mask_lds,
                                                               uint32_t* __restrict__ counts,
                                                               uint32_t* __restrict__ partials,
                                                               uint32_t* __restrict__ nseg) {
    extern __shared__ uint32_t s_mpre[];
    __shared__ uint32_t s4[4];
    if (mask_lds > 0) {  // uniform over the grid
        for (int i = threadIdx.x; i < mask_lds; i += 256) s_mpre[i] = mask.prefix[i];
        __syncthreads();
        mask.prefix = s_mpre;
    }
    const int i = blockIdx.x * 256 + threadIdx.x;
    uint32_t c = 0, segs = 0, k = 0;
    uint2 r = make_uint2(1u, 0u);
    bool tall = false;
    if (i < n) {
        k = order[i];
        r = rects[k];
        if (!(r.x > r.y)) {
            const int tx0 = (int)(r.x & 0xFFFFu), ty0 = (int)(r.x >> 16), tx1 = (int)(r.y & 0xFFFFu),
                      ty1 = (int)(r.y >> 16);
            if (masked_count(mask, tx0, ty0, tx1, ty1) != 0) {
                if (ty1 - ty0 + 1 > kCoopRows)
                    tall = true;  // counted by the whole wave below
                else
                    c = band_count(BandRows(recs[k]), mask, tx0, ty0, tx1, ty1, &segs);
            }
        }
    }
    // Surfels across many tile rows (the nearest ones span the image): the
    // wave counts each one's rows together, a row per lane.
    const int lane = (int)(threadIdx.x & 63);
    for (uint64_t tb = __ballot(tall); tb; tb &= tb - 1) {
        const int src = __ffsll((unsigned long long)tb) - 1;
        const uint32_t kk = (uint32_t)__shfl((int)k, src, 64);
        const uint32_t rx = (uint32_t)__shfl((int)r.x, src, 64), ry = (uint32_t)__shfl((int)r.y, src, 64);
        const int hx0 = (int)(rx & 0xFFFFu), hy0 = (int)(rx >> 16), hx1 = (int)(ry & 0xFFFFu), hy1 = (int)(ry >> 16);
        const BandRows hb(recs[kk]);
        uint32_t cc = 0, ss = 0;
        for (int y = hy0 + lane; y <= hy1; y += 64) {
            int a, b;
            hb.row(y, hx0, hx1, &a, &b);
            if (b < a) continue;
            const int64_t rb = (int64_t)y * mask.tiles_x;
            const uint32_t cy = mask.prefix[rb + b + 1] - mask.prefix[rb + a];
            cc += cy;
            ss += cy ? 1u : 0u;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            cc += (uint32_t)__shfl_xor((int)cc, off, 64);
            ss += (uint32_t)__shfl_xor((int)ss, off, 64);
        }
        if (lane == src) {
            c = cc;
            segs = ss;
        }
    }
    if (i < n) {
        counts[i] = c;
        nseg[i] = segs;  // by position in the order, as the counts
    }
    uint32_t sum = c;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += (uint32_t)__shfl_xor((int)sum, off, 64);
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = s4[0] + s4[1] + s4[2] + s4[3];
}

// ---------------------------------------------------------------------------
// Key emission, per block of up to 256 surfels in compositing order: one thread
// per surfel lists the non-empty rows of its band within its rect as
// segments (start of the segment's keys in the block, the first tile's key
// and the surfel), in LDS.  The block's keys are then taken in windows: each
// segment marks its keys of the window with its index in an owner table,
// and each key is written from its owner's segment, with consecutive
// threads on consecutive keys, so a surfel that covers many tiles does not
// serialise one thread.  A block with more segments than the table holds
// takes them in turns of the table's size.  With a tile mask, its prefix
// table is staged in LDS (dynamic shared memory) when it fits.
// ---------------------------------------------------------------------------
constexpr int kEmitSegs = 2048;
constexpr int kEmitWin = 2048;
constexpr int kEmitMaskLds = 8192;  // mask prefix words staged in LDS at most (32 KiB)

__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ order, const uint32_t* __restrict__ offs,
                                              const uint2* __restrict__ rects, const SurfelRec* __restrict__ recs,
                                              int n, int spb, int tiles_x, MaskArgs mask, int mask_lds,
                                              uint32_t cap, int vbits, uint32_t* __restrict__ tkeys,
                                              uint32_t* __restrict__ tvals, const uint32_t* __restrict__ nseg,
                                              int nseg_by_pos) {
    extern __shared__ uint32_t s_mpre[];  // mask_lds words: the mask prefix, when staged
    __shared__ uint32_t sk[256];
    __shared__ uint32_t seg_start[kEmitSegs + 1];
    __shared__ uint32_t seg_tile[kEmitSegs];  // first tile's key | surfel << 24 (keys < 2^20: sides <= 16384 px)
    __shared__ uint16_t owner[kEmitWin];
    __shared__ uint32_t lds[4];
    __shared__ uint32_t s_nh;                // surfels listed by a wave
    __shared__ float4 s_hrec[kCoopMax];      // their band words: centre x, y and the two packed band words
    __shared__ uint4 s_hinfo[kCoopMax];      // rect (two packed words), first key in the block, first segment
    __shared__ uint2 s_howner[kCoopMax];     // owning thread, segment count
    const int r0 = blockIdx.x * spb;  // spb <= 256 surfels, one thread each; all 256 threads write keys
    const int m = min(spb, n - r0);
    const uint32_t base = offs[r0];
    // A block whose surfels have no key (culled ones sort last; most of a
    // masked pass's surfels miss its tiles) leaves before staging anything.
    if (offs[r0 + m] == base) return;
    const int t = threadIdx.x;
    const uint32_t* pref = mask.prefix;
    if (mask_lds > 0) {  // uniform over the block
        for (int i = t; i < mask_lds; i += 256) s_mpre[i] = mask.prefix[i];
        __syncthreads();
        pref = s_mpre;
    }
    uint2 rc = make_uint2(0xFFFFFFFFu, 0u);
    uint32_t cnt = 0, loc = 0, ns_given = 0;
    SurfelRec rec;
    if (t < m) {
        const uint32_t k = order[r0 + t];
        loc = offs[r0 + t] - base;
        cnt = offs[r0 + t + 1] - offs[r0 + t];
        sk[t] = k;
        if (cnt) {
            rc = rects[k];
            rec = recs[k];
            if (nseg) ns_given = nseg[nseg_by_pos ? (uint32_t)(r0 + t) : k];
        }
    }
    const int tx0 = rc.x & 0xFFFF, ty0 = rc.x >> 16, tx1 = rc.y & 0xFFFF, ty1 = rc.y >> 16;
    const BandRows br = cnt ? BandRows(rec) : BandRows();
    // Segments of this thread's surfel: counted by the pass that counted
    // its keys, or here.
    uint32_t ns = ns_given;
    MaskArgs mk = mask;
    mk.tiles_x = tiles_x;
    if (cnt && !nseg) {
        for_band_rows(br, mk, pref, tx0, ty0, tx1, ty1, [&](uint32_t c, uint32_t) {
            ns += c ? 1u : 0u;
            return true;
        });
    }
    // Exclusive scan of the segment counts over the block.
    uint32_t v = ns;
    const int lane = t & 63, w = t >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    if (t == 0) s_nh = 0;
    if (lane == 63) lds[w] = v;
    __syncthreads();
    uint32_t sbase = v - ns;
    for (int q = 0; q < w; ++q) sbase += lds[q];
    const uint32_t tot_seg = lds[0] + lds[1] + lds[2] + lds[3];
    bool coop = false;
    if (ns && ty1 - ty0 + 1 > kCoopRows) {
        const uint32_t h = atomicAdd(&s_nh, 1u);
        if (h < (uint32_t)kCoopMax) {
            coop = true;
            s_hrec[h] = make_float4(rec.a.x, rec.a.y, rec.c.w, rec.d.w);
            s_hinfo[h] = make_uint4(rc.x, rc.y, loc, sbase);
            s_howner[h] = make_uint2((uint32_t)t, ns);
        }
    }
    __syncthreads();
    const uint32_t n_coop = min(s_nh, (uint32_t)kCoopMax);
    for (uint32_t w0 = 0; w0 < tot_seg; w0 += kEmitSegs) {
        const uint32_t w1 = min(tot_seg, w0 + (uint32_t)kEmitSegs);
        if (ns && !coop && sbase < w1 && sbase + ns > w0) {
            uint32_t si = sbase, kpos = loc;
            for_band_rows(br, mk, pref, tx0, ty0, tx1, ty1, [&](uint32_t c, uint32_t first) {
                if (si >= w1) return false;
                if (!c) return true;
                if (si >= w0) {
                    seg_start[si - w0] = kpos;
                    seg_tile[si - w0] = first | ((uint32_t)t << 24);
                    if (si + 1 == w1) seg_start[w1 - w0] = kpos + c;  // end of the turn's keys
                }
                kpos += c;
                ++si;
                return true;
            });
        }
        // The wave-listed surfels: 64 rows at a time, the row's segment slot
        // from a ballot of the rows with keys and its first key from a
        // prefix sum of the row counts.
        for (uint32_t h = (uint32_t)w; h < n_coop; h += 4) {
            const uint4 hi = s_hinfo[h];
            const uint2 ho = s_howner[h];
            if (!(hi.w < w1 && hi.w + ho.y > w0)) continue;  // uniform over the wave
            const float4 hr = s_hrec[h];
            SurfelRec q{};
            q.a.x = hr.x;
            q.a.y = hr.y;
            q.c.w = hr.z;
            q.d.w = hr.w;
            const BandRows hb(q);
            const int hx0 = (int)(hi.x & 0xFFFFu), hy0 = (int)(hi.x >> 16), hx1 = (int)(hi.y & 0xFFFFu),
                      hy1 = (int)(hi.y >> 16);
            uint32_t seg_carry = 0, key_carry = 0;
            for (int y0 = hy0; y0 <= hy1 && hi.w + seg_carry < w1; y0 += 64) {
                const int y = y0 + lane;
                int a = 1, b = 0;
                if (y <= hy1) hb.row(y, hx0, hx1, &a, &b);
                uint32_t c = 0, first = 0;
                if (b >= a) {
                    const int64_t rb = (int64_t)y * tiles_x;
                    if (mask.enabled) {
                        first = pref[rb + a];
                        c = pref[rb + b + 1] - first;
                    } else {
                        first = (uint32_t)(rb + a);
                        c = (uint32_t)(b - a + 1);
                    }
                }
                const uint64_t bal = __ballot(c != 0);
                const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                uint32_t kin = c;  // inclusive prefix of the row counts over the wave
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint32_t yv = __shfl_up(kin, off, 64);
                    if (lane >= off) kin += yv;
                }
                const uint32_t si = hi.w + seg_carry + before;
                const uint32_t kpos = hi.z + key_carry + kin - c;
                if (c != 0 && si >= w0 && si < w1) {
                    seg_start[si - w0] = kpos;
                    seg_tile[si - w0] = first | (ho.x << 24);
                    if (si + 1 == w1) seg_start[w1 - w0] = kpos + c;  // end of the turn's keys
                }
                seg_carry += (uint32_t)__popcll(bal);
                key_carry += __shfl(kin, 63, 64);
            }
        }
        __syncthreads();
        const int nw = (int)(w1 - w0);
        const uint32_t p0 = seg_start[0], p1 = seg_start[nw];
        for (uint32_t kw = p0; kw < p1; kw += kEmitWin) {
            const uint32_t ke = min(p1, kw + (uint32_t)kEmitWin);
            // Owner of every key of the window: each segment marks where its
            // keys start in the window (segment index + 1; the segment that
            // covers the window's first key marks position 0), and an
            // inclusive max-scan carries each mark over its segment's keys.
            // A segment's keys are not filled by one thread in turn: a
            // surfel across a whole row of tiles would serialise it.
            static_assert(kEmitWin == 8 * 256, "eight window positions per thread");
            const uint32_t len = ke - kw;
            for (uint32_t i = t; i < len; i += 256) owner[i] = 0;
            __syncthreads();
            for (int j = t; j < nw; j += 256) {
                const uint32_t s0 = seg_start[j], s1 = seg_start[j + 1];
                if (s0 < ke && s1 > kw) owner[(s0 > kw ? s0 : kw) - kw] = (uint16_t)(j + 1);
            }
            __syncthreads();
            uint32_t run[8], mx = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t i = 8u * (uint32_t)t + (uint32_t)e;
                mx = max(mx, i < len ? (uint32_t)owner[i] : 0u);
                run[e] = mx;
            }
            uint32_t xm = mx;  // inclusive max over the wave's threads, then over the waves before
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(xm, off, 64);
                if (lane >= off) xm = max(xm, y);
            }
            __syncthreads();  // every mark is read before the LDS word below is reused
            if (lane == 63) lds[w] = xm;
            __syncthreads();
            uint32_t before = __shfl_up(xm, 1, 64);
            if (lane == 0) before = 0;
            for (int q = 0; q < w; ++q) before = max(before, lds[q]);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t i = 8u * (uint32_t)t + (uint32_t)e;
                if (i < len) owner[i] = (uint16_t)(max(run[e], before) - 1u);
            }
            __syncthreads();
            for (uint32_t p = kw + t; p < ke; p += 256) {
                const int j = owner[p - kw];
                const uint32_t st = seg_tile[j];
                const uint32_t g = base + p;
                if (g < cap) {
                    const uint32_t tile = (st & 0xFFFFFFu) + (p - seg_start[j]);
                    if (vbits) {
                        tkeys[g] = tile << vbits | sk[st >> 24];
                    } else {
                        tkeys[g] = tile;
                        tvals[g] = sk[st >> 24];
                    }
                }
            }
            __syncthreads();
        }
    }
}

// [start, end) of every tile in the sorted keys: a key that differs from
// its predecessor starts its tile's range and ends the predecessor's.  The
// ranges were cleared to empty beforehand (by the count scan), so a tile
// with no key keeps an empty range.  Grid-stride over the *n_dev keys.
// Each thread takes four consecutive keys (one 16-byte load; the keys
// buffer is 16-byte aligned) and the key before them.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
                                                uint2* __restrict__ ranges, uint32_t n_tiles, int shift) {
    const uint32_t n = *n_dev;
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; 4 * q < n; q += (uint64_t)gridDim.x * 256) {
        const uint32_t i0 = (uint32_t)(4 * q);
        uint32_t k[4];
        if (i0 + 3 < n) {
            const uint4 v = *reinterpret_cast<const uint4*>(keys + i0);
            k[0] = v.x >> shift; k[1] = v.y >> shift; k[2] = v.z >> shift; k[3] = v.w >> shift;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) k[u] = i0 + u < n ? keys[i0 + u] >> shift : 0xFFFFFFFFu;
        }
        uint32_t prev = i0 > 0 ? keys[i0 - 1] >> shift : 0xFFFFFFFFu;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + u;
            if (i >= n) break;
            if (k[u] != prev) {
                if (k[u] < n_tiles) ranges[k[u]].x = i;
                if (i > 0 && prev < n_tiles) ranges[prev].y = i;
            }
            if (i + 1 == n && k[u] < n_tiles) ranges[k[u]].y = n;
            prev = k[u];
        }
    }
}

__global__ void k_status_keys(const uint32_t* __restrict__ offs, int n, DevStatus* st, uint32_t cap, int which) {
    st->n_slots = 0;
    st->n_items = 0;
    const uint32_t K = offs[n];
    st->n_keys = K;
    st->n_sort = K < cap ? K : cap;
    if (K > cap) st->overflow |= 1u;
    if (which == 0) st->n_keys_dom = K;
    else st->n_keys_roi = K;
}

constexpr int kMaskLds = 15360;  // tile-mask prefix words staged in LDS (60 KiB)

// Bit j set iff byte j of w is nonzero (j = 0..3).
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) {
    const uint32_t h = (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
    return ((h >> 7) & 1u) | ((h >> 14) & 2u) | ((h >> 21) & 4u) | ((h >> 28) & 8u);
}

// Tables of an ROI tile mask, one workgroup: prefix[t] = masked tiles before
// tile t (t = 0..n_tiles), the compact list of masked tile ids, their count,
// and colcum[ty][x] = sum over rows <= ty of prefix[row * tiles_x + x] for
// x = 0..tiles_x, from which any rect's masked count takes four loads.
// A mask of fewer than kMaskLds tiles is read in one step (16 tiles a
// thread, loads issued together), its prefix built in LDS, and the column
// sums taken by (column, band of rows) pairs: each pair sums its band, the
// bands before it give its start, and it writes its rows.  Larger masks
// take 4096 tiles per step and one wave per column.
__global__ __launch_bounds__(1024) void k_mask_tables(const uint8_t* __restrict__ m, int n_tiles, int tiles_x,
                                                      uint32_t* __restrict__ prefix, uint32_t* __restrict__ list,
                                                      uint32_t* __restrict__ colcum, DevStatus* st) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t s_run;
    __shared__ uint32_t s_pre[kMaskLds];
    __shared__ uint32_t s_band[1024];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_y = n_tiles / tiles_x;
    const bool staged = n_tiles + 1 <= kMaskLds;
    static_assert(kMaskLds <= 16 * 1024, "one step of 16 tiles a thread covers a staged mask");
    if (staged) {
        const int t0 = 16 * tid;
        uint32_t bits = 0;  // bit j: tile t0 + j is masked
        if (t0 + 16 <= n_tiles && ((reinterpret_cast<uintptr_t>(m) & 15u) == 0)) {
            const uint4 w = *reinterpret_cast<const uint4*>(m + t0);
            bits = nonzero_bytes(w.x) | (nonzero_bytes(w.y) << 4) | (nonzero_bytes(w.z) << 8) |
                   (nonzero_bytes(w.w) << 12);
        } else {
            uint8_t b[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) b[j] = t0 + j < n_tiles ? m[t0 + j] : 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) bits |= (b[j] != 0 ? 1u : 0u) << j;
        }
        const uint32_t sum = __popc(bits);
        uint32_t x = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t acc = x - sum, total = 0;
        for (int w = 0; w < 16; ++w) {
            const uint32_t ws = wsum[w];
            if (w < wave) acc += ws;
            total += ws;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int t = t0 + j;
            if (t < n_tiles) {
                s_pre[t] = acc;
                if ((bits >> j) & 1u) list[acc] = (uint32_t)t;
            }
            acc += (bits >> j) & 1u;
        }
        if (tid == 0) {
            s_pre[n_tiles] = total;
            st->n_masked = total;
            st->n_roi_tiles = total;
        }
        __syncthreads();
        for (int t = tid; t <= n_tiles; t += 1024) prefix[t] = s_pre[t];  // coalesced
        // Column x = tiles_x reads the next row's first entry (the last
        // row's is the total).
        const int C = tiles_x + 1;
        if (C <= 1024) {
            const int K = max(1, min(tiles_y, 1024 / C)), R = (tiles_y + K - 1) / K;
            const int k = tid / C, xc = tid - k * C;
            const bool on = k < K;
            const int r0 = on ? min(tiles_y, k * R) : 0, r1 = on ? min(tiles_y, r0 + R) : 0;
            uint32_t bs = 0;
            for (int r = r0; r < r1; ++r) bs += s_pre[r * tiles_x + xc];
            s_band[tid] = bs;
            __syncthreads();
            uint32_t run = 0;
            for (int q = 0; q < k && on; ++q) run += s_band[q * C + xc];
            for (int r = r0; r < r1; ++r) {
                run += s_pre[r * tiles_x + xc];
                colcum[(int64_t)r * C + xc] = run;
            }
        } else {
            for (int xc = tid; xc < C; xc += 1024) {
                uint32_t run = 0;
                for (int r = 0; r < tiles_y; ++r) {
                    run += s_pre[r * tiles_x + xc];
                    colcum[(int64_t)r * C + xc] = run;
                }
            }
        }
        return;
    }
    if (tid == 0) s_run = 0;
    __syncthreads();
    for (int base = 0; base < n_tiles; base += 1024 * 4) {
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = base + tid * 4 + j;
            v[j] = (t < n_tiles && m[t]) ? 1u : 0u;
            sum += v[j];
        }
        uint32_t x = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t acc = s_run;
        for (int w = 0; w < wave; ++w) acc += wsum[w];
        acc += x - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = base + tid * 4 + j;
            if (t < n_tiles) {
                prefix[t] = acc;
                if (v[j]) list[acc] = (uint32_t)t;
            }
            acc += v[j];
        }
        __syncthreads();
        if (tid == 1023) s_run = acc;
        __syncthreads();
    }
    if (tid == 0) {
        prefix[n_tiles] = s_run;
        st->n_masked = s_run;
        st->n_roi_tiles = s_run;
    }
    __syncthreads();  // prefix is read back below by other threads of this block
    // Column sums: a wave takes a column and scans it down the rows 64 at a
    // time with shuffles.
    for (int xc = wave; xc <= tiles_x; xc += 16) {
        uint32_t carry = 0;
        for (int y0 = 0; y0 < tiles_y; y0 += 64) {
            const int ty = y0 + lane;
            const int q = ty * tiles_x + xc;  // xc = tiles_x reads the next row's first entry
            uint32_t x = ty < tiles_y ? prefix[q] : 0u;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off, 64);
                if (lane >= off) x += y;
            }
            if (ty < tiles_y) colcum[(int64_t)ty * (tiles_x + 1) + xc] = carry + x;
            carry += __shfl(x, 63, 64);
        }
    }
}

// ---------------------------------------------------------------------------
// Tile order for the blend: tiles by decreasing key count, bucketed by the
// leading bit and the next four bits of the count (about 6% resolution), so
// that the heaviest tiles are dispatched first and spread over all CUs.
// The order only decides which block renders which tile; every tile's
// pixels are computed the same way whatever the order.
// ---------------------------------------------------------------------------
constexpr int kOrderBuckets = 32 * 16 + 1;  // (octave, 4 mantissa bits), then empty tiles

__device__ __forceinline__ uint32_t order_bucket(uint32_t len) {
    if (len == 0) return kOrderBuckets - 1;
    const uint32_t e = 31u - (uint32_t)__clz((int)len);
    const uint32_t m = e >= 4 ? (len >> (e - 4)) & 15u : (len << (4 - e)) & 15u;
    return (31u - e) * 16u + (15u - m);
}

// Up to kOrderHeld tiles: each thread loads its ranges at once (bounded by
// n_tiles, so the loads need not wait for the live count) and keeps their
// buckets in registers for both passes.
constexpr uint32_t kOrderRegs = 8, kOrderHeld = 1024 * kOrderRegs;

__global__ __launch_bounds__(1024) void k_tile_order(const uint2* __restrict__ ranges, const uint32_t* n_live,
                                                     uint32_t n_tiles, uint32_t* __restrict__ order) {
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ uint32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool held = n_tiles <= kOrderHeld;
    uint32_t bk[kOrderRegs];
    if (held) {
        uint2 r[kOrderRegs];
#pragma unroll
        for (uint32_t u = 0; u < kOrderRegs; ++u) {
            const uint32_t t = tid + 1024u * u;
            r[u] = t < n_tiles ? ranges[t] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (uint32_t u = 0; u < kOrderRegs; ++u) bk[u] = order_bucket(r[u].y - r[u].x);
    }
    const uint32_t n = n_live ? min(*n_live, n_tiles) : n_tiles;
    for (int i = tid; i < kOrderBuckets; i += 1024) hist[i] = 0;
    __syncthreads();
    if (held) {
#pragma unroll
        for (uint32_t u = 0; u < kOrderRegs; ++u)
            if (tid + 1024u * u < n) atomicAdd(&hist[bk[u]], 1u);
    } else {
        for (uint32_t t = tid; t < n; t += 1024) {
            const uint2 r = ranges[t];
            atomicAdd(&hist[order_bucket(r.y - r.x)], 1u);
        }
    }
    __syncthreads();
    // Exclusive scan of the buckets (one per thread).
    uint32_t v = tid < kOrderBuckets ? hist[tid] : 0u, x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += wsum[w];
    if (tid < kOrderBuckets) hist[tid] = wbase + x - v;
    __syncthreads();
    if (held) {
#pragma unroll
        for (uint32_t u = 0; u < kOrderRegs; ++u) {
            const uint32_t t = tid + 1024u * u;
            if (t < n) order[atomicAdd(&hist[bk[u]], 1u)] = t;
        }
    } else {
        for (uint32_t t = tid; t < n; t += 1024) {
            const uint2 r = ranges[t];
            order[atomicAdd(&hist[order_bucket(r.y - r.x)], 1u)] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Blend.  One 256-thread block per 16x16 tile; wave w owns the 8x8 quadrant
// (w & 1, w >> 1) of the tile.  walk_range composites the records [b, e)
// of the tile's sorted list into the block's pixels: batches of 256 records
// are fetched by all threads with vector loads (the next batch while the
// current one is composited) and put in LDS; each wave tests the whole
// batch against its region (the record's strip band) in one vector pass and
// writes the byte offsets of the records that can touch it, in list order,
// to its own LDS list, padded with an all-zero
// record that never contributes.  It then takes kTrip records per trip: their
// alphas are independent and computed together, and only the short
// transmittance chain runs in sequence.  The walk ends at the first batch
// boundary where all 256 pixels are done.  Every thread of the block must
// call it (it has block barriers).
// ---------------------------------------------------------------------------
constexpr int kBatch = 256;
constexpr int kTrip = 4;                // records per trip of the walk
constexpr int kDummy = kBatch;          // LDS record index of the zero record
constexpr int kListLen = kBatch + 4;    // per-wave hit list, with padding
// Continuation segments are walked in kRounds rounds: round r takes the
// segments [round_lo(r), round_lo(r + 1)) of every continued tile.  One
// round: a second one (the later segments walked from the exact
// transmittance after the first four) saved speculative work but cost a
// launch of latency (800x600 frames: 1.5% slower, 256x256 2%).
constexpr int kRounds = 1;
__host__ __device__ constexpr uint32_t round_lo(int r) { return r <= 0 ? 0u : kContMaxSeg; }
static_assert(round_lo(kRounds) == kContMaxSeg, "the rounds cover every segment");
constexpr uint32_t kChainBatch = 8;     // earlier segments' parts loaded together when chaining


// A pixel's compositing state.  A pixel that has stopped, or that takes no
// part in a walk, has T = 0: every later pair then adds nothing, so no
// separate flag is needed.  The background weight of a stopped pixel is its
// transmittance at the stop, which equals 1 - A (A is the sum of the
// weights alpha * T, and each step lowers T by exactly its weight).
struct PixelState {
    float T, c0, c1, c2, D, A;
    float x0, x1, x2;  // view-colour transfer only: the affiliated eye's colours, same weights
};

__device__ __forceinline__ bool live(const PixelState& p) { return p.T > 0.f; }

struct WalkCounts {
    uint32_t eval, used, walk, test;
};

struct TileGeom {
    int tid, lane;
    float fpx, fpy;
    float scx, scy;  // centre of the wave's 8x8 region
};

// Alpha of one (pixel, surfel) pair (Eq. 2 with the plane homography of the
// record): alpha = min(alpha_max, o * max(G3, G2)), and the depth the pair
// adds to the proxy (the ray-plane depth where G3 wins, else the centre
// depth).
__device__ __forceinline__ void pair_alpha(const float4& r0, const float4& r1, const float4& r2, float fpx, float fpy,
                                           const BlendArgs& a, float& al, float& dsel) {
    const float dx = fpx - r0.x, dy = fpy - r0.y;
    const float den = fmaf(r1.z, dx, fmaf(r1.w, dy, 1.f));
    const float w = __builtin_amdgcn_rcpf(den);
    const float u = fmaf(r0.z, dx, r0.w * dy) * w;
    const float v = fmaf(r1.x, dx, r1.y * dy) * w;
    const float lam = r2.x * w;
    // lam <= z_near covers hits behind the camera and edge-on records; a
    // non-finite u, v near the plane's horizon gives -inf or NaN, and
    // fmaxf then keeps the low-pass term.
    // The record's u and v coefficients carry a factor sqrt(1/2), so
    // -(u^2 + v^2) here is the G3 exponent -(u^2 + v^2) / 2 of the plane.
    const float e3 = lam > a.z_near ? -fmaf(u, u, v * v) : -INFINITY;
    const float e2 = a.lowpass ? -fmaf(dx, dx, dy * dy) : -INFINITY;
    al = fminf(a.alpha_max, r2.z * __expf(fmaxf(e3, e2)));
    dsel = (e3 >= e2) ? lam : r2.y;
}

// One front-to-back compositing step: a pair below alpha_min is skipped;
// the pixel stops before the surfel that would take T below t_min;
// otherwise RGB, the depth proxy D and A accumulate with the same weight
// w = alpha * T, and T drops by w.
template <bool kXfer>
__device__ __forceinline__ void accumulate(float al, float dsel, const float4& r3, const float4& xc, const BlendArgs& a,
                                           PixelState& p, WalkCounts& wc, bool count, bool valid) {
    float wt = (al >= a.alpha_min ? al : 0.f) * p.T;
    const float Tn = p.T - wt;
    const bool stop = Tn < a.t_min;  // also for a pixel already stopped (T = 0)
    wt = stop ? 0.f : wt;
    if (count && valid) {
        wc.eval += p.T > 0.f ? 1u : 0u;
        wc.used += wt > 0.f ? 1u : 0u;
    }
    p.c0 = fmaf(wt, r3.x, p.c0);
    p.c1 = fmaf(wt, r3.y, p.c1);
    p.c2 = fmaf(wt, r3.z, p.c2);
    p.D = fmaf(wt, dsel, p.D);
    p.A += wt;
    p.T = stop ? 0.f : Tn;
    if (kXfer) {
        p.x0 = fmaf(wt, xc.x, p.x0);
        p.x1 = fmaf(wt, xc.y, p.x1);
        p.x2 = fmaf(wt, xc.z, p.x2);
    }
}

// Region test, compaction and compositing of one staged batch of nb records
// by one wave (no block barriers).
template <bool kCount, bool kXfer = false>
__device__ __forceinline__ void walk_batch(const float4* s_rec, uint32_t nb, uint16_t* s_list, const TileGeom& g,
                                           const BlendArgs& a, PixelState& p, WalkCounts& wc,
                                           const float4* s_xc = nullptr) {
    const char* s_bytes = reinterpret_cast<const char*>(s_rec);
    uint32_t nhit = 0;
#pragma unroll
    for (int q = 0; q < kBatch / 64; ++q) {
        const uint32_t j = (uint32_t)(q * 64 + g.lane);
        bool h = false;
        if (j < nb) {
            const uint32_t nq = __float_as_uint(s_rec[4 * j + 2].w), bq = __float_as_uint(s_rec[4 * j + 3].w);
            const float nx = snorm16_value((int)(int16_t)(nq & 0xFFFFu));
            const float ny = snorm16_value((int)(int16_t)(nq >> 16));
            const float4 r0 = s_rec[4 * j];
            const float pr = fmaf(nx, g.scx - r0.x, ny * (g.scy - r0.y)) - half_value(bq);
            h = fabsf(pr) <= half_value(bq >> 16) + 3.5f * (fabsf(nx) + fabsf(ny));
        }
        const uint64_t m = __ballot(h);
        if (h) {
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            s_list[nhit + below] = (uint16_t)(j * 64u);
        }
        nhit += (uint32_t)__popcll(m);
    }
    if (g.lane < kTrip) s_list[nhit + g.lane] = (uint16_t)(kDummy * 64);
    // The list is written and read by this wave only.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (kCount) {
        wc.walk += nb;
        wc.test += nhit;
    }
    for (uint32_t k = 0; k < nhit; k += kTrip) {
        if (__ballot(live(p)) == 0ull) break;
        uint32_t off[kTrip];
        if (kTrip == 4) {
            const uint2 o = *reinterpret_cast<const uint2*>(s_list + k);
            off[0] = o.x & 0xFFFFu;
            off[1] = o.x >> 16;
            off[2 % kTrip] = o.y & 0xFFFFu;
            off[3 % kTrip] = o.y >> 16;
        } else {
            const uint32_t o = *reinterpret_cast<const uint32_t*>(s_list + k);
            off[0] = o & 0xFFFFu;
            off[1 % kTrip] = o >> 16;
        }
        float al[kTrip], ds[kTrip];
#pragma unroll
        for (int i = 0; i < kTrip; ++i) {
            const float4* r = reinterpret_cast<const float4*>(s_bytes + off[i]);
            pair_alpha(r[0], r[1], r[2], g.fpx, g.fpy, a, al[i], ds[i]);
        }
#pragma unroll
        for (int i = 0; i < kTrip; ++i) {
            const float4* r = reinterpret_cast<const float4*>(s_bytes + off[i]);
            const float4 xc = kXfer ? s_xc[off[i] >> 6] : make_float4(0.f, 0.f, 0.f, 0.f);
            accumulate<kXfer>(al[i], ds[i], r[3], xc, a, p, wc, kCount, k + i < nhit);
        }
    }
}

__device__ __forceinline__ void load_rec(const SurfelRec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                         uint32_t pos, uint32_t vmask, float4& q0, float4& q1, float4& q2,
                                         float4& q3) {
    const SurfelRec* r = recs + (vals[pos] & vmask);
    q0 = r->a;
    q1 = r->b;
    q2 = r->c;
    q3 = r->d;
}

// The same, and with the transfer the surfel's colour seen from the other
// eye (the last float4 of its record there).
template <bool kXfer>
__device__ __forceinline__ void load_rec(const SurfelRec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                         uint32_t pos, const BlendArgs& a, float4& q0, float4& q1, float4& q2,
                                         float4& q3, float4& qx) {
    const uint32_t k = vals[pos] & a.vmask;
    const SurfelRec* r = recs + k;
    q0 = r->a;
    q1 = r->b;
    q2 = r->c;
    q3 = r->d;
    if (kXfer) qx = a.xrecs[k].d;
}

__device__ __forceinline__ void stage_rec(float4* s_rec, int t, const float4& q0, const float4& q1, const float4& q2,
                                          const float4& q3) {
    s_rec[4 * t + 0] = q0;
    s_rec[4 * t + 1] = q1;
    s_rec[4 * t + 2] = q2;
    s_rec[4 * t + 3] = q3;
}

template <bool kCount>
__device__ __forceinline__ void walk_range(const SurfelRec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                           uint32_t b, uint32_t e, float4* s_rec, uint16_t* s_list,
                                           const TileGeom& g, const BlendArgs& a, PixelState& p, WalkCounts& wc) {
    float4 q0, q1, q2, q3;
    if (b + g.tid < e) load_rec(recs, vals, b + g.tid, a.vmask, q0, q1, q2, q3);
    for (uint32_t base = b; base < e; base += kBatch) {
        const uint32_t nb = min((uint32_t)kBatch, e - base);
        __syncthreads();
        if ((uint32_t)g.tid < nb) stage_rec(s_rec, g.tid, q0, q1, q2, q3);
        __syncthreads();
        if (base + kBatch + g.tid < e) load_rec(recs, vals, base + kBatch + g.tid, a.vmask, q0, q1, q2, q3);
        walk_batch<kCount>(s_rec, nb, s_list, g, a, p, wc);
        if (__syncthreads_count(live(p)) == 0) break;
    }
}

__device__ __forceinline__ TileGeom tile_geom(uint32_t tile, int tid, const BlendArgs& a, bool* inside, int* px,
                                              int* py) {
    TileGeom g;
    const int tx = (int)(tile % (uint32_t)a.tiles_x), ty = (int)(tile / (uint32_t)a.tiles_x);
    g.tid = tid;
    g.lane = g.tid & 63;
    const int wave = g.tid >> 6;
    *px = tx * kTile + (wave & 1) * 8 + (g.lane & 7);
    *py = ty * kTile + (wave >> 1) * 8 + (g.lane >> 3);
    *inside = *px < a.W && *py < a.H &&
              (!a.qmask || a.qmask[(int64_t)(2 * ty + (wave >> 1)) * a.qmask_w + 2 * tx + (wave & 1)] != 0);
    g.fpx = (float)*px;
    g.fpy = (float)*py;
    g.scx = (float)(tx * kTile + (wave & 1) * 8) + 3.5f;
    g.scy = (float)(ty * kTile + (wave >> 1) * 8) + 3.5f;
    return g;
}

template <bool kPatch, bool kXfer = false>
__device__ __forceinline__ void write_pixel(const PixelState& p, int px, int py, const BlendArgs& a,
                                            float* __restrict__ rgb, float* __restrict__ dz, float* __restrict__ alpha,
                                            uint8_t* __restrict__ cls) {
    const int64_t hw = (int64_t)a.W * a.H;
    const int64_t q = (int64_t)py * a.W + px;
    const float tb = p.T > 0.f ? p.T : 1.f - p.A;  // background weight
    rgb[q] = fmaf(tb, a.bg0, p.c0);
    rgb[hw + q] = fmaf(tb, a.bg1, p.c1);
    rgb[2 * hw + q] = fmaf(tb, a.bg2, p.c2);
    if (kXfer) {
        a.xrgb[q] = fmaf(tb, a.bg0, p.x0);
        a.xrgb[hw + q] = fmaf(tb, a.bg1, p.x1);
        a.xrgb[2 * hw + q] = fmaf(tb, a.bg2, p.x2);
    }
    alpha[q] = p.A;
    if (!kPatch) {
        dz[q] = p.D;
    } else {
        dz[q] = p.A >= a.a_min ? p.D / p.A : INFINITY;
        cls[q] = (uint8_t)BGS_CLS_ROI;
    }
}

__device__ __forceinline__ void count_flush(const WalkCounts& wc, int lane, int wave, uint32_t len,
                                            unsigned long long* pair_counts, uint32_t* s_walk) {
    unsigned long long e = wc.eval, u = wc.used;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        e += __shfl_xor(e, off, 64);
        u += __shfl_xor(u, off, 64);
    }
    if (lane == 0) {
        // walk / test are wave-uniform: records walked by this wave and
        // records that passed its strip test.
        atomicAdd(&pair_counts[0], e);
        atomicAdd(&pair_counts[1], u);
        atomicAdd(&pair_counts[2], (unsigned long long)wc.walk);
        atomicAdd(&pair_counts[3], (unsigned long long)wc.test);
        atomicMax(&pair_counts[4], (unsigned long long)wc.walk);
        if (wave == 0) atomicMax(&pair_counts[5], (unsigned long long)len);
        if (s_walk) s_walk[wave] = wc.test;
    }
}

// One block per tile (compact id blk, taken in the order given, heaviest
// lists first): composite the whole list, then write the pixels.  kPatch:
// ROI patch of the affiliated eye (writes the depth proxy and the class).
template <bool kCount, bool kPatch, bool kXfer = false>
__global__ __launch_bounds__(256) void k_blend(const SurfelRec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                               const uint2* __restrict__ ranges, const uint32_t* __restrict__ tile_list,
                                               const uint32_t* __restrict__ order,
                                               const uint32_t* __restrict__ n_live, BlendArgs a, ContArgs ca,
                                               float* __restrict__ rgb, float* __restrict__ dz,
                                               float* __restrict__ alpha, uint8_t* __restrict__ cls,
                                               unsigned long long* __restrict__ pair_counts,
                                               long long* __restrict__ trace) {
    __shared__ float4 s_rec[(kBatch + 1) * 4];
    __shared__ float4 s_xc[kXfer ? kBatch + 1 : 1];  // transfer colours, one per staged record
    __shared__ __align__(8) uint16_t s_list[4 * kListLen];
    __shared__ uint32_t s_walk[4];
    __shared__ uint32_t s_slot, s_ibase, s_nseg;
    __shared__ float s_far[4];
    const long long t_begin = kCount ? wall_clock64() : 0;
    const uint32_t blk = blockIdx.x;
    if (n_live && blk >= *n_live) return;
    const uint32_t cid = order ? order[blk] : blk;
    const uint32_t tile = tile_list ? tile_list[cid] : cid;
    bool inside;
    int px, py;
    const TileGeom g = tile_geom(tile, (int)threadIdx.x, a, &inside, &px, &py);
    const uint2 rg = ranges[cid];
    PixelState p{inside ? 1.f : 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    WalkCounts wc{0, 0, 0, 0};
    if (g.tid < 4) s_rec[4 * kDummy + g.tid] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (kXfer && g.tid == 0) s_xc[kDummy] = make_float4(0.f, 0.f, 0.f, 0.f);
    uint16_t* my_list = s_list + (g.tid >> 6) * kListLen;
    // The transfer keeps three more sums per pixel, which the continuation
    // does not carry: such a walk never hands over.
    const uint32_t cap_end = (!kXfer && ca.cap && ca.max_slots && rg.y - rg.x > ca.cap) ? rg.x + ca.cap : rg.y;
    // A capped walk also breaks its batches at its midpoint, where the
    // transmittance is sampled for the hand-over decision.
    const uint32_t mid = cap_end < rg.y ? rg.x + (cap_end - rg.x) / 2 : rg.y;
    float t_half = 1.f;
    uint32_t at_half = rg.x;  // records walked when t_half was taken
    bool half_taken = false, handed = false;
    // One batch loop over the whole list; batches stop at the cap, where the
    // tile decides once whether to hand the rest over (then it leaves the
    // loop) or to walk on.
    float4 q0, q1, q2, q3, qx;
    if (rg.x + g.tid < rg.y) load_rec<kXfer>(recs, vals, rg.x + g.tid, a, q0, q1, q2, q3, qx);
    for (uint32_t base = rg.x; base < rg.y;) {
        const uint32_t lim = base < mid ? mid : base < cap_end ? cap_end : rg.y;
        const uint32_t nb = min((uint32_t)kBatch, lim - base);
        __syncthreads();
        if ((uint32_t)g.tid < nb) {
            stage_rec(s_rec, g.tid, q0, q1, q2, q3);
            if (kXfer) s_xc[g.tid] = qx;
        }
        __syncthreads();
        if (base + nb + g.tid < rg.y) load_rec<kXfer>(recs, vals, base + nb + g.tid, a, q0, q1, q2, q3, qx);
        walk_batch<kCount, kXfer>(s_rec, nb, my_list, g, a, p, wc, s_xc);
        base += nb;
        if (!half_taken && base >= mid) {
            half_taken = true;
            t_half = p.T;
            at_half = base;
        }
        const int n_live_px = __syncthreads_count(live(p));
        if (n_live_px == 0) break;
        if (base != cap_end || cap_end == rg.y) continue;
        // Pixels still compositing past the cap: hand the rest of the list
        // to continuation segments if a slot is free and the split pays,
        // else walk on.  It pays when some pixel is expected to walk far:
        // extrapolating the transmittance's decay over the second half of
        // the capped walk, a pixel needs about ln(T / t_min) / (decay per
        // record) more records.  Segments started for pixels that will stop
        // soon would mostly be walked in vain.
        float far = 0.f;
        if (live(p)) {
            const float drop = t_half > p.T ? __logf(t_half / p.T) : 0.f;
            const float need = __logf(p.T / a.t_min) * (float)(cap_end - at_half);
            far = need >= 1e30f * drop ? 1e30f : need / drop;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) far = fmaxf(far, __shfl_xor(far, off, 64));
        if (g.lane == 0) s_far[g.tid >> 6] = far;
        __syncthreads();
        const float far_max = fmaxf(fmaxf(s_far[0], s_far[1]), fmaxf(s_far[2], s_far[3]));
        const uint32_t rem = rg.y - cap_end;
        if (g.tid == 0) {
            s_slot = 0xFFFFFFFFu;
            if (far_max >= (float)ca.min_far && rem >= 2 * ca.seg_len) {
                const uint32_t slot = atomicAdd(ca.n_slots, 1u);
                if (slot < ca.max_slots) {
                    const uint32_t nseg = min(kContMaxSeg, max(1u, (rem + ca.seg_len - 1) / ca.seg_len));
                    const uint32_t ibase = atomicAdd(ca.n_items, nseg);
                    ca.slot_desc[slot] = make_uint4(cid, cap_end, rg.y, ibase | (nseg << kContSegShift));
                    s_slot = slot;
                    s_ibase = ibase;
                    s_nseg = nseg;
                }
            }
        }
        __syncthreads();
        const uint32_t slot = s_slot;
        if (slot != 0xFFFFFFFFu) {
            if ((uint32_t)g.tid < s_nseg) ca.item_slot[s_ibase + g.tid] = slot;
            float4* st = ca.st1 + (size_t)slot * 512;
            st[2 * g.tid] = make_float4(p.c0, p.c1, p.c2, p.D);
            st[2 * g.tid + 1] = make_float4(p.A, p.T, live(p) ? 1.f : 0.f, 0.f);
            handed = live(p);  // pixels already done are final now
            break;
        }
    }
    if (kCount) {
        count_flush(wc, g.lane, g.tid >> 6, rg.y - rg.x, pair_counts, s_walk);
        __syncthreads();
        if (trace && g.tid == 0) {
            // Per tile: id, list length, most records one wave evaluated, CU,
            // start, end.
            long long* t = trace + 6 * (long long)blk;
            t[0] = tile;
            t[1] = rg.y - rg.x;
            t[2] = max(max(s_walk[0], s_walk[1]), max(s_walk[2], s_walk[3]));
            t[3] = __smid();
            t[4] = t_begin;
            t[5] = wall_clock64();
        }
    }
    if (inside && !handed) write_pixel<kPatch, kXfer>(p, px, py, a, rgb, dz, alpha, cls);
}

// ---------------------------------------------------------------------------
// Continuation of the lists handed over by k_blend.  Segment k of a slot's
// remaining records is walked by k_blend_seg from an upper bound of the
// true transmittance at the segment's start: its sums divided by that bound
// are the segment's contribution per unit of incoming transmittance, which
// chains exactly while no pixel would stop inside the segment, and a pixel
// that stops in this walk stops at or before the same record in the true
// one.
// k_blend_chain chains a slot's segments for every pixel and writes the
// pixels that never stop; a pixel whose transmittance would cross t_min
// inside a segment (or that stopped in the speculative walk) is composited
// again over that segment, in order, from its exact state, by k_blend_fix,
// and written there.  k_blend writes the pixels already done when it hands
// a tile over, so every pixel is written once.
// ---------------------------------------------------------------------------
struct Chain {
    float T, c0, c1, c2, D, A;
};

// One segment of the chain.  Returns false where the pixel stops inside the
// segment (nothing is added then).
// One segment of the chain; the segment's sums are stored per unit of the
// transmittance its walk started from.  Returns false where the pixel stops
// inside the segment, or the segment was not walked for it (nothing is added
// then).
__device__ __forceinline__ bool chain_step(const float4& x0, const float4& x1, float t_min, Chain& c) {
    if (x1.z != 0.f || c.T * x1.y < t_min) return false;
    c.c0 = fmaf(c.T, x0.x, c.c0);
    c.c1 = fmaf(c.T, x0.y, c.c1);
    c.c2 = fmaf(c.T, x0.z, c.c2);
    c.D = fmaf(c.T, x0.w, c.D);
    c.A = fmaf(c.T, x1.x, c.A);
    c.T *= x1.y;
    return true;
}

__device__ __forceinline__ void item_segment(const uint4& d, uint32_t k, uint32_t* sb, uint32_t* se) {
    const uint32_t nseg = d.w >> kContSegShift;
    const uint64_t rem = d.z - d.y;
    *sb = d.y + (uint32_t)(rem * k / nseg);
    *se = d.y + (uint32_t)(rem * (k + 1) / nseg);
}

// Round 0 walks the first segments of every continued tile from the
// transmittance T1 after the capped walk.  Each later round (if kRounds > 1)
// walks its segments from every pixel's exact transmittance after the
// segments of the rounds before (a tighter bound than T1), and only for the
// pixels that get through them.
template <bool kCount>
__global__ __launch_bounds__(256) void k_blend_seg(const SurfelRec* __restrict__ recs,
                                                   const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ tile_list, BlendArgs a, ContArgs ca,
                                                   int round, unsigned long long* __restrict__ pair_counts) {
    __shared__ float4 s_rec[(kBatch + 1) * 4];
    __shared__ __align__(8) uint16_t s_list[4 * kListLen];
    const uint32_t n_items = min(*ca.n_items, ca.max_slots * kContMaxSeg);
    if (blockIdx.x >= n_items) return;
    const int tid = (int)threadIdx.x;
    if (tid < 4) s_rec[4 * kDummy + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
    WalkCounts wc{0, 0, 0, 0};
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint32_t slot = ca.item_slot[item];
        const uint4 d = ca.slot_desc[slot];
        const uint32_t ibase = d.w & ((1u << kContSegShift) - 1u), k = item - ibase;
        const uint32_t lo = round_lo(round);
        if (k < lo || k >= round_lo(round + 1)) continue;
        uint32_t sb, se;
        item_segment(d, k, &sb, &se);
        bool inside;
        int px, py;
        const TileGeom g = tile_geom(tile_list ? tile_list[d.x] : d.x, tid, a, &inside, &px, &py);
        const float4 s1 = ca.st1[(size_t)slot * 512 + 2 * tid + 1];
        Chain c{s1.y, 0.f, 0.f, 0.f, 0.f, 0.f};
        bool live = s1.z != 0.f;
        // Chain the lo segments of the earlier rounds, four parts loaded
        // together at a time.
        const float4* xb = ca.part + (size_t)ibase * 512 + 2 * tid;
        for (uint32_t j0 = 0; j0 < lo && live; j0 += 4) {
            float4 x0[4], x1[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                if (j0 + u < lo) {
                    x0[u] = xb[(size_t)(j0 + u) * 512];
                    x1[u] = xb[(size_t)(j0 + u) * 512 + 1];
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u)
                if (j0 + u < lo && live) live = chain_step(x0[u], x1[u], a.t_min, c);
        }
        const float ts = c.T;
        PixelState p{live ? ts : 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (__syncthreads_or(live))
            walk_range<kCount>(recs, vals, sb, se, s_rec, s_list + (tid >> 6) * kListLen, g, a, p, wc);
        const float inv = live ? 1.f / ts : 0.f;
        float4* o = ca.part + (size_t)item * 512;
        o[2 * tid] = make_float4(p.c0 * inv, p.c1 * inv, p.c2 * inv, p.D * inv);
        o[2 * tid + 1] = make_float4(p.A * inv, p.T * inv, live ? (p.T > 0.f ? 0.f : 1.f) : 3.f, 0.f);
    }
    if (kCount) count_flush(wc, tid & 63, tid >> 6, 0, pair_counts, nullptr);
}

// After all segment rounds, one workgroup per slot chains the segments of
// every pixel from the state after the capped walk.  A pixel that never
// stops is written here, and so is one that stops in a segment walked from
// its exact transmittance; for one that stops inside any other segment j
// (or stopped in its speculative walk), the exact state at the start of
// segment j and j + 1 replace the slot's state after the capped walk, for
// k_blend_fix.
template <bool kPatch>
__global__ __launch_bounds__(256) void k_blend_chain(const uint32_t* __restrict__ tile_list, BlendArgs a, ContArgs ca,
                                                     float* __restrict__ rgb, float* __restrict__ dz,
                                                     float* __restrict__ alpha, uint8_t* __restrict__ cls) {
    const uint32_t n_slots = min(*ca.n_slots, ca.max_slots);
    const int tid = (int)threadIdx.x;
    for (uint32_t slot = blockIdx.x; slot < n_slots; slot += gridDim.x) {
        const uint4 d = ca.slot_desc[slot];
        const uint32_t ibase = d.w & ((1u << kContSegShift) - 1u), nseg = d.w >> kContSegShift;
        bool inside;
        int px, py;
        (void)tile_geom(tile_list ? tile_list[d.x] : d.x, tid, a, &inside, &px, &py);
        float4* st = ca.st1 + (size_t)slot * 512 + 2 * tid;
        const float4 s0 = st[0], s1 = st[1];
        if (s1.z == 0.f) continue;  // done before the cap and written then
        Chain c{s1.y, s0.x, s0.y, s0.z, s0.w, s1.x};
        uint32_t stop = nseg;
        bool exact = false;
        const float4* xb = ca.part + (size_t)ibase * 512 + 2 * tid;
        for (uint32_t j0 = 0; j0 < nseg && stop == nseg; j0 += kChainBatch) {
            float4 x0[kChainBatch], x1[kChainBatch];
#pragma unroll
            for (uint32_t u = 0; u < kChainBatch; ++u) {
                if (j0 + u < nseg) {
                    x0[u] = xb[(size_t)(j0 + u) * 512];
                    x1[u] = xb[(size_t)(j0 + u) * 512 + 1];
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < kChainBatch; ++u) {
                const uint32_t j = j0 + u;
                if (j < nseg && stop == nseg && !chain_step(x0[u], x1[u], a.t_min, c)) {
                    stop = j;
                    // The first segment of each round was walked from the
                    // pixel's exact transmittance: where the pixel stopped
                    // in that walk, the walk is the true one and needs no
                    // repeat.
                    if (x1[u].z == 1.f && (j == round_lo(0) || j == round_lo(1))) {
                        c.c0 = fmaf(c.T, x0[u].x, c.c0);
                        c.c1 = fmaf(c.T, x0[u].y, c.c1);
                        c.c2 = fmaf(c.T, x0[u].z, c.c2);
                        c.D = fmaf(c.T, x0[u].w, c.D);
                        c.A = fmaf(c.T, x1[u].x, c.A);
                        c.T = 0.f;
                        exact = true;
                    }
                }
            }
        }
        if (stop == nseg || exact) {
            if (inside) write_pixel<kPatch>(PixelState{c.T, c.c0, c.c1, c.c2, c.D, c.A}, px, py, a, rgb, dz, alpha, cls);
            st[1] = make_float4(c.A, c.T, 0.f, 0.f);
        } else {
            st[0] = make_float4(c.c0, c.c1, c.c2, c.D);
            st[1] = make_float4(c.A, c.T, (float)(stop + 1), 0.f);
        }
    }
}

// Item k of a slot composites segment k again, in order, from the exact
// state k_blend_chain recorded, for the pixels that stop inside it, and
// writes them.
template <bool kCount, bool kPatch>
__global__ __launch_bounds__(256) void k_blend_fix(const SurfelRec* __restrict__ recs,
                                                   const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ tile_list, BlendArgs a, ContArgs ca,
                                                   float* __restrict__ rgb, float* __restrict__ dz,
                                                   float* __restrict__ alpha, uint8_t* __restrict__ cls,
                                                   unsigned long long* __restrict__ pair_counts) {
    __shared__ float4 s_rec[(kBatch + 1) * 4];
    __shared__ __align__(8) uint16_t s_list[4 * kListLen];
    const uint32_t n_items = min(*ca.n_items, ca.max_slots * kContMaxSeg);
    if (blockIdx.x >= n_items) return;
    const int tid = (int)threadIdx.x;
    if (tid < 4) s_rec[4 * kDummy + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
    WalkCounts wc{0, 0, 0, 0};
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint32_t slot = ca.item_slot[item];
        const uint4 d = ca.slot_desc[slot];
        const uint32_t k = item - (d.w & ((1u << kContSegShift) - 1u));
        const float4 s0 = ca.st1[(size_t)slot * 512 + 2 * tid], s1 = ca.st1[(size_t)slot * 512 + 2 * tid + 1];
        const bool need = s1.z == (float)(k + 1);
        if (!__syncthreads_or(need)) continue;
        uint32_t sb, se;
        item_segment(d, k, &sb, &se);
        bool inside;
        int px, py;
        const TileGeom g = tile_geom(tile_list ? tile_list[d.x] : d.x, tid, a, &inside, &px, &py);
        PixelState q{need ? s1.y : 0.f, s0.x, s0.y, s0.z, s0.w, s1.x};
        walk_range<kCount>(recs, vals, sb, se, s_rec, s_list + (tid >> 6) * kListLen, g, a, q, wc);
        // A pixel still compositing at the segment's end (whose crossing of
        // t_min the chained product placed in this segment by rounding) walks
        // on, in order, to its stop or the end of the list.
        if (__syncthreads_or(live(q)))
            walk_range<kCount>(recs, vals, se, d.z, s_rec, s_list + (tid >> 6) * kListLen, g, a, q, wc);
        if (inside && need) write_pixel<kPatch>(q, px, py, a, rgb, dz, alpha, cls);
    }
    if (kCount) count_flush(wc, tid & 63, tid >> 6, 0, pair_counts, nullptr);
}

}  // namespace

hipError_t launch_preprocess(const SceneArgs& sc, const PreCam& cam, float alpha_min, int lowpass,
                             const MaskArgs& mask, SurfelRec* recs, uint32_t* zkeys, uint2* rects,
                             uint32_t* counts, const PreCam* cam2, SurfelRec* recs2, uint32_t* zkeys2,
                             uint2* rects2, uint32_t* nseg, hipStream_t s) {
    if (sc.n <= 0) return hipSuccess;
    const dim3 g((sc.n + 255) / 256);
    if (cam2)
        hipLaunchKernelGGL(k_preprocess<true>, g, dim3(256), 0, s, sc, cam, *cam2, alpha_min, lowpass, mask, recs, zkeys,
                           rects, counts, recs2, zkeys2, rects2, nseg);
    else
        hipLaunchKernelGGL(k_preprocess<false>, g, dim3(256), 0, s, sc, cam, cam, alpha_min, lowpass, mask, recs, zkeys,
                           rects, counts, nullptr, nullptr, nullptr, nseg);
    return hipGetLastError();
}

hipError_t launch_masked_counts_ordered(const uint2* rects, const SurfelRec* recs, const uint32_t* order, int n,
                                        int n_tiles, const MaskArgs& mask, uint32_t* counts, uint32_t* partials,
                                        uint32_t* nseg, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // The mask prefix is read from global memory (it stays in L2): staging it
    // in LDS per workgroup cost more than the lookups (emission and counts of
    // a 1M-surfel, 6700-tile ROI pass: 111 -> 94 us).
    const int mask_lds = 0;
    hipLaunchKernelGGL(k_masked_counts_ordered, dim3((unsigned)((n + 255) / 256)), dim3(256),
                       (size_t)mask_lds * sizeof(uint32_t), s, rects, recs, order, n, mask, mask_lds, counts,
                       partials, nseg);
    return hipGetLastError();
}

hipError_t launch_masked_counts(const uint2* rects, const SurfelRec* recs, int n, int n_tiles, const MaskArgs& mask,
                                uint32_t* counts, uint32_t* nseg, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int mask_lds = n_tiles + 1 <= kEmitMaskLds ? n_tiles + 1 : 0;
    hipLaunchKernelGGL(k_masked_counts, dim3((n + 255) / 256), dim3(256), (size_t)mask_lds * sizeof(uint32_t), s,
                       rects, recs, n, mask, mask_lds, counts, nseg);
    return hipGetLastError();
}

hipError_t launch_emit(const uint32_t* order, const uint32_t* offs, const uint2* rects, const SurfelRec* recs, int n,
                       int tiles_x, int n_tiles, const MaskArgs& mask, uint32_t cap, int vbits, uint32_t* tkeys,
                       uint32_t* tvals, const uint32_t* nseg, int nseg_by_pos, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (vbits < 0 || vbits > 31 || (vbits && (int64_t)n > ((int64_t)1 << vbits))) return hipErrorInvalidValue;
    const int mask_lds = 0;  // the mask prefix is read from global memory (see launch_masked_counts_ordered)
    // Unmasked, the surfels nearest the camera (first in compositing order)
    // carry several times the mean key count: 128 surfels per workgroup
    // halve the heaviest workgroups (65 -> 49 us on a 5.9M-key frame).
    // Masked, most surfels have no key and 256 per workgroup cost less.
    const int spb = mask.enabled ? 256 : 128;
    hipLaunchKernelGGL(k_emit, dim3((n + spb - 1) / spb), dim3(256), (size_t)mask_lds * sizeof(uint32_t), s, order,
                       offs, rects, recs, n, spb, tiles_x, mask, mask_lds, cap, vbits, tkeys, tvals, nseg, nseg_by_pos);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched blend: one persistent launch over the tiles of many frames.  Each
// workgroup takes the next (frame, compact tile) item from a queue counter,
// composites the tile's whole list (no continuation: the batch itself keeps
// the GPU full) and writes its pixels, until the queue is empty.  Items go
// frame by frame, each frame's tiles heaviest first.  Workgroups never wait
// for one another, so every workgroup reaches the end of the queue.
// ---------------------------------------------------------------------------
__global__ void k_put_desc(BatchBlendDesc d, BatchBlendDesc* dst) {
    if (threadIdx.x == 0) *dst = d;
}

hipError_t launch_put_desc(const BatchBlendDesc& d, BatchBlendDesc* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, dst);
    return hipGetLastError();
}

__global__ void k_batch_prefix(const BatchBlendDesc* __restrict__ descs, int n, uint32_t* __restrict__ prefix,
                               uint32_t* __restrict__ counter) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int f = 0; f < n; ++f) {
        prefix[f] = run;
        run += descs[f].n_live ? min(*descs[f].n_live, descs[f].n_tiles) : descs[f].n_tiles;
    }
    prefix[n] = run;
    *counter = 0u;
}

template <bool kPatch>
__global__ __launch_bounds__(256) void k_blend_batch(const BatchBlendDesc* __restrict__ descs, int n,
                                                     const uint32_t* __restrict__ prefix, uint32_t* counter) {
    __shared__ float4 s_rec[(kBatch + 1) * 4];
    __shared__ __align__(8) uint16_t s_list[4 * kListLen];
    __shared__ uint32_t s_item;
    const int tid = (int)threadIdx.x;
    if (tid < 4) s_rec[4 * kDummy + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t total = prefix[n];
    WalkCounts wc{0, 0, 0, 0};
    for (;;) {
        __syncthreads();  // the previous item's use of s_item and the LDS batches is over
        if (tid == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= total) break;
        // The frame: the last f with prefix[f] <= item (a frame with no item
        // shares its prefix with the next one and is never chosen).
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchBlendDesc d = descs[lo];
        const uint32_t blk = item - prefix[lo];
        const uint32_t cid = d.order ? d.order[blk] : blk;
        const uint32_t tile = d.tile_list ? d.tile_list[cid] : cid;
        bool inside;
        int px, py;
        const TileGeom g = tile_geom(tile, tid, d.a, &inside, &px, &py);
        const uint2 rg = d.ranges[cid];
        PixelState p{inside ? 1.f : 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        walk_range<false>(d.recs, d.vals, rg.x, rg.y, s_rec, s_list + (tid >> 6) * kListLen, g, d.a, p, wc);
        if (inside) write_pixel<kPatch>(p, px, py, d.a, d.rgb, d.dz, d.alpha, d.cls);
    }
}

hipError_t launch_blend_batch(const BatchBlendDesc* descs, int n, uint32_t* scratch, int grid, bool patch,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    uint32_t* prefix = scratch;
    uint32_t* counter = scratch + n + 1;
    hipLaunchKernelGGL(k_batch_prefix, dim3(1), dim3(64), 0, s, descs, n, prefix, counter);
    if (patch)
        hipLaunchKernelGGL((k_blend_batch<true>), dim3(grid), dim3(256), 0, s, descs, n, prefix, counter);
    else
        hipLaunchKernelGGL((k_blend_batch<false>), dim3(grid), dim3(256), 0, s, descs, n, prefix, counter);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mask_to16(const uint8_t* __restrict__ tm, int T, int tw, int th, int tiles_x,
                                                   int tiles_y, uint8_t* __restrict__ m16) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= tiles_x * tiles_y) return;
    const int tx = t % tiles_x, ty = t / tiles_x;
    uint8_t v = 0;
    if (T == 32) {
        v = tm[(ty >> 1) * tw + (tx >> 1)] != 0;
    } else {  // T == 8: any of the (up to) four 8x8 tiles of this 16x16 tile
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int qx = 2 * tx + dx, qy = 2 * ty + dy;
                if (qx < tw && qy < th && tm[qy * tw + qx]) v = 1;
            }
    }
    m16[t] = v;
}

hipError_t launch_mask_to16(const uint8_t* tmask, int T, int W, int H, uint8_t* mask16, hipStream_t s) {
    if (T != 8 && T != 32) return hipErrorInvalidValue;
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const int tw = (W + T - 1) / T, th = (H + T - 1) / T;
    hipLaunchKernelGGL(k_mask_to16, dim3((unsigned)((tiles_x * tiles_y + 255) / 256)), dim3(256), 0, s, tmask, T, tw,
                       th, tiles_x, tiles_y, mask16);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mask_copy(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                   int64_t n, uint32_t mask) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i] & mask;
}

hipError_t launch_mask_copy(const uint32_t* src, uint32_t* dst, int64_t n, uint32_t mask, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mask_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n, mask);
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* tkeys, const uint32_t* n_dev, int64_t cap, uint2* ranges, int n_tiles,
                         int key_shift, hipStream_t s) {
    if (key_shift < 0 || key_shift > 31) return hipErrorInvalidValue;
    if (n_tiles <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(4096, std::max<int64_t>(1, (cap + 1023) / 1024));
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s, tkeys, n_dev, ranges, (uint32_t)n_tiles,
                       key_shift);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_u2(uint2* p, int64_t n, uint2 v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_clear_ranges(uint2* ranges, int n_tiles, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u2, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, s, ranges, (int64_t)n_tiles,
                       make_uint2(0u, 0u));
    return hipGetLastError();
}

hipError_t launch_tile_order(const uint2* ranges, const uint32_t* n_live, int n_tiles, uint32_t* order,
                             hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, ranges, n_live, (uint32_t)n_tiles, order);
    return hipGetLastError();
}

hipError_t launch_blend(const SurfelRec* recs, const uint32_t* vals, const uint2* ranges, const uint32_t* tile_list,
                        const uint32_t* order, const uint32_t* n_live, int n_blocks, const BlendArgs& a,
                        const ContArgs& ca, float* rgb, float* d_or_z, float* alpha, uint8_t* cls,
                        unsigned long long* pair_counts, long long* trace, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    const dim3 g(n_blocks), b(256);
    const bool cont = ca.cap != 0 && ca.max_slots != 0;
    const dim3 gc(min(ca.max_slots * kContMaxSeg, 4096u)), gs(ca.max_slots);
    if (a.patch && a.xrecs) return hipErrorInvalidValue;  // the transfer belongs to the dominant eye
    if (a.patch) {
        if (pair_counts) {
            hipLaunchKernelGGL((k_blend<true, true>), g, b, 0, s, recs, vals, ranges, tile_list, order, n_live, a, ca,
                               rgb, d_or_z, alpha, cls, pair_counts, trace);
            if (cont) {
                for (int round = 0; round < kRounds; ++round)
                    hipLaunchKernelGGL((k_blend_seg<true>), gc, b, 0, s, recs, vals, tile_list, a, ca, round,
                                       pair_counts);
                hipLaunchKernelGGL((k_blend_chain<true>), gs, b, 0, s, tile_list, a, ca, rgb, d_or_z, alpha, cls);
                hipLaunchKernelGGL((k_blend_fix<true, true>), gc, b, 0, s, recs, vals, tile_list, a, ca, rgb, d_or_z,
                                   alpha, cls, pair_counts);
            }
        } else {
            hipLaunchKernelGGL((k_blend<false, true>), g, b, 0, s, recs, vals, ranges, tile_list, order, n_live, a, ca,
                               rgb, d_or_z, alpha, cls, pair_counts, (long long*)nullptr);
            if (cont) {
                for (int round = 0; round < kRounds; ++round)
                    hipLaunchKernelGGL((k_blend_seg<false>), gc, b, 0, s, recs, vals, tile_list, a, ca, round,
                                       pair_counts);
                hipLaunchKernelGGL((k_blend_chain<true>), gs, b, 0, s, tile_list, a, ca, rgb, d_or_z, alpha, cls);
                hipLaunchKernelGGL((k_blend_fix<false, true>), gc, b, 0, s, recs, vals, tile_list, a, ca, rgb, d_or_z,
                                   alpha, cls, pair_counts);
            }
        }
    } else {
        if (pair_counts && a.xrecs) {
            hipLaunchKernelGGL((k_blend<true, false, true>), g, b, 0, s, recs, vals, ranges, tile_list, order, n_live,
                               a, ca, rgb, d_or_z, alpha, cls, pair_counts, trace);
        } else if (pair_counts) {
            hipLaunchKernelGGL((k_blend<true, false>), g, b, 0, s, recs, vals, ranges, tile_list, order, n_live, a, ca,
                               rgb, d_or_z, alpha, cls, pair_counts, trace);
            if (cont) {
                for (int round = 0; round < kRounds; ++round)
                    hipLaunchKernelGGL((k_blend_seg<true>), gc, b, 0, s, recs, vals, tile_list, a, ca, round,
                                       pair_counts);
                hipLaunchKernelGGL((k_blend_chain<false>), gs, b, 0, s, tile_list, a, ca, rgb, d_or_z, alpha, cls);
                hipLaunchKernelGGL((k_blend_fix<true, false>), gc, b, 0, s, recs, vals, tile_list, a, ca, rgb, d_or_z,
                                   alpha, cls, pair_counts);
            }
        } else if (a.xrecs) {
            // View-colour transfer: never continued.
            hipLaunchKernelGGL((k_blend<false, false, true>), g, b, 0, s, recs, vals, ranges, tile_list, order, n_live,
                               a, ca, rgb, d_or_z, alpha, cls, pair_counts, (long long*)nullptr);
        } else {
            hipLaunchKernelGGL((k_blend<false, false>), g, b, 0, s, recs, vals, ranges, tile_list, order, n_live, a,
                               ca, rgb, d_or_z, alpha, cls, pair_counts, (long long*)nullptr);
            if (cont) {
                for (int round = 0; round < kRounds; ++round)
                    hipLaunchKernelGGL((k_blend_seg<false>), gc, b, 0, s, recs, vals, tile_list, a, ca, round,
                                       pair_counts);
                hipLaunchKernelGGL((k_blend_chain<false>), gs, b, 0, s, tile_list, a, ca, rgb, d_or_z, alpha, cls);
                hipLaunchKernelGGL((k_blend_fix<false, false>), gc, b, 0, s, recs, vals, tile_list, a, ca, rgb,
                                   d_or_z, alpha, cls, pair_counts);
            }
        }
    }
    return hipGetLastError();
}

hipError_t launch_mask_tables(const uint8_t* tile_mask, int n_tiles, int tiles_x, uint32_t* prefix,
                              uint32_t* tile_list, uint32_t* colcum, DevStatus* st, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_tables, dim3(1), dim3(1024), 0, s, tile_mask, n_tiles, tiles_x, prefix, tile_list,
                       colcum, st);
    return hipGetLastError();
}

hipError_t launch_status_keys(const uint32_t* offs, int n, DevStatus* st, uint32_t cap, int which, hipStream_t s) {
    hipLaunchKernelGGL(k_status_keys, dim3(1), dim3(1), 0, s, offs, n, st, cap, which);
    return hipGetLastError();
}

}  // namespace bgs
