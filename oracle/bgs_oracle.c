/*
 * CPU oracle for the binocular 2DGS frame path.  TEST INFRASTRUCTURE ONLY:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path never calls it.
 *
 * Plain, slow and written for checking by eye against the paper: fp64
 * arithmetic, per-pixel brute force over every surfel, no tiling, no
 * sorting beyond one qsort per camera.  It shares no code with the HIP
 * library.
 *
 * What it follows (sections and equations of the paper):
 *   - 2D Gaussian surfel: centre p_k, tangents t_u, t_v, scales s_u, s_v,
 *     normal t_w = t_u x t_v (Sec. 3.3, Eq. 1); Gaussian
 *     G(u,v) = exp(-(u^2+v^2)/2) (Eq. 2); the pixel ray is intersected
 *     exactly with the surfel plane (Sec. 3.3, last paragraph).
 *   - Front-to-back compositing with w_i = alpha_i T_i; the depth proxy
 *     D = sum d_i w_i uses the same weights (Sec. 3.1, Stage 1).
 *   - Pinhole projection / unprojection and reprojection (Eq. 3-5).
 *   - Edge ROIs from reprojected boundary samples (Eq. 6-8), tile
 *     alignment and margin m (Sec. 3.5, Step 1).
 *   - Gap interpolation, center holes, connected components, bounding
 *     boxes expanded by m and tile aligned (Sec. 3.1 Stage 3-4, Sec. 3.5
 *     Step 2).
 *   - ROI re-rasterisation of the affiliated eye (Sec. 3.1 Stage 4).
 *
 * Readings where the paper is silent (the constants alpha_min = 1/255,
 * alpha_max = 0.99, T_min = 1e-4, the screen-space low-pass term, the SH
 * colour model inherited from 2DGS, the depth used when the low-pass term
 * wins, the fp32 sort key, the z-test, the interpolation rule) are given
 * where they are used below.
 *
 * Parity status: every function here is pinned by the CPU test-suite
 * (closed forms, invariants, brute force, independent library routines);
 * the choices the paper leaves open are pinned only by their stated
 * reading.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_API __attribute__((visibility("default")))

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9]; /* camera-to-world rotation, row-major */
    double t[3]; /* camera centre in world */
    double z_near, z_far;
} orc_camera;

typedef struct {
    double alpha_min, alpha_max, t_min;
    int32_t lowpass;
    int32_t pad;
    double bg[3];
} orc_raster;

typedef struct {
    int32_t margin, tile, edge_samples, gap_passes, center_roi;
    int32_t edge_bounds; /* 0: Eq. 6 over all samples; 1: each side from its own edge, worst case */
    double a_min;
} orc_roi;

/* ------------------------------------------------------------------ */
/* Real spherical harmonics from their definition:                     */
/*   Y_l^m = sqrt(2) K_l^m cos(m phi) P_l^m(cos theta)     m > 0       */
/*   Y_l^0 = K_l^0 P_l^0(cos theta)                                    */
/*   Y_l^m = sqrt(2) K_l^|m| sin(|m| phi) P_l^|m|(cos theta)  m < 0    */
/*   K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)                         */
/* with the Condon-Shortley phase inside P_l^m.  Coefficient index is  */
/* l*l + l + m.                                                        */
/* ------------------------------------------------------------------ */
static double assoc_legendre(int l, int m, double x) {
    double pmm = 1.0;
    if (m > 0) {
        double s = sqrt((1.0 - x) * (1.0 + x));
        double f = 1.0;
        for (int i = 1; i <= m; ++i) {
            pmm *= -f * s;
            f += 2.0;
        }
    }
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pll;
    }
    return pll;
}

static double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

static double sh_real(int l, int m, double theta, double phi) {
    int am = m < 0 ? -m : m;
    double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
    double P = assoc_legendre(l, am, cos(theta));
    if (m > 0) return sqrt(2.0) * K * cos(m * phi) * P;
    if (m < 0) return sqrt(2.0) * K * sin(am * phi) * P;
    return K * P;
}

/* Y values for unit directions dirs[3*i..], all coefficients up to deg. */
ORC_API void orc_sh_basis(int32_t deg, const double* dirs, int64_t m, double* out) {
    int nc = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < m; ++i) {
        double x = dirs[3 * i], y = dirs[3 * i + 1], z = dirs[3 * i + 2];
        double r = sqrt(x * x + y * y + z * z);
        double zz = z / r;
        if (zz > 1.0) zz = 1.0;
        if (zz < -1.0) zz = -1.0;
        double theta = acos(zz);
        double phi = atan2(y, x);
        for (int l = 0; l <= deg; ++l)
            for (int mm = -l; mm <= l; ++mm) out[i * nc + l * l + l + mm] = sh_real(l, mm, theta, phi);
    }
}

/* ------------------------------------------------------------------ */
/* Surfel preparation for one camera.                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    double pc[3];      /* centre in camera frame */
    double a[3], b[3]; /* tangents t_u, t_v in camera frame */
    double n[3];       /* normal a x b */
    double su, sv, o;
    double col[3];
    double mu[2];      /* projected centre, pixels */
    double reach;      /* radius of the alpha >= alpha_min disk: rho*max(su,sv) (0 if none) */
    double reach2d;    /* radius of the alpha >= alpha_min low-pass disk, pixels */
    float zkey;
    int64_t k;
} osurf;

typedef struct {
    int64_t n;
    int32_t sh_degree;
    const float *pos, *quat, *scale, *opacity, *sh;
} oscene;

/* The centre depth used as the compositing order key.  It is fp32 and is
 * computed with one fixed operation order so that any fp32 implementation
 * that follows the same order reproduces it bit for bit:
 *   z = ((r20*px + r21*py) + r22*pz) + tz
 * where (r20, r21, r22) is row 2 of the world-to-camera rotation R^T
 * (i.e. column 2 of R) and tz = -(((R02*t0 + R12*t1) + R22*t2)), each
 * rounded from fp64 to fp32; no fused multiply-add. */
static void zkey_coeffs(const orc_camera* c, float out[4]) {
    double r20 = c->R[0 * 3 + 2], r21 = c->R[1 * 3 + 2], r22 = c->R[2 * 3 + 2];
    double tz = -(((r20 * c->t[0]) + (r21 * c->t[1])) + (r22 * c->t[2]));
    out[0] = (float)r20;
    out[1] = (float)r21;
    out[2] = (float)r22;
    out[3] = (float)tz;
}

static float zkey_of(const float co[4], float px, float py, float pz) {
    float a = co[0] * px;
    float b = co[1] * py;
    float s = a + b;
    float c = co[2] * pz;
    s = s + c;
    return s + co[3];
}

ORC_API void orc_center_zkeys(const oscene* sc, const orc_camera* cam, float* zkeys) {
    float co[4];
    zkey_coeffs(cam, co);
    for (int64_t k = 0; k < sc->n; ++k)
        zkeys[k] = zkey_of(co, sc->pos[k], sc->pos[sc->n + k], sc->pos[2 * sc->n + k]);
}

static uint32_t fbits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static int cmp_surf(const void* x, const void* y) {
    const osurf* a = (const osurf*)x;
    const osurf* b = (const osurf*)y;
    uint32_t ka = fbits(a->zkey), kb = fbits(b->zkey);
    if (ka != kb) return ka < kb ? -1 : 1;
    return a->k < b->k ? -1 : (a->k > b->k ? 1 : 0);
}

/* World-to-camera: X_c = R^T (X_w - t). */
static void to_cam(const orc_camera* c, const double w[3], double out[3]) {
    double d0 = w[0] - c->t[0], d1 = w[1] - c->t[1], d2 = w[2] - c->t[2];
    for (int r = 0; r < 3; ++r) out[r] = c->R[0 * 3 + r] * d0 + c->R[1 * 3 + r] * d1 + c->R[2 * 3 + r] * d2;
}

static void rot_cam(const orc_camera* c, const double w[3], double out[3]) {
    for (int r = 0; r < 3; ++r) out[r] = c->R[0 * 3 + r] * w[0] + c->R[1 * 3 + r] * w[1] + c->R[2 * 3 + r] * w[2];
}

/* Rotation matrix of the unit quaternion q/|q| (w, x, y, z); columns are
 * t_u, t_v, t_w (Sec. 3.3). */
static void quat_frame(const double q0[4], double tu[3], double tv[3], double tw[3]) {
    double nq = sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
    double w = q0[0] / nq, x = q0[1] / nq, y = q0[2] / nq, z = q0[3] / nq;
    double R[3][3] = {
        {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
        {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
        {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)},
    };
    for (int r = 0; r < 3; ++r) {
        tu[r] = R[r][0];
        tv[r] = R[r][1];
        tw[r] = R[r][2];
    }
}

/* eye: the point the colours are seen from (NULL: the camera's own centre). */
static int prepare_eye(const oscene* sc, const orc_camera* cam, const double* eye, const orc_raster* rp,
                       osurf** out_list, int64_t* out_n) {
    if (!eye) eye = cam->t;
    int64_t n = sc->n;
    osurf* L = (osurf*)malloc(sizeof(osurf) * (size_t)(n > 0 ? n : 1));
    if (!L) return -1;
    float co[4];
    zkey_coeffs(cam, co);
    int nc = (sc->sh_degree + 1) * (sc->sh_degree + 1);
    int64_t m = 0;
    for (int64_t k = 0; k < n; ++k) {
        float px = sc->pos[k], py = sc->pos[n + k], pz = sc->pos[2 * n + k];
        float zk = zkey_of(co, px, py, pz);
        /* Surfels whose centre is not in front of the near plane are culled. */
        if (!((double)zk > cam->z_near)) continue;
        osurf* s = &L[m++];
        s->zkey = zk;
        s->k = k;
        double pw[3] = {px, py, pz};
        to_cam(cam, pw, s->pc);
        double q[4] = {sc->quat[k], sc->quat[n + k], sc->quat[2 * n + k], sc->quat[3 * n + k]};
        double tu[3], tv[3], tw[3];
        quat_frame(q, tu, tv, tw);
        rot_cam(cam, tu, s->a);
        rot_cam(cam, tv, s->b);
        s->n[0] = s->a[1] * s->b[2] - s->a[2] * s->b[1];
        s->n[1] = s->a[2] * s->b[0] - s->a[0] * s->b[2];
        s->n[2] = s->a[0] * s->b[1] - s->a[1] * s->b[0];
        s->su = sc->scale[k];
        s->sv = sc->scale[n + k];
        s->o = sc->opacity[k];
        s->mu[0] = cam->fx * s->pc[0] / s->pc[2] + cam->cx;
        s->mu[1] = cam->fy * s->pc[1] / s->pc[2] + cam->cy;
        /* Colour: degree-(deg) real SH evaluated towards the surfel from this
         * camera's centre (or the given eye), plus 0.5, clamped at 0 (the
         * 2DGS/3DGS colour model). */
        double dir[3] = {px - eye[0], py - eye[1], pz - eye[2]};
        double Y[16];
        orc_sh_basis(sc->sh_degree, dir, 1, Y);
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int c = 0; c < nc; ++c) acc += Y[c] * (double)sc->sh[(int64_t)(c * 3 + ch) * n + k];
            acc += 0.5;
            s->col[ch] = acc > 0.0 ? acc : 0.0;
        }
        double ratio = s->o / rp->alpha_min;
        if (ratio > 1.0) {
            double smax = s->su > s->sv ? s->su : s->sv;
            s->reach = sqrt(2.0 * log(ratio)) * smax;
            s->reach2d = sqrt(log(ratio));
        } else {
            s->reach = 0.0;
            s->reach2d = 0.0;
        }
    }
    qsort(L, (size_t)m, sizeof(osurf), cmp_surf);
    *out_list = L;
    *out_n = m;
    return 0;
}

static int prepare(const oscene* sc, const orc_camera* cam, const orc_raster* rp, osurf** out_list,
                   int64_t* out_n) {
    return prepare_eye(sc, cam, NULL, rp, out_list, out_n);
}

/* One (surfel, pixel) evaluation: exact ray-plane intersection (Sec. 3.3),
 * Gaussian of Eq. 2, optional screen-space low-pass term G2 =
 * exp(-|x - mu|^2) with G = max(G3, G2).  The depth d of the pair is the
 * intersection depth when the surfel's own Gaussian wins, else the centre
 * depth. */
typedef struct {
    double G3, G2, G, lambda, u, v, depth, cosang;
    int valid3;
} opair;

static void eval_pair(const osurf* s, const orc_camera* cam, const orc_raster* rp, double i, double j,
                      opair* e) {
    double r[3] = {(i - cam->cx) / cam->fx, (j - cam->cy) / cam->fy, 1.0};
    double nr = s->n[0] * r[0] + s->n[1] * r[1] + s->n[2] * r[2];
    double nn = sqrt(s->n[0] * s->n[0] + s->n[1] * s->n[1] + s->n[2] * s->n[2]);
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    e->cosang = fabs(nr) / (nn * rn);
    e->valid3 = 0;
    e->G3 = 0.0;
    e->lambda = 0.0;
    e->u = e->v = 0.0;
    if (fabs(nr) > 1e-12 * nn * rn) {
        double np = s->n[0] * s->pc[0] + s->n[1] * s->pc[1] + s->n[2] * s->pc[2];
        double lam = np / nr;
        e->lambda = lam;
        if (lam > cam->z_near) {
            double d[3] = {lam * r[0] - s->pc[0], lam * r[1] - s->pc[1], lam * r[2] - s->pc[2]};
            double u = (d[0] * s->a[0] + d[1] * s->a[1] + d[2] * s->a[2]) / s->su;
            double v = (d[0] * s->b[0] + d[1] * s->b[1] + d[2] * s->b[2]) / s->sv;
            e->u = u;
            e->v = v;
            e->G3 = exp(-0.5 * (u * u + v * v));
            e->valid3 = 1;
        }
    }
    e->G2 = 0.0;
    if (rp->lowpass) {
        double dx = i - s->mu[0], dy = j - s->mu[1];
        e->G2 = exp(-(dx * dx + dy * dy));
    }
    e->G = e->G3 > e->G2 ? e->G3 : e->G2;
    e->depth = (e->valid3 && e->G3 >= e->G2) ? e->lambda : s->pc[2];
}

/* Can the surfel reach alpha_min at this pixel at all?  A provable miss
 * lets the prefiltered mode skip it; the result is identical to visiting
 * every surfel because a skipped pair always has alpha well below
 * alpha_min (the tests check this bit for bit). */
static int may_touch(const osurf* s, const orc_camera* cam, double i, double j) {
    if (s->reach <= 0.0) return 0;
    double r[3] = {(i - cam->cx) / cam->fx, (j - cam->cy) / cam->fy, 1.0};
    double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double pr = s->pc[0] * r[0] + s->pc[1] * r[1] + s->pc[2] * r[2];
    double pp = s->pc[0] * s->pc[0] + s->pc[1] * s->pc[1] + s->pc[2] * s->pc[2];
    double dist2 = pp - pr * pr / rr;
    double R3 = s->reach * (1.0 + 1e-3);
    if (dist2 <= R3 * R3) return 1;
    double dx = i - s->mu[0], dy = j - s->mu[1];
    double R2 = s->reach2d * (1.0 + 1e-3) + 1e-6;
    if (dx * dx + dy * dy <= R2 * R2) return 1;
    return 0;
}

/* Ambiguity flags: threshold decisions that an fp32 evaluation of the same
 * pixel may take differently.  The bands are a few times the relative error
 * of fp32 arithmetic on fp32 inputs: alpha ~1e-6 (up to ~2e-5 for surfels
 * seen nearly edge-on), a transmittance product of ~100 factors ~1e-5. */
#define AMB_ALPHA 1 /* alpha within 5e-5 (relative) of alpha_min */
#define AMB_TSTOP 2 /* transmittance within 1e-4 (relative) of T_min */
#define AMB_DEPTH 4 /* G3 and G2 within 1e-5 (relative): depth choice */
#define AMB_GRAZE 8 /* contributing pair with a ray within 1e-3 of the surfel plane, or lambda near z_near */

static void render_pixel(const osurf* L, int64_t m, const orc_camera* cam, const orc_raster* rp, double i,
                         double j, int prefilter, double out[5], uint8_t* amb) {
    double T = 1.0, C[3] = {0, 0, 0}, D = 0.0, A = 0.0;
    uint8_t flags = 0;
    for (int64_t q = 0; q < m; ++q) {
        const osurf* s = &L[q];
        if (prefilter && !may_touch(s, cam, i, j)) continue;
        opair e;
        eval_pair(s, cam, rp, i, j, &e);
        double og = s->o * e.G;
        if (fabs(og - rp->alpha_min) <= 5e-5 * rp->alpha_min) flags |= AMB_ALPHA;
        double alpha = og < rp->alpha_max ? og : rp->alpha_max;
        if (alpha < rp->alpha_min) continue;
        if (e.G2 > 0.0 && fabs(e.G3 - e.G2) <= 1e-5 * e.G) flags |= AMB_DEPTH;
        if (e.valid3 && e.G3 >= e.G2 && alpha > 1e-3 &&
            (e.cosang < 1e-3 || fabs(e.lambda - cam->z_near) <= 1e-5 * cam->z_near))
            flags |= AMB_GRAZE;
        double Tn = T * (1.0 - alpha);
        if (fabs(Tn - rp->t_min) <= 1e-4 * rp->t_min) flags |= AMB_TSTOP;
        if (Tn < rp->t_min) break;
        double w = alpha * T;
        C[0] += w * s->col[0];
        C[1] += w * s->col[1];
        C[2] += w * s->col[2];
        D += w * e.depth;
        A += w;
        T = Tn;
    }
    out[0] = C[0] + T * rp->bg[0];
    out[1] = C[1] + T * rp->bg[1];
    out[2] = C[2] + T * rp->bg[2];
    out[3] = D;
    out[4] = A;
    *amb = flags;
}

/* Render a list of pixels (pix = NULL: every pixel, row-major).  Outputs
 * are planar per channel over the npx pixels: rgb[3][npx], depth_raw[npx]
 * (D = sum d_i w_i), alpha[npx] (A = sum w_i), amb[npx].  eye (NULL: the
 * camera's centre) is the point every surfel's colour is seen from; the
 * weights, depth and alpha are always the camera's own. */
ORC_API int orc_render_eye(const oscene* sc, const orc_camera* cam, const double* eye, const orc_raster* rp,
                           const int32_t* pix, int64_t npx, int32_t prefilter, int32_t nthreads, double* rgb,
                           double* depth_raw, double* alpha, uint8_t* amb) {
    osurf* L = NULL;
    int64_t m = 0;
    if (prepare_eye(sc, cam, eye, rp, &L, &m)) return -1;
    int64_t total = pix ? npx : (int64_t)cam->width * cam->height;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t p = 0; p < total; ++p) {
        double i, j;
        if (pix) {
            i = pix[2 * p];
            j = pix[2 * p + 1];
        } else {
            i = (double)(p % cam->width);
            j = (double)(p / cam->width);
        }
        double o[5];
        uint8_t f;
        render_pixel(L, m, cam, rp, i, j, prefilter, o, &f);
        rgb[p] = o[0];
        rgb[total + p] = o[1];
        rgb[2 * total + p] = o[2];
        depth_raw[p] = o[3];
        alpha[p] = o[4];
        if (amb) amb[p] = f;
    }
    free(L);
    return 0;
}

ORC_API int orc_render(const oscene* sc, const orc_camera* cam, const orc_raster* rp, const int32_t* pix,
                       int64_t npx, int32_t prefilter, int32_t nthreads, double* rgb, double* depth_raw,
                       double* alpha, uint8_t* amb) {
    return orc_render_eye(sc, cam, NULL, rp, pix, npx, prefilter, nthreads, rgb, depth_raw, alpha, amb);
}

/* Order in which surfels are composited: the surviving surfel indices
 * sorted by (fp32 centre-depth bits, index). */
ORC_API int64_t orc_composite_order(const oscene* sc, const orc_camera* cam, const orc_raster* rp,
                                    int64_t* order) {
    osurf* L = NULL;
    int64_t m = 0;
    if (prepare(sc, cam, rp, &L, &m)) return -1;
    for (int64_t q = 0; q < m; ++q) order[q] = L[q].k;
    free(L);
    return m;
}

/* Per-surfel pair quantities at one pixel, for closed-form checks:
 * out = {alpha, G3, G2, lambda, u, v, depth, valid3, colour r, g, b}. */
ORC_API int orc_pair(const oscene* sc, const orc_camera* cam, const orc_raster* rp, int64_t k, double i,
                     double j, double out[11]) {
    osurf* L = NULL;
    int64_t m = 0;
    if (prepare(sc, cam, rp, &L, &m)) return -1;
    int found = -1;
    for (int64_t q = 0; q < m; ++q)
        if (L[q].k == k) found = (int)q;
    if (found < 0) {
        free(L);
        return 1; /* culled */
    }
    opair e;
    eval_pair(&L[found], cam, rp, i, j, &e);
    double og = L[found].o * e.G;
    out[0] = og < rp->alpha_max ? og : rp->alpha_max;
    out[1] = e.G3;
    out[2] = e.G2;
    out[3] = e.lambda;
    out[4] = e.u;
    out[5] = e.v;
    out[6] = e.depth;
    out[7] = e.valid3;
    out[8] = L[found].col[0];
    out[9] = L[found].col[1];
    out[10] = L[found].col[2];
    free(L);
    return 0;
}

/* For every surfel, the pixel bounding box [x0,x1]x[y0,y1] (inclusive) of
 * the pixels where its alpha reaches alpha_min; x0 = -1 when there is
 * none.  Brute force over every pixel; used to check that a binning
 * scheme never drops a contributing pair. */
ORC_API int orc_coverage_boxes(const oscene* sc, const orc_camera* cam, const orc_raster* rp,
                               int32_t nthreads, int32_t* boxes) {
    osurf* L = NULL;
    int64_t m = 0;
    if (prepare(sc, cam, rp, &L, &m)) return -1;
    for (int64_t k = 0; k < sc->n; ++k) {
        boxes[4 * k] = -1;
        boxes[4 * k + 1] = -1;
        boxes[4 * k + 2] = -1;
        boxes[4 * k + 3] = -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
#endif
    for (int64_t q = 0; q < m; ++q) {
        const osurf* s = &L[q];
        int32_t x0 = INT32_MAX, y0 = INT32_MAX, x1 = -1, y1 = -1;
        for (int32_t j = 0; j < cam->height; ++j)
            for (int32_t i = 0; i < cam->width; ++i) {
                if (!may_touch(s, cam, i, j)) continue;
                opair e;
                eval_pair(s, cam, rp, i, j, &e);
                double og = s->o * e.G;
                double alpha = og < rp->alpha_max ? og : rp->alpha_max;
                if (alpha < rp->alpha_min) continue;
                if (i < x0) x0 = i;
                if (i > x1) x1 = i;
                if (j < y0) y0 = j;
                if (j > y1) y1 = j;
            }
        if (x1 >= 0) {
            int64_t k = s->k;
            boxes[4 * k] = x0;
            boxes[4 * k + 1] = y0;
            boxes[4 * k + 2] = x1;
            boxes[4 * k + 3] = y1;
        }
    }
    free(L);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Reprojection (Eq. 3-5) with a z-test.                               */
/* ------------------------------------------------------------------ */

/* Relative pose in fp64 with a fixed operation order:
 *   M = R_dst^T R_src,  c = R_dst^T (t_src - t_dst),
 * each entry summed as ((a0*b0 + a1*b1) + a2*b2).  A point in the source
 * camera frame X maps to X' = M X + c in the destination frame, which is
 * Eq. 4 followed by the transform inside Eq. 5. */
static void rel_pose(const orc_camera* src, const orc_camera* dst, double M[9], double c[3]) {
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            double p0 = dst->R[0 * 3 + r] * src->R[0 * 3 + q];
            double p1 = dst->R[1 * 3 + r] * src->R[1 * 3 + q];
            double p2 = dst->R[2 * 3 + r] * src->R[2 * 3 + q];
            M[r * 3 + q] = (p0 + p1) + p2;
        }
    double d0 = src->t[0] - dst->t[0], d1 = src->t[1] - dst->t[1], d2 = src->t[2] - dst->t[2];
    for (int r = 0; r < 3; ++r) {
        double p0 = dst->R[0 * 3 + r] * d0;
        double p1 = dst->R[1 * 3 + r] * d1;
        double p2 = dst->R[2 * 3 + r] * d2;
        c[r] = (p0 + p1) + p2;
    }
}

/* Map one source pixel (i, j) at depth d (fp64) into the destination
 * camera frame.  with_t = 0 drops the translation (a point at infinity).
 * Returns X' in out[3]. */
static void map_point(const double M[9], const double c[3], int with_t, double X, double Y, double Z,
                      double out[3]) {
    for (int r = 0; r < 3; ++r) {
        double p0 = M[r * 3 + 0] * X;
        double p1 = M[r * 3 + 1] * Y;
        double p2 = M[r * 3 + 2] * Z;
        double s = (p0 + p1) + p2;
        out[r] = with_t ? s + c[r] : s;
    }
}

/* Pinhole projection pi (Eq. 3) without rounding: u = fx*(X/Z) + cx. */
static void project(const orc_camera* cam, const double X[3], double* u, double* v) {
    double qx = X[0] / X[2];
    double qy = X[1] / X[2];
    double sx = cam->fx * qx;
    double sy = cam->fy * qy;
    *u = sx + cam->cx;
    *v = sy + cam->cy;
}

static uint64_t pack_key(float z, uint32_t s) { return ((uint64_t)fbits(z) << 32) | (uint64_t)s; }

/* Forward reprojection of the dominant image to the affiliated eye.
 * A source pixel with A >= a_min carries the depth proxy d = D/A (fp32
 * division) and is unprojected with pi^-1 (Eq. 4) and projected into the
 * destination (Eq. 5); a pixel with A < a_min is treated as background at
 * infinite depth (rotation only).  Each lands on the nearest destination
 * pixel (floor(x+0.5)); the z-test keeps the smallest (depth bits, source
 * index) key.  Destination pixels no source pixel reached are holes.
 * depth_range receives (min, max) of the fp32 depth proxy over pixels
 * with A >= a_min, or (z_near, z_far) of the source when there are none. */
ORC_API void orc_reproject(const orc_camera* src, const orc_camera* dst, double a_min, const float* rgb,
                           const float* depth_raw, const float* alpha, float* rgb_dst, float* z_dst,
                           float* alpha_dst, uint8_t* hole, uint64_t* zbuf, float* depth_range) {
    int64_t Ws = src->width, Hs = src->height, Wd = dst->width, Hd = dst->height;
    int64_t ns = Ws * Hs, nd = Wd * Hd;
    double M[9], c[3];
    rel_pose(src, dst, M, c);
    for (int64_t t = 0; t < nd; ++t) zbuf[t] = UINT64_MAX;
    float dmin = INFINITY, dmax = -INFINITY;
    int any = 0;
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = s % Ws, j = s / Ws;
        double xn = ((double)i - src->cx) / src->fx;
        double yn = ((double)j - src->cy) / src->fy;
        double Xp[3];
        int fg = alpha[s] >= (float)a_min; /* the threshold is an fp32 parameter */
        float zf;
        if (fg) {
            float df = depth_raw[s] / alpha[s];
            if (df < dmin) dmin = df;
            if (df > dmax) dmax = df;
            any = 1;
            double d = (double)df;
            map_point(M, c, 1, d * xn, d * yn, d, Xp);
            if (!(Xp[2] > dst->z_near)) continue;
            zf = (float)Xp[2];
        } else {
            map_point(M, c, 0, xn, yn, 1.0, Xp);
            if (!(Xp[2] > 0.0)) continue;
            zf = INFINITY;
        }
        double u, v;
        project(dst, Xp, &u, &v);
        double fu = floor(u + 0.5), fv = floor(v + 0.5);
        if (!(fu >= 0.0 && fu <= (double)(Wd - 1) && fv >= 0.0 && fv <= (double)(Hd - 1))) continue;
        int64_t t = (int64_t)fv * Wd + (int64_t)fu;
        uint64_t key = pack_key(zf, (uint32_t)s);
        if (key < zbuf[t]) zbuf[t] = key;
    }
    for (int64_t t = 0; t < nd; ++t) {
        uint64_t key = zbuf[t];
        if (key == UINT64_MAX) {
            hole[t] = 1;
            rgb_dst[t] = rgb_dst[nd + t] = rgb_dst[2 * nd + t] = 0.0f;
            z_dst[t] = INFINITY;
            alpha_dst[t] = 0.0f;
        } else {
            uint32_t s = (uint32_t)(key & 0xffffffffu);
            uint32_t zb = (uint32_t)(key >> 32);
            float z;
            memcpy(&z, &zb, 4);
            hole[t] = 0;
            rgb_dst[t] = rgb[s];
            rgb_dst[nd + t] = rgb[ns + s];
            rgb_dst[2 * nd + t] = rgb[2 * ns + s];
            z_dst[t] = z;
            alpha_dst[t] = alpha[s];
        }
    }
    if (any) {
        depth_range[0] = dmin;
        depth_range[1] = dmax;
    } else {
        depth_range[0] = (float)src->z_near;
        depth_range[1] = (float)src->z_far;
    }
}

/* ------------------------------------------------------------------ */
/* Hole classification: edge ROIs (Eq. 6-8), gap interpolation, center */
/* holes -> connected components -> boxes, ROI tile mask.              */
/* ------------------------------------------------------------------ */

enum { CLS_WARPED = 0, CLS_HOLE = 1, CLS_GAP = 2, CLS_ROI = 3, CLS_ROWFILL = 4 };
enum { BOX_LEFT = 0, BOX_RIGHT = 1, BOX_TOP = 2, BOX_BOTTOM = 3, BOX_CENTER = 4 };

static int64_t align_down(int64_t x, int64_t T) { return (x / T) * T; }
static int64_t align_up(int64_t x, int64_t T) { return ((x + T - 1) / T) * T; }

static double snap(double x) {
    double r = nearbyint(x);
    return fabs(x - r) <= 1e-6 ? r : x;
}

static double clampd(double x, double a, double b) { return x < a ? a : (x > b ? b : x); }

/* Sample position k of N along an edge of length L: round(k(L-1)/(N-1)),
 * halves rounded up, in integer arithmetic. */
static int64_t edge_pos(int64_t k, int64_t N, int64_t L) {
    if (N <= 1) return 0;
    return (2 * k * (L - 1) + (N - 1)) / (2 * (N - 1));
}

/* Step 1 (Eq. 6-8).  Writes the border widths (left, right, top, bottom)
 * and returns the number of edge boxes written to boxes[6*...]. */
ORC_API int orc_edge_rois(const orc_camera* src, const orc_camera* dst, const orc_roi* rp,
                          const float* depth_range, int32_t widths[4], int32_t* boxes) {
    double M[9], c[3];
    rel_pose(src, dst, M, c);
    int64_t N = rp->edge_samples;
    double hyp[2] = {(double)depth_range[0], (double)depth_range[1]};
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    /* The uncovered strip along a side ends where that side's own edge
       lands: at any depth in the range it is at most as wide as the worst
       case over the edge's samples and both hypotheses (largest x of the
       left edge, smallest x of the right edge, largest y of the top edge,
       smallest y of the bottom edge). */
    double left_x = -INFINITY, right_x = INFINITY, top_y = -INFINITY, bottom_y = INFINITY;
    int64_t Ws = src->width, Hs = src->height;
    for (int edge = 0; edge < 4; ++edge) {
        for (int64_t k = 0; k < N; ++k) {
            int64_t i, j;
            if (edge == 0) { i = edge_pos(k, N, Ws); j = 0; }
            else if (edge == 1) { i = edge_pos(k, N, Ws); j = Hs - 1; }
            else if (edge == 2) { i = 0; j = edge_pos(k, N, Hs); }
            else { i = Ws - 1; j = edge_pos(k, N, Hs); }
            double xn = ((double)i - src->cx) / src->fx;
            double yn = ((double)j - src->cy) / src->fy;
            for (int h = 0; h < 2; ++h) {
                double d = hyp[h];
                double Xp[3];
                map_point(M, c, 1, d * xn, d * yn, d, Xp);
                if (!(Xp[2] > dst->z_near)) continue;
                double u, v;
                project(dst, Xp, &u, &v);
                if (u < xmin) xmin = u;
                if (u > xmax) xmax = u;
                if (v < ymin) ymin = v;
                if (v > ymax) ymax = v;
                if (edge == 0 && v > top_y) top_y = v;
                if (edge == 1 && v < bottom_y) bottom_y = v;
                if (edge == 2 && u > left_x) left_x = u;
                if (edge == 3 && u < right_x) right_x = u;
            }
        }
    }
    if (rp->edge_bounds) {
        /* A side whose edge has no valid projection keeps Eq. 6. */
        if (left_x > -INFINITY) xmin = left_x;
        if (right_x < INFINITY) xmax = right_x;
        if (top_y > -INFINITY) ymin = top_y;
        if (bottom_y < INFINITY) ymax = bottom_y;
    }
    double W = dst->width, H = dst->height;
    double m = rp->margin;
    double hw = floor(W / 2.0), hh = floor(H / 2.0);
    double umin = snap(xmin), umax = snap(xmax), vmin = snap(ymin), vmax = snap(ymax);
    double lw = umin > 0.0 ? clampd(ceil(umin) + m, 0.0, hw) : 0.0;
    double rw = umax < W - 1.0 ? clampd((W - 1.0) - floor(umax) + m, 0.0, hw) : 0.0;
    double th = vmin > 0.0 ? clampd(ceil(vmin) + m, 0.0, hh) : 0.0;
    double bh = vmax < H - 1.0 ? clampd((H - 1.0) - floor(vmax) + m, 0.0, hh) : 0.0;
    widths[0] = (int32_t)lw;
    widths[1] = (int32_t)rw;
    widths[2] = (int32_t)th;
    widths[3] = (int32_t)bh;
    int64_t T = rp->tile, Wi = dst->width, Hi = dst->height;
    int nb = 0;
    if (widths[0] > 0) {
        int64_t x1 = align_up(widths[0], T);
        int32_t b[6] = {0, 0, (int32_t)(x1 < Wi ? x1 : Wi), (int32_t)Hi, BOX_LEFT, -1};
        memcpy(&boxes[6 * nb++], b, sizeof b);
    }
    if (widths[1] > 0) {
        int32_t b[6] = {(int32_t)align_down(Wi - widths[1], T), 0, (int32_t)Wi, (int32_t)Hi, BOX_RIGHT, -1};
        memcpy(&boxes[6 * nb++], b, sizeof b);
    }
    if (widths[2] > 0) {
        int64_t y1 = align_up(widths[2], T);
        int32_t b[6] = {0, 0, (int32_t)Wi, (int32_t)(y1 < Hi ? y1 : Hi), BOX_TOP, -1};
        memcpy(&boxes[6 * nb++], b, sizeof b);
    }
    if (widths[3] > 0) {
        int32_t b[6] = {0, (int32_t)align_down(Hi - widths[3], T), (int32_t)Wi, (int32_t)Hi, BOX_BOTTOM, -1};
        memcpy(&boxes[6 * nb++], b, sizeof b);
    }
    return nb;
}

static int in_boxes(const int32_t* boxes, int nb, int64_t x, int64_t y) {
    for (int b = 0; b < nb; ++b)
        if (x >= boxes[6 * b] && x < boxes[6 * b + 2] && y >= boxes[6 * b + 1] && y < boxes[6 * b + 3]) return 1;
    return 0;
}

/* Connected components of a binary mask with flood fill; every pixel of a
 * component gets the smallest linear index in it, non-mask pixels -1.
 * conn is 4 or 8. */
ORC_API int orc_label_components(const uint8_t* mask, int32_t W, int32_t H, int32_t conn, int32_t* labels) {
    int64_t n = (int64_t)W * H;
    int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!stack) return -1;
    for (int64_t p = 0; p < n; ++p) labels[p] = -1;
    for (int64_t p = 0; p < n; ++p) {
        if (!mask[p] || labels[p] >= 0) continue;
        int32_t lab = (int32_t)p;
        int64_t top = 0;
        stack[top++] = p;
        labels[p] = lab;
        while (top > 0) {
            int64_t q = stack[--top];
            int64_t x = q % W, y = q / W;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    if (conn == 4 && dx && dy) continue;
                    int64_t xx = x + dx, yy = y + dy;
                    if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                    int64_t r = yy * W + xx;
                    if (mask[r] && labels[r] < 0) {
                        labels[r] = lab;
                        stack[top++] = r;
                    }
                }
        }
    }
    free(stack);
    return 0;
}

typedef struct {
    int64_t n_holes, n_gap, n_center, n_boxes, n_roi_tiles, n_rowfill;
} orc_cls_stats;

/* Stage 3 and the interpolation half of Stage 4 (Sec. 3.1, Sec. 3.5).
 *   cls   in: hole mask (1 = hole); out: per-pixel class
 *         (0 warped, 1 hole left for an ROI, 2 gap, 4 row-filled).
 *   rgb/z/alpha in: warped image; out: gaps and row fills applied.
 *   labels out: component label (smallest linear index) of center-hole
 *         pixels, -1 elsewhere.
 *   boxes out: edge boxes (left, right, top, bottom that exist) followed
 *         by center boxes in increasing label order, 6 int32 each
 *         {x0, y0, x1, y1, kind, label}, half-open, tile aligned, up to
 *         box_cap of them; *n_boxes receives the full count.
 *   tile_mask out: 1 for tiles that intersect any box.
 * Gap rule: gap_passes Jacobi passes; a hole outside the edge ROIs with at
 * least one non-hole 8-neighbour takes the fp32 mean of those neighbours
 * (summed in the fixed order (-1,-1) (0,-1) (1,-1) (-1,0) (1,0) (-1,1)
 * (0,1) (1,1)) for RGB and alpha, and their largest depth.  With the
 * center step off, each remaining hole outside the edge ROIs copies the
 * nearest non-hole pixel on its row, taking the farther of the left and
 * right candidates (right wins only if strictly farther); with none it
 * becomes background. */
ORC_API int orc_classify(const orc_camera* src, const orc_camera* dst, const orc_roi* rp,
                         const float* depth_range, const float bg[3], float* rgb, float* z, float* alpha,
                         uint8_t* cls, int32_t* labels, int32_t* boxes, int32_t box_cap, int32_t* n_boxes,
                         uint8_t* tile_mask, orc_cls_stats* st) {
    int64_t W = dst->width, H = dst->height, n = W * H, T = rp->tile;
    int32_t eb[24];
    int32_t widths[4];
    int ne = orc_edge_rois(src, dst, rp, depth_range, widths, eb);
    memset(st, 0, sizeof *st);
    uint8_t* hole = (uint8_t*)malloc((size_t)n);
    uint8_t* nhole = (uint8_t*)malloc((size_t)n);
    float* nrgb = (float*)malloc(sizeof(float) * 3 * (size_t)n);
    float* nz = (float*)malloc(sizeof(float) * (size_t)n);
    float* na = (float*)malloc(sizeof(float) * (size_t)n);
    uint8_t* inE = (uint8_t*)malloc((size_t)n);
    if (!hole || !nhole || !nrgb || !nz || !na || !inE) return -1;
    for (int64_t p = 0; p < n; ++p) {
        hole[p] = cls[p] ? 1 : 0;
        cls[p] = hole[p] ? CLS_HOLE : CLS_WARPED;
        st->n_holes += hole[p];
        inE[p] = (uint8_t)in_boxes(eb, ne, p % W, p / W);
    }
    static const int NB[8][2] = {{-1, -1}, {0, -1}, {1, -1}, {-1, 0}, {1, 0}, {-1, 1}, {0, 1}, {1, 1}};
    for (int pass = 0; pass < rp->gap_passes; ++pass) {
        memcpy(nhole, hole, (size_t)n);
        memcpy(nrgb, rgb, sizeof(float) * 3 * (size_t)n);
        memcpy(nz, z, sizeof(float) * (size_t)n);
        memcpy(na, alpha, sizeof(float) * (size_t)n);
        for (int64_t p = 0; p < n; ++p) {
            if (!hole[p] || inE[p]) continue;
            int64_t x = p % W, y = p / W;
            int cnt = 0;
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, sa = 0.0f, zm = -INFINITY;
            for (int q = 0; q < 8; ++q) {
                int64_t xx = x + NB[q][0], yy = y + NB[q][1];
                if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                int64_t r = yy * W + xx;
                if (hole[r]) continue;
                s0 = s0 + rgb[r];
                s1 = s1 + rgb[n + r];
                s2 = s2 + rgb[2 * n + r];
                sa = sa + alpha[r];
                if (z[r] > zm) zm = z[r];
                ++cnt;
            }
            if (cnt == 0) continue;
            float fc = (float)cnt;
            nrgb[p] = s0 / fc;
            nrgb[n + p] = s1 / fc;
            nrgb[2 * n + p] = s2 / fc;
            na[p] = sa / fc;
            nz[p] = zm;
            nhole[p] = 0;
            cls[p] = CLS_GAP;
            st->n_gap += 1;
        }
        memcpy(hole, nhole, (size_t)n);
        memcpy(rgb, nrgb, sizeof(float) * 3 * (size_t)n);
        memcpy(z, nz, sizeof(float) * (size_t)n);
        memcpy(alpha, na, sizeof(float) * (size_t)n);
    }
    /* Holes left after interpolation and outside the edge ROIs. */
    uint8_t* center = nhole;
    for (int64_t p = 0; p < n; ++p) center[p] = (uint8_t)(hole[p] && !inE[p]);
    for (int64_t p = 0; p < n; ++p) labels[p] = -1;
    int64_t total_boxes = ne;
    for (int b = 0; b < ne && b < box_cap; ++b) memcpy(&boxes[6 * b], &eb[6 * b], 6 * sizeof(int32_t));
    int32_t* allbox = NULL;
    int64_t nall = ne;
    if (rp->center_roi) {
        orc_label_components(center, (int32_t)W, (int32_t)H, 8, labels);
        /* Bounding box per label, in increasing label order. */
        int64_t ncomp = 0;
        for (int64_t p = 0; p < n; ++p)
            if (center[p] && labels[p] == p) ++ncomp;
        st->n_center = 0;
        for (int64_t p = 0; p < n; ++p) st->n_center += center[p];
        allbox = (int32_t*)malloc(sizeof(int32_t) * 6 * (size_t)(ncomp + ne + 1));
        memcpy(allbox, eb, sizeof(int32_t) * 6 * (size_t)ne);
        int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t q = 0;
        for (int64_t p = 0; p < n; ++p) {
            if (center[p] && labels[p] == p) {
                slot[p] = q;
                int32_t* b = &allbox[6 * (ne + q)];
                b[0] = INT32_MAX;
                b[1] = INT32_MAX;
                b[2] = -1;
                b[3] = -1;
                b[4] = BOX_CENTER;
                b[5] = (int32_t)p;
                ++q;
            }
        }
        for (int64_t p = 0; p < n; ++p) {
            if (!center[p]) continue;
            int32_t* b = &allbox[6 * (ne + slot[labels[p]])];
            int32_t x = (int32_t)(p % W), y = (int32_t)(p / W);
            if (x < b[0]) b[0] = x;
            if (y < b[1]) b[1] = y;
            if (x + 1 > b[2]) b[2] = x + 1;
            if (y + 1 > b[3]) b[3] = y + 1;
        }
        for (int64_t c = 0; c < ncomp; ++c) {
            int32_t* b = &allbox[6 * (ne + c)];
            int64_t x0 = b[0] - rp->margin, y0 = b[1] - rp->margin;
            int64_t x1 = b[2] + rp->margin, y1 = b[3] + rp->margin;
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
            b[0] = (int32_t)x0;
            b[1] = (int32_t)y0;
            b[2] = (int32_t)x1;
            b[3] = (int32_t)y1;
        }
        free(slot);
        nall = ne + ncomp;
        total_boxes = nall;
        for (int64_t b = ne; b < nall && b < box_cap; ++b) memcpy(&boxes[6 * b], &allbox[6 * b], 6 * sizeof(int32_t));
    } else {
        /* Row fill of the remaining holes outside the edge ROIs. */
        allbox = (int32_t*)malloc(sizeof(int32_t) * 6 * (size_t)(ne + 1));
        memcpy(allbox, eb, sizeof(int32_t) * 6 * (size_t)ne);
        for (int64_t p = 0; p < n; ++p) {
            if (!center[p]) continue;
            int64_t x = p % W, y = p / W;
            int64_t xl = -1, xr = -1;
            for (int64_t xx = x - 1; xx >= 0; --xx)
                if (!hole[y * W + xx]) { xl = xx; break; }
            for (int64_t xx = x + 1; xx < W; ++xx)
                if (!hole[y * W + xx]) { xr = xx; break; }
            int64_t pick = -1;
            if (xl >= 0 && xr >= 0) pick = z[y * W + xr] > z[y * W + xl] ? xr : xl;
            else if (xl >= 0) pick = xl;
            else if (xr >= 0) pick = xr;
            if (pick >= 0) {
                int64_t r = y * W + pick;
                nrgb[p] = rgb[r];
                nrgb[n + p] = rgb[n + r];
                nrgb[2 * n + p] = rgb[2 * n + r];
                nz[p] = z[r];
                na[p] = alpha[r];
            } else {
                nrgb[p] = bg[0];
                nrgb[n + p] = bg[1];
                nrgb[2 * n + p] = bg[2];
                nz[p] = INFINITY;
                na[p] = 0.0f;
            }
            cls[p] = CLS_ROWFILL;
            st->n_rowfill += 1;
        }
        for (int64_t p = 0; p < n; ++p) {
            if (!center[p]) continue;
            rgb[p] = nrgb[p];
            rgb[n + p] = nrgb[n + p];
            rgb[2 * n + p] = nrgb[2 * n + p];
            z[p] = nz[p];
            alpha[p] = na[p];
        }
    }
    *n_boxes = (int32_t)total_boxes;
    st->n_boxes = total_boxes;
    int64_t tw = (W + T - 1) / T, th = (H + T - 1) / T;
    st->n_roi_tiles = 0;
    for (int64_t ty = 0; ty < th; ++ty)
        for (int64_t tx = 0; tx < tw; ++tx) {
            int64_t x0 = tx * T, y0 = ty * T, x1 = x0 + T, y1 = y0 + T;
            int hit = 0;
            for (int64_t b = 0; b < nall && !hit; ++b) {
                const int32_t* bb = &allbox[6 * b];
                if (x0 < bb[2] && bb[0] < x1 && y0 < bb[3] && bb[1] < y1) hit = 1;
            }
            tile_mask[ty * tw + tx] = (uint8_t)hit;
            st->n_roi_tiles += hit;
        }
    free(allbox);
    free(hole);
    free(nhole);
    free(nrgb);
    free(nz);
    free(na);
    free(inE);
    return 0;
}

/* ROI re-rasterisation (Stage 4): every pixel of every masked tile is
 * rendered at the destination camera with the same per-pixel definition as
 * the full render; RGB, alpha and the depth proxy D/A (infinite when
 * A < a_min) overwrite the warped values and the class becomes ROI. */
ORC_API int orc_patch(const oscene* sc, const orc_camera* cam, const orc_raster* rp, double a_min,
                      int32_t tile, const uint8_t* tile_mask, int32_t nthreads, float* rgb, float* z,
                      float* alpha, uint8_t* cls, uint8_t* amb) {
    int64_t W = cam->width, H = cam->height, n = W * H;
    int64_t tw = (W + tile - 1) / tile;
    int64_t cnt = 0;
    for (int64_t p = 0; p < n; ++p)
        if (tile_mask[((p / W) / tile) * tw + (p % W) / tile]) ++cnt;
    int32_t* pix = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(cnt > 0 ? cnt : 1));
    int64_t* where = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
    double* o = (double*)malloc(sizeof(double) * 5 * (size_t)(cnt > 0 ? cnt : 1));
    uint8_t* f = (uint8_t*)malloc((size_t)(cnt > 0 ? cnt : 1));
    if (!pix || !where || !o || !f) return -1;
    int64_t q = 0;
    for (int64_t p = 0; p < n; ++p)
        if (tile_mask[((p / W) / tile) * tw + (p % W) / tile]) {
            pix[2 * q] = (int32_t)(p % W);
            pix[2 * q + 1] = (int32_t)(p / W);
            where[q] = p;
            ++q;
        }
    int rc = 0;
    if (cnt > 0) rc = orc_render(sc, cam, rp, pix, cnt, 1, nthreads, o, o + 3 * cnt, o + 4 * cnt, f);
    for (int64_t k = 0; k < cnt && rc == 0; ++k) {
        int64_t p = where[k];
        rgb[p] = (float)o[k];
        rgb[n + p] = (float)o[cnt + k];
        rgb[2 * n + p] = (float)o[2 * cnt + k];
        double A = o[4 * cnt + k], D = o[3 * cnt + k];
        alpha[p] = (float)A;
        z[p] = A >= a_min ? (float)(D / A) : INFINITY;
        cls[p] = CLS_ROI;
        if (amb) amb[p] = f[k];
    }
    free(pix);
    free(where);
    free(o);
    free(f);
    return rc;
}
