/*
 * oracle.c -- plain, slow CPU reference for time-resolved (transient) Monte
 * Carlo path tracing into a pixel x time film.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation: every routine below is written independently from
 * the paper (arXiv 2510.25660, "mitransient") and from the published methods
 * it names.
 *
 * What it computes (paper, Sec. 3 "Transient rendering"):
 *   - light paths x0 -> ... -> xk (Eq. 1) sampled by path tracing with
 *     next-event estimation; the Monte Carlo estimator of Eq. 9;
 *   - the time of flight of a path is the sum of its segment lengths
 *     (Eqs. 3-4) with eta = 1 and c = 1, i.e. optical path length in metres;
 *   - emitters pulse at t = 0 (Eq. 5), the sensor window is a box (Eq. 6);
 *   - path reuse and histogramming: each contribution lands in bin
 *     floor((tof - b_start) / b_width) (Sec. 3, "Path reuse and
 *     histogramming"); the steady image receives every contribution;
 *   - camera unwarping drops the camera segment (Sec. 3, "Camera warp");
 *   - homogeneous participating media with analog free-flight sampling
 *     (Sec. 4.1, "Volumetric scattering");
 *   - backward-mode derivatives of L = sum (I - I*)^2 w.r.t. per-triangle
 *     albedo and roughness (Sec. 4.4, Eqs. 15-17), as a per-path adjoint
 *     with detached sampling.
 *
 * Precision: the path geometry is FP32 following the numerics contract
 * (fixed operation order, explicit fmaf, correctly rounded / and sqrt), so
 * that a bin decision here and on the GPU is taken on identical bits; every
 * accumulation (film, steady, gradients) is FP64 in a fixed order.
 * Gradient factors d(log f)/d(theta) are evaluated in FP64 from the FP32
 * path geometry.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------------------ */
/* FP32 vector helpers (operation order is part of the numerics contract).  */
/* ------------------------------------------------------------------------ */
typedef struct { float x, y, z; } v3;

static v3 mk(float x, float y, float z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vscale(v3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
static v3 vneg(v3 a) { return mk(-a.x, -a.y, -a.z); }
/* dot(a,b) = fma(ax,bx, fma(ay,by, az*bz)) */
static float vdot(v3 a, v3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
static v3 vcross(v3 a, v3 b)
{
    return mk(fmaf(a.y, b.z, -(a.z * b.y)),
              fmaf(a.z, b.x, -(a.x * b.z)),
              fmaf(a.x, b.y, -(a.y * b.x)));
}
static v3 vnormalize(v3 a)
{
    float inv = 1.0f / sqrtf(vdot(a, a));
    return vscale(a, inv);
}
/* point along a ray: per component fma(t, d, o) */
static v3 vray(v3 o, v3 d, float t) { return mk(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z)); }
static v3 vload(const float* p) { return mk(p[0], p[1], p[2]); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).*/
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t prod_a, prod_b;
        uint32_t y0, y1, y2, y3;
        if (round > 0) {
            k0 += 0x9E3779B9u; /* golden-ratio Weyl increment */
            k1 += 0xBB67AE85u; /* sqrt(3)-1 Weyl increment */
        }
        prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        y1 = (uint32_t)prod_b;
        y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        y3 = (uint32_t)prod_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 24-bit uniform in [0, 1 - 2^-24], exact. */
float orc_uniform(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

static void draw(const orc_render* R, uint32_t pix, uint32_t sample, uint32_t block, float u[4])
{
    uint32_t ctr[4], key[2], o[4];
    ctr[0] = pix; ctr[1] = sample; ctr[2] = block; ctr[3] = R->stream_id;
    key[0] = (uint32_t)(R->seed & 0xffffffffu);
    key[1] = (uint32_t)(R->seed >> 32);
    orc_philox4x32_10(ctr, key, o);
    u[0] = orc_uniform(o[0]); u[1] = orc_uniform(o[1]);
    u[2] = orc_uniform(o[2]); u[3] = orc_uniform(o[3]);
}

/* ------------------------------------------------------------------------ */
/* sin/cos of 2*pi*u and ln(1-u) without library transcendentals.           */
/* ------------------------------------------------------------------------ */
/* Octant reduction is exact because u*8 and its fractional part are exact
 * for u = k * 2^-24; the octant angle lies in [0, pi/4] where the Taylor
 * series truncated after the 11th (sine) / 12th (cosine) power is accurate
 * far below FP32 rounding. */
void orc_sincos2pi(float u, float* s_out, float* c_out)
{
    const float quarter_pi = (float)(3.14159265358979323846 / 4.0);
    const float s3 = (float)(-1.0 / 6.0), s5 = (float)(1.0 / 120.0), s7 = (float)(-1.0 / 5040.0);
    const float s9 = (float)(1.0 / 362880.0), s11 = (float)(-1.0 / 39916800.0);
    const float c2 = -0.5f, c4 = (float)(1.0 / 24.0), c6 = (float)(-1.0 / 720.0);
    const float c8 = (float)(1.0 / 40320.0), c10 = (float)(-1.0 / 3628800.0), c12 = (float)(1.0 / 479001600.0);
    float x = u * 8.0f;
    int octant = (int)x;
    float frac = x - (float)octant;
    int quadrant = octant >> 1, odd = octant & 1;
    float a = odd ? (1.0f - frac) : frac;
    float th = a * quarter_pi;
    float z = th * th;
    float ps, pc, sn, cs, s0, k0;
    ps = fmaf(z, s11, s9);
    ps = fmaf(z, ps, s7);
    ps = fmaf(z, ps, s5);
    ps = fmaf(z, ps, s3);
    sn = fmaf(th * z, ps, th);
    pc = fmaf(z, c12, c10);
    pc = fmaf(z, pc, c8);
    pc = fmaf(z, pc, c6);
    pc = fmaf(z, pc, c4);
    pc = fmaf(z, pc, c2);
    cs = fmaf(z, pc, 1.0f);
    /* odd octants: angle = (q+1)*pi/2 - th, so sine and cosine swap */
    s0 = odd ? cs : sn;
    k0 = odd ? sn : cs;
    switch (quadrant) {
    case 0: *s_out = s0;  *c_out = k0;  break;
    case 1: *s_out = k0;  *c_out = -s0; break;
    case 2: *s_out = -s0; *c_out = -k0; break;
    default: *s_out = -k0; *c_out = s0; break;
    }
}

/* ln(1-u): exponent/mantissa split, mantissa folded into [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh((m-1)/(m+1)) by its odd series, e*ln2 in two pieces. */
float orc_log1m(float u)
{
    const float sqrt2 = (float)1.41421356237309504880;
    const float l3 = (float)(1.0 / 3.0), l5 = (float)(1.0 / 5.0), l7 = (float)(1.0 / 7.0);
    const float l9 = (float)(1.0 / 9.0), l11 = (float)(1.0 / 11.0), l13 = (float)(1.0 / 13.0);
    const float ln2_hi = 0.693145751953125f;
    const float ln2_lo = (float)(0.693147180559945309417232 - 0.693145751953125);
    float y = 1.0f - u;
    uint32_t bits, mbits;
    int e;
    float m, s, z, p, r, ef;
    memcpy(&bits, &y, 4);
    e = (int)((bits >> 23) & 0xffu) - 127;
    mbits = (bits & 0x007fffffu) | 0x3f800000u;
    memcpy(&m, &mbits, 4);
    if (m > sqrt2) {
        m = m * 0.5f;
        e = e + 1;
    }
    s = (m - 1.0f) / (m + 1.0f);
    z = s * s;
    p = fmaf(z, l13, l11);
    p = fmaf(z, p, l9);
    p = fmaf(z, p, l7);
    p = fmaf(z, p, l5);
    p = fmaf(z, p, l3);
    r = fmaf(s * z, p, s);
    r = r + r;
    ef = (float)e;
    return fmaf(ef, ln2_hi, fmaf(ef, ln2_lo, r));
}

/* ------------------------------------------------------------------------ */
/* Frames and self-intersection avoidance.                                  */
/* ------------------------------------------------------------------------ */
/* Orthonormal basis from a unit normal (Duff et al., JCGT 2017). */
static void onb(v3 n, v3* t, v3* b)
{
    float sgn = copysignf(1.0f, n.z);
    float a = -1.0f / (sgn + n.z);
    float bb = n.x * n.y * a;
    *t = mk(1.0f + sgn * n.x * n.x * a, sgn * bb, -sgn * n.x);
    *b = mk(bb, sgn + n.y * n.y * a, -n.y);
}
static v3 to_world(v3 t, v3 b, v3 n, v3 l)
{
    return mk(fmaf(n.x, l.z, fmaf(b.x, l.y, t.x * l.x)),
              fmaf(n.y, l.z, fmaf(b.y, l.y, t.y * l.x)),
              fmaf(n.z, l.z, fmaf(b.z, l.y, t.z * l.x)));
}

/* Ray origin offset along the normal in integer ulps (Waechter & Binder,
 * "A Fast and Robust Method for Avoiding Self-Intersection", Ray Tracing
 * Gems, 2019); n points to the side the new ray leaves toward. */
static float off1(float p, float n)
{
    const float origin = 1.0f / 32.0f, float_scale = 1.0f / 65536.0f, int_scale = 256.0f;
    int32_t of = (int32_t)(int_scale * n);
    int32_t pi;
    float moved;
    if (fabsf(p) < origin) return p + float_scale * n;
    memcpy(&pi, &p, 4);
    pi = pi + ((p < 0.0f) ? -of : of);
    memcpy(&moved, &pi, 4);
    return moved;
}
static v3 offset_ray(v3 p, v3 n) { return mk(off1(p.x, n.x), off1(p.y, n.y), off1(p.z, n.z)); }

/* ------------------------------------------------------------------------ */
/* Scene preparation: per-triangle inflated boxes, a median-split BVH.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    float lo[3], hi[3];
    int left, right;  /* children; -1 for a leaf */
    int first, count; /* leaf triangle range into order[] */
} onode;

struct orc_prepared {
    orc_scene sc;       /* shallow copy; arrays below are owned copies */
    float* tri;         /* [nt][9] */
    float* box;         /* [nt][6] inflated lo xyz, hi xyz */
    uint8_t* mat;
    float* albedo;
    float* rough;
    float* scan;        /* [n_scan][3] (confocal) */
    float* ior;         /* [nt] or NULL */
    float* delay;       /* [nt] or NULL */
    float pad;
    /* BVH (used when nt > ORC_BRUTE_MAX) */
    onode* nodes;
    int n_nodes;
    int* order;
    /* NLOS area sampling (confocal): inclusive prefix sums of the sampling
     * weights (triangle areas, zero on the relay wall's plane) */
    double* area_cdf;   /* [region][nt] inclusive prefix sums of the weights */
    float* area_invp;   /* [region][nt] W_r A_k / w_k: the inverse area density */
    double* weight_total; /* [region] W_r */
    int* pix_region;    /* [scan point] its region */
    double area_total;  /* area of the sampling set */
};

#define ORC_BRUTE_MAX 64
#define ORC_AREA_G 4 /* NLOS area sampling: scan-point regions per axis */

static float f3min(float a, float b, float c) { return fminf(fminf(a, b), c); }
static float f3max(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

typedef struct { int* idx; const float* cen; int axis; } sort_ctx;
static int cmp_axis_x(const void* a, const void* b, const float* cen, int axis)
{
    int ia = *(const int*)a, ib = *(const int*)b;
    float ca = cen[3 * ia + axis], cb = cen[3 * ib + axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}
static const float* g_sort_cen;
static int g_sort_axis;
static int cmp_axis(const void* a, const void* b) { return cmp_axis_x(a, b, g_sort_cen, g_sort_axis); }

static int build_rec(struct orc_prepared* P, const float* cen, int first, int count)
{
    int id = P->n_nodes++;
    onode* nd = &P->nodes[id];
    int i, axis;
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    nd->lo[0] = nd->lo[1] = nd->lo[2] = INFINITY;
    nd->hi[0] = nd->hi[1] = nd->hi[2] = -INFINITY;
    for (i = first; i < first + count; ++i) {
        int k = P->order[i], a;
        for (a = 0; a < 3; ++a) {
            nd->lo[a] = fminf(nd->lo[a], P->box[6 * k + a]);
            nd->hi[a] = fmaxf(nd->hi[a], P->box[6 * k + 3 + a]);
            clo[a] = fminf(clo[a], cen[3 * k + a]);
            chi[a] = fmaxf(chi[a], cen[3 * k + a]);
        }
    }
    if (count <= 4) {
        nd->left = nd->right = -1;
        nd->first = first;
        nd->count = count;
        return id;
    }
    axis = 0;
    if (chi[1] - clo[1] > chi[axis] - clo[axis]) axis = 1;
    if (chi[2] - clo[2] > chi[axis] - clo[axis]) axis = 2;
    g_sort_cen = cen;
    g_sort_axis = axis;
    qsort(P->order + first, (size_t)count, sizeof(int), cmp_axis);
    {
        int half = count / 2;
        int l = build_rec(P, cen, first, half);
        int r = build_rec(P, cen, first + half, count - half);
        nd = &P->nodes[id];
        nd->left = l;
        nd->right = r;
        nd->first = 0;
        nd->count = 0;
    }
    return id;
}

orc_prepared* orc_prepare(const orc_scene* sc)
{
    struct orc_prepared* P;
    int k, nt = sc->n_tris;
    float maxabs = 0.0f;
    if (nt <= 0 || !sc->tri) return NULL;
    for (k = 0; k < nt; ++k)
        if (sc->mat[k] == ORC_MAT_DIELECTRIC && (!sc->ior || !(sc->ior[k] > 0.0f))) return NULL;
    P = (struct orc_prepared*)calloc(1, sizeof(*P));
    P->sc = *sc;
    P->tri = (float*)malloc(sizeof(float) * 9 * (size_t)nt);
    P->box = (float*)malloc(sizeof(float) * 6 * (size_t)nt);
    P->mat = (uint8_t*)malloc((size_t)nt);
    P->albedo = (float*)malloc(sizeof(float) * (size_t)nt);
    P->rough = (float*)malloc(sizeof(float) * (size_t)nt);
    memcpy(P->tri, sc->tri, sizeof(float) * 9 * (size_t)nt);
    memcpy(P->mat, sc->mat, (size_t)nt);
    memcpy(P->albedo, sc->albedo, sizeof(float) * (size_t)nt);
    memcpy(P->rough, sc->roughness, sizeof(float) * (size_t)nt);
    if (sc->sensor == ORC_SENSOR_CONFOCAL) {
        size_t ns = (size_t)sc->width * (size_t)sc->height;
        P->scan = (float*)malloc(sizeof(float) * 3 * ns);
        memcpy(P->scan, sc->scan_points, sizeof(float) * 3 * ns);
    }
    if (sc->ior) {
        P->ior = (float*)malloc(sizeof(float) * (size_t)nt);
        memcpy(P->ior, sc->ior, sizeof(float) * (size_t)nt);
    }
    if (sc->delay) {
        P->delay = (float*)malloc(sizeof(float) * (size_t)nt);
        memcpy(P->delay, sc->delay, sizeof(float) * (size_t)nt);
    }
    P->sc.tri = P->tri; P->sc.mat = P->mat; P->sc.albedo = P->albedo;
    P->sc.roughness = P->rough; P->sc.scan_points = P->scan;
    P->sc.ior = P->ior; P->sc.delay = P->delay;
    /* box padding: (largest |coordinate|) * 2^-16, an exact scaling */
    for (k = 0; k < 9 * nt; ++k) maxabs = fmaxf(maxabs, fabsf(P->tri[k]));
    P->pad = maxabs * 0x1p-16f;
    for (k = 0; k < nt; ++k) {
        const float* t = P->tri + 9 * k;
        int a;
        for (a = 0; a < 3; ++a) {
            P->box[6 * k + a] = f3min(t[a], t[3 + a], t[6 + a]) - P->pad;
            P->box[6 * k + 3 + a] = f3max(t[a], t[3 + a], t[6 + a]) + P->pad;
        }
    }
    if (nt > ORC_BRUTE_MAX) {
        float* cen = (float*)malloc(sizeof(float) * 3 * (size_t)nt);
        for (k = 0; k < nt; ++k) {
            int a;
            for (a = 0; a < 3; ++a)
                cen[3 * k + a] = 0.5f * (P->box[6 * k + a] + P->box[6 * k + 3 + a]);
        }
        P->order = (int*)malloc(sizeof(int) * (size_t)nt);
        for (k = 0; k < nt; ++k) P->order[k] = k;
        P->nodes = (onode*)malloc(sizeof(onode) * 2 * (size_t)nt);
        P->n_nodes = 0;
        build_rec(P, cen, 0, nt);
        free(cen);
    }
    if (sc->sensor == ORC_SENSOR_CONFOCAL) {
        /* NLOS area sampling.  Sampling set: every triangle not lying in the
         * relay wall's plane (through the first scan point, along the wall
         * normal): seen from a scan point those subtend no solid angle.
         * The scan points are split into ORC_AREA_G x ORC_AREA_G regions of
         * their bounding box, over the two axes of largest extent (the
         * larger first, ties to the lower axis); region r has its own
         * triangle pdf: triangle k of the set with probability w_k / W_r,
         * w_k = A_k (g_k + g_max / 20), A_k its area, g_k = (cos_s cos_h / r^2)^2
         * the square of the geometry term between the region's
         * representative c (the mean of its scan points; the mean of all of
         * them for an empty region) and the triangle's centroid m_k (d = m_k
         * - c, r = |d|, cos_s = the wall normal's cosine with d, clamped at
         * 0, cos_h = |n_k . d| / r), g_max the region's largest g_k; the floor
         * keeps every triangle of the set drawable (uniform by area if every
         * g_k is 0).  The point is uniform within the triangle, so its area
         * density is w_k / (W_r A_k); area_invp holds W_r A_k / w_k.  All in
         * FP64 (float differences are exact there). */
        const size_t ns = (size_t)sc->width * (size_t)sc->height;
        const int nreg = ORC_AREA_G * ORC_AREA_G;
        double area_sum = 0.0, tol, n[3], s0[3], lo[3], hi[3], ext[3], all[3] = {0.0, 0.0, 0.0};
        double (*repr)[3] = (double(*)[3])calloc((size_t)nreg, sizeof(double[3]));
        double* cnt = (double*)calloc((size_t)nreg, sizeof(double));
        double* area = (double*)malloc(sizeof(double) * (size_t)nt);
        double* nrm = (double*)malloc(sizeof(double) * 3 * (size_t)nt);
        double* cen3 = (double*)malloc(sizeof(double) * 3 * (size_t)nt);
        double* geo = (double*)malloc(sizeof(double) * (size_t)nt);
        size_t i;
        int a, ax0, ax1, r;
        for (a = 0; a < 3; ++a) {
            n[a] = (double)sc->wall_normal[a];
            s0[a] = (double)P->scan[a];
            lo[a] = hi[a] = (double)P->scan[a];
        }
        for (i = 0; i < ns; ++i)
            for (a = 0; a < 3; ++a) {
                const double v = (double)P->scan[3 * i + a];
                all[a] += v;
                if (v < lo[a]) lo[a] = v;
                if (v > hi[a]) hi[a] = v;
            }
        for (a = 0; a < 3; ++a) {
            all[a] = all[a] / (double)ns;
            ext[a] = hi[a] - lo[a];
        }
        /* the two axes of largest extent */
        ax0 = 0;
        for (a = 1; a < 3; ++a)
            if (ext[a] > ext[ax0]) ax0 = a;
        ax1 = (ax0 == 0) ? 1 : 0;
        for (a = 0; a < 3; ++a)
            if (a != ax0 && ext[a] > ext[ax1]) ax1 = a;
        P->pix_region = (int*)malloc(sizeof(int) * ns);
        for (i = 0; i < ns; ++i) {
            int cell[2], q;
            const int axes[2] = {ax0, ax1};
            for (q = 0; q < 2; ++q) {
                const int b = axes[q];
                const double f = ext[b] > 0.0 ? ((double)P->scan[3 * i + b] - lo[b]) / ext[b] : 0.0;
                int c = (int)floor(f * (double)ORC_AREA_G);
                if (c < 0) c = 0;
                if (c > ORC_AREA_G - 1) c = ORC_AREA_G - 1;
                cell[q] = c;
            }
            r = cell[0] * ORC_AREA_G + cell[1];
            P->pix_region[i] = r;
            cnt[r] += 1.0;
            for (a = 0; a < 3; ++a) repr[r][a] += (double)P->scan[3 * i + a];
        }
        for (r = 0; r < nreg; ++r)
            for (a = 0; a < 3; ++a) repr[r][a] = cnt[r] > 0.0 ? repr[r][a] / cnt[r] : all[a];
        tol = 1e-6 * (1.0 + (double)maxabs);
        for (k = 0; k < nt; ++k) {
            const float* t = P->tri + 9 * k;
            double e1[3], e2[3], c[3], len;
            int on_wall = 1, j;
            for (j = 0; j < 3; ++j) {
                double h = ((double)t[3 * j] - s0[0]) * n[0] + ((double)t[3 * j + 1] - s0[1]) * n[1] +
                           ((double)t[3 * j + 2] - s0[2]) * n[2];
                if (fabs(h) > tol) on_wall = 0;
            }
            area[k] = 0.0;
            if (on_wall) continue;
            for (a = 0; a < 3; ++a) {
                e1[a] = (double)t[3 + a] - (double)t[a];
                e2[a] = (double)t[6 + a] - (double)t[a];
                cen3[3 * k + a] = (((double)t[a] + (double)t[3 + a]) + (double)t[6 + a]) / 3.0;
            }
            c[0] = e1[1] * e2[2] - e1[2] * e2[1];
            c[1] = e1[2] * e2[0] - e1[0] * e2[2];
            c[2] = e1[0] * e2[1] - e1[1] * e2[0];
            len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            area[k] = 0.5 * len;
            for (a = 0; a < 3; ++a) nrm[3 * k + a] = c[a] / len;
            area_sum += area[k];
        }
        P->area_cdf = (double*)malloc(sizeof(double) * (size_t)nt * (size_t)nreg);
        P->area_invp = (float*)malloc(sizeof(float) * (size_t)nt * (size_t)nreg);
        P->weight_total = (double*)malloc(sizeof(double) * (size_t)nreg);
        for (r = 0; r < nreg; ++r) {
            double gmax = 0.0, floor_w, acc = 0.0;
            for (k = 0; k < nt; ++k) {
                double dd[3], r2;
                geo[k] = 0.0;
                if (!(area[k] > 0.0)) continue;
                for (a = 0; a < 3; ++a) dd[a] = cen3[3 * k + a] - repr[r][a];
                r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
                if (r2 > 0.0) {
                    const double rr = sqrt(r2);
                    double cos_s = (n[0] * dd[0] + n[1] * dd[1] + n[2] * dd[2]) / rr, cos_h, q;
                    if (cos_s < 0.0) cos_s = 0.0;
                    cos_h = fabs(nrm[3 * k] * dd[0] + nrm[3 * k + 1] * dd[1] + nrm[3 * k + 2] * dd[2]) / rr;
                    q = (cos_s * cos_h) / r2;
                    geo[k] = q * q;
                }
                if (geo[k] > gmax) gmax = geo[k];
            }
            floor_w = (gmax > 0.0) ? gmax / 20.0 : 1.0;
            for (k = 0; k < nt; ++k) {
                acc += area[k] * (geo[k] + floor_w);
                P->area_cdf[(size_t)r * nt + k] = acc;
            }
            for (k = 0; k < nt; ++k) {
                const double w = area[k] * (geo[k] + floor_w);
                P->area_invp[(size_t)r * nt + k] = (w > 0.0) ? (float)((acc * area[k]) / w) : 0.0f;
            }
            P->weight_total[r] = acc;
        }
        P->area_total = area_sum;
        free(repr); free(cnt); free(area); free(nrm); free(cen3); free(geo);
    }
    return P;
}

void orc_release(orc_prepared* P)
{
    if (!P) return;
    free(P->tri); free(P->box); free(P->mat); free(P->albedo); free(P->rough);
    free(P->scan); free(P->nodes); free(P->order); free(P->area_cdf); free(P->area_invp); free(P->ior); free(P->delay);
    free(P->weight_total); free(P->pix_region);
    free(P);
}

float orc_pad(const orc_prepared* P) { return P->pad; }
double orc_area_total(const orc_prepared* P) { return P->area_total; }

/* ------------------------------------------------------------------------ */
/* Ray - box (slab) and ray - triangle (Moller-Trumbore) tests.             */
/* ------------------------------------------------------------------------ */
typedef struct { v3 o, d, inv, oi; } ray_t;

static ray_t make_ray(v3 o, v3 d)
{
    ray_t r;
    float dx = (fabsf(d.x) < 1e-30f) ? copysignf(1e-30f, d.x) : d.x;
    float dy = (fabsf(d.y) < 1e-30f) ? copysignf(1e-30f, d.y) : d.y;
    float dz = (fabsf(d.z) < 1e-30f) ? copysignf(1e-30f, d.z) : d.z;
    r.o = o;
    r.d = d;
    r.inv = mk(1.0f / dx, 1.0f / dy, 1.0f / dz);
    r.oi = mk(o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z);
    return r;
}

/* slab interval [tn, tf] of a box; slab planes at fma(bound, inv, -o*inv) */
static void slab(const ray_t* r, const float* lo, const float* hi, float* tn, float* tf)
{
    float ax = fmaf(lo[0], r->inv.x, -r->oi.x), bx = fmaf(hi[0], r->inv.x, -r->oi.x);
    float ay = fmaf(lo[1], r->inv.y, -r->oi.y), by = fmaf(hi[1], r->inv.y, -r->oi.y);
    float az = fmaf(lo[2], r->inv.z, -r->oi.z), bz = fmaf(hi[2], r->inv.z, -r->oi.z);
    *tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
    *tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
}

/* Moller & Trumbore (JGT 1997), two-sided; returns 1 and t on a hit with t>0. */
static int moller_trumbore(const ray_t* r, const float* tri, float* t_out)
{
    v3 v0 = vload(tri), v1 = vload(tri + 3), v2 = vload(tri + 6);
    v3 e1 = vsub(v1, v0), e2 = vsub(v2, v0);
    v3 p = vcross(r->d, e2);
    float det = vdot(e1, p), inv, u, v, t;
    v3 s, q;
    if (det == 0.0f) return 0;
    inv = 1.0f / det;
    s = vsub(r->o, v0);
    u = vdot(s, p) * inv;
    if (u < 0.0f || u > 1.0f) return 0;
    q = vcross(s, e1);
    v = vdot(r->d, q) * inv;
    if (v < 0.0f || u + v > 1.0f) return 0;
    t = vdot(e2, q) * inv;
    if (!(t > 0.0f)) return 0;
    *t_out = t;
    return 1;
}

/* A triangle is hit at t iff Moller-Trumbore accepts it AND t lies at or
 * beyond the entry of the triangle's own inflated box (whose slab interval
 * is non-empty and reaches t >= 0).  The second clause makes the closest hit
 * a function of the triangle set alone: any box that contains the
 * triangle's box passes the pruning test whenever the triangle is hit. */
static int tri_hit(const struct orc_prepared* P, const ray_t* r, int k, float* t_out)
{
    float tn, tf, t;
    slab(r, P->box + 6 * k, P->box + 6 * k + 3, &tn, &tf);
    if (!(tn <= tf && tf >= 0.0f)) return 0;
    if (!moller_trumbore(r, P->tri + 9 * k, &t)) return 0;
    if (tn > t) return 0;
    *t_out = t;
    return 1;
}

/* closest: smallest t, ties to the smallest triangle index */
static int closest_brute(const struct orc_prepared* P, const ray_t* r, int exclude, float* t_best, int* k_best)
{
    int k, found = 0;
    float best = INFINITY;
    int bk = -1;
    for (k = 0; k < P->sc.n_tris; ++k) {
        float t;
        if (k == exclude) continue;
        if (!tri_hit(P, r, k, &t)) continue;
        if (t < best || (t == best && k < bk)) {
            best = t;
            bk = k;
            found = 1;
        }
    }
    *t_best = best;
    *k_best = bk;
    return found;
}

static int closest_bvh(const struct orc_prepared* P, const ray_t* r, int exclude, float* t_best, int* k_best)
{
    int stack[256], sp = 0, found = 0, bk = -1;
    float best = INFINITY;
    stack[sp++] = 0;
    while (sp > 0) {
        const onode* nd = &P->nodes[stack[--sp]];
        float tn, tf;
        slab(r, nd->lo, nd->hi, &tn, &tf);
        if (!(tn <= tf && tf >= 0.0f && tn <= best)) continue;
        if (nd->left < 0) {
            int i;
            for (i = nd->first; i < nd->first + nd->count; ++i) {
                int k = P->order[i];
                float t;
                if (k == exclude) continue;
                if (!tri_hit(P, r, k, &t)) continue;
                if (t < best || (t == best && k < bk)) {
                    best = t;
                    bk = k;
                    found = 1;
                }
            }
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    *t_best = best;
    *k_best = bk;
    return found;
}

static int closest(const struct orc_prepared* P, const ray_t* r, int exclude, float* t, int* k)
{
    if (P->nodes) return closest_bvh(P, r, exclude, t, k);
    return closest_brute(P, r, exclude, t, k);
}

/* occluded: some triangle other than `exclude` is hit at t < tmax */
static int occluded(const struct orc_prepared* P, const ray_t* r, int exclude, float tmax)
{
    if (P->nodes) {
        int stack[256], sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const onode* nd = &P->nodes[stack[--sp]];
            float tn, tf;
            slab(r, nd->lo, nd->hi, &tn, &tf);
            if (!(tn <= tf && tf >= 0.0f && tn <= tmax)) continue;
            if (nd->left < 0) {
                int i;
                for (i = nd->first; i < nd->first + nd->count; ++i) {
                    int k = P->order[i];
                    float t;
                    if (k == exclude) continue;
                    if (tri_hit(P, r, k, &t) && t < tmax) return 1;
                }
            } else {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
            }
        }
        return 0;
    } else {
        int k;
        for (k = 0; k < P->sc.n_tris; ++k) {
            float t;
            if (k == exclude) continue;
            if (tri_hit(P, r, k, &t) && t < tmax) return 1;
        }
        return 0;
    }
}

int orc_closest_hit(const orc_prepared* P, const float o[3], const float d[3], int exclude, int use_bvh,
                    float* t, int* prim)
{
    ray_t r = make_ray(vload(o), vload(d));
    if (use_bvh && P->nodes) return closest_bvh(P, &r, exclude, t, prim);
    return closest_brute(P, &r, exclude, t, prim);
}

/* ------------------------------------------------------------------------ */
/* BSDFs: Lambertian and a GGX conductor with constant reflectance F.       */
/* ------------------------------------------------------------------------ */
#define ORC_PI_F ((float)3.14159265358979323846)
#define ORC_INV_PI_F ((float)(1.0 / 3.14159265358979323846))
#define ORC_INV_4PI_F ((float)(1.0 / (4.0 * 3.14159265358979323846)))

/* Smith Lambda for GGX: (sqrt(1 + a^2 tan^2) - 1) / 2 */
static float ggx_lambda(v3 w, float a2)
{
    float tan2 = fmaf(w.x, w.x, w.y * w.y) / (w.z * w.z);
    return (sqrtf(fmaf(a2, tan2, 1.0f)) - 1.0f) * 0.5f;
}

/* GGX normal distribution D(h) = a^2 / (pi (cos^2 (a^2 - 1) + 1)^2) */
static float ggx_d(float hz, float a2)
{
    float c2 = hz * hz;
    float dd = fmaf(c2, a2 - 1.0f, 1.0f);
    return a2 / ((ORC_PI_F * dd) * dd);
}

/* f(wo, wi) for the GGX conductor in the local frame (z = normal),
 * height-correlated Smith masking-shadowing, F = albedo. */
static float ggx_f(v3 wo, v3 wi, float alpha, float F)
{
    float a2, lo, li, g2, d;
    v3 h;
    if (!(wo.z > 0.0f) || !(wi.z > 0.0f)) return 0.0f;
    h = vnormalize(mk(wo.x + wi.x, wo.y + wi.y, wo.z + wi.z));
    a2 = alpha * alpha;
    d = ggx_d(h.z, a2);
    lo = ggx_lambda(wo, a2);
    li = ggx_lambda(wi, a2);
    g2 = 1.0f / ((1.0f + lo) + li);
    return ((F * d) * g2) / ((4.0f * wo.z) * wi.z);
}

/* visible-normal pdf of wi: G1(wo) D(h) / (4 cos_o) */
static float ggx_pdf(v3 wo, v3 wi, float alpha)
{
    float a2 = alpha * alpha;
    v3 h = vnormalize(mk(wo.x + wi.x, wo.y + wi.y, wo.z + wi.z));
    float g1 = 1.0f / (1.0f + ggx_lambda(wo, a2));
    return (g1 * ggx_d(h.z, a2)) / (4.0f * wo.z);
}

/* Visible-normal sampling (Heitz, "Sampling the GGX Distribution of Visible
 * Normals", JCGT 2018).  Returns wi in the local frame. */
static v3 ggx_sample_vndf(v3 wo, float alpha, float u0, float u1)
{
    v3 vh = vnormalize(mk(alpha * wo.x, alpha * wo.y, wo.z));
    float lensq = fmaf(vh.x, vh.x, vh.y * vh.y);
    v3 t1, t2, nh, ne;
    float r, sn, cs, p1, p2, s, rest, k;
    if (lensq > 0.0f) {
        float inv = 1.0f / sqrtf(lensq);
        t1 = mk(-vh.y * inv, vh.x * inv, 0.0f);
    } else {
        t1 = mk(1.0f, 0.0f, 0.0f);
    }
    t2 = vcross(vh, t1);
    r = sqrtf(u0);
    orc_sincos2pi(u1, &sn, &cs);
    p1 = r * cs;
    p2 = r * sn;
    s = 0.5f * (1.0f + vh.z);
    p2 = fmaf(1.0f - s, sqrtf(fmaxf(0.0f, 1.0f - p1 * p1)), s * p2);
    rest = sqrtf(fmaxf(0.0f, (1.0f - p1 * p1) - p2 * p2));
    nh = mk(fmaf(vh.x, rest, fmaf(t2.x, p2, t1.x * p1)),
            fmaf(vh.y, rest, fmaf(t2.y, p2, t1.y * p1)),
            fmaf(vh.z, rest, fmaf(t2.z, p2, t1.z * p1)));
    ne = vnormalize(mk(alpha * nh.x, alpha * nh.y, fmaxf(0.0f, nh.z)));
    k = 2.0f * vdot(wo, ne);
    return mk(fmaf(k, ne.x, -wo.x), fmaf(k, ne.y, -wo.y), fmaf(k, ne.z, -wo.z));
}

/* d/d(alpha) log f_ggx(wo, wi), FP64 from the FP32 directions */
static double ggx_dlogf_dalpha(v3 wo, v3 wi, double alpha)
{
    double hx = (double)wo.x + wi.x, hy = (double)wo.y + wi.y, hz = (double)wo.z + wi.z;
    double hl = sqrt(hx * hx + hy * hy + hz * hz);
    double c2 = (hz / hl) * (hz / hl), a2 = alpha * alpha;
    double dlogd = 2.0 / alpha - 4.0 * alpha * c2 / (c2 * (a2 - 1.0) + 1.0);
    double to = ((double)wo.x * wo.x + (double)wo.y * wo.y) / ((double)wo.z * wo.z);
    double ti = ((double)wi.x * wi.x + (double)wi.y * wi.y) / ((double)wi.z * wi.z);
    double so = sqrt(1.0 + a2 * to), si = sqrt(1.0 + a2 * ti);
    double lam_o = 0.5 * (so - 1.0), lam_i = 0.5 * (si - 1.0);
    double dlo = 0.5 * alpha * to / so, dli = 0.5 * alpha * ti / si;
    return dlogd - (dlo + dli) / (1.0 + lam_o + lam_i);
}

/* exposed for the BSDF pins (local frame, z = normal) */
float orc_ggx_f(const float wo[3], const float wi[3], float alpha, float F)
{
    return ggx_f(vload(wo), vload(wi), alpha, F);
}
float orc_ggx_pdf(const float wo[3], const float wi[3], float alpha) { return ggx_pdf(vload(wo), vload(wi), alpha); }
void orc_ggx_sample(const float wo[3], float alpha, float u0, float u1, float wi[3])
{
    v3 w = ggx_sample_vndf(vload(wo), alpha, u0, u1);
    wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
}
double orc_ggx_dlogf_dalpha(const float wo[3], const float wi[3], double alpha)
{
    return ggx_dlogf_dalpha(vload(wo), vload(wi), alpha);
}
void orc_cosine_sample(float u0, float u1, float out[3])
{
    float r = sqrtf(u0), sn, cs;
    orc_sincos2pi(u1, &sn, &cs);
    out[0] = r * cs;
    out[1] = r * sn;
    out[2] = sqrtf(1.0f - u0);
}

/* Isotropic phase function of the homogeneous medium (Sec. 4.1): a
 * direction uniform on the unit sphere, z = 1 - 2 u0 uniform in [-1, 1] and
 * the azimuth 2 pi u1 (Archimedes' hat-box theorem). */
void orc_phase_sample(float u0, float u1, float out[3])
{
    float z = 1.0f - (u0 + u0);
    float r = sqrtf(fmaxf(0.0f, 1.0f - z * z)), sn, cs;
    orc_sincos2pi(u1, &sn, &cs);
    out[0] = r * cs;
    out[1] = r * sn;
    out[2] = z;
}

/* ------------------------------------------------------------------------ */
/* One path (Eqs. 1-9 and the histogram rule).                              */
/* ------------------------------------------------------------------------ */
#define SHADOW_SHRINK (1.0f - 0x1p-10f)

static void path_reset(orc_path* rec)
{
    rec->n_vert = 0;
}

/* Evaluates f*cos for the light direction at a surface vertex and the
 * derivative factors of log f.  Returns 0 if the BSDF is zero there. */
static float surface_fcos(const struct orc_prepared* P, const orc_render* R, int k, v3 n, v3 wo, v3 wl,
                          double* dalb, double* drough)
{
    float albedo = R->albedo ? R->albedo[k] : P->albedo[k];
    float cos_l = vdot(n, wl);
    *dalb = 0.0;
    *drough = 0.0;
    if (!(cos_l > 0.0f)) return 0.0f;
    if (P->mat[k] == ORC_MAT_GGX) {
        float alpha = R->roughness ? R->roughness[k] : P->rough[k];
        v3 t, b, wol, wll;
        float f;
        onb(n, &t, &b);
        wol = mk(vdot(wo, t), vdot(wo, b), vdot(wo, n));
        wll = mk(vdot(wl, t), vdot(wl, b), vdot(wl, n));
        f = ggx_f(wol, wll, alpha, albedo);
        if (!(f > 0.0f)) return 0.0f;
        *dalb = 1.0 / (double)albedo;
        *drough = ggx_dlogf_dalpha(wol, wll, (double)alpha);
        return f * wll.z;
    }
    *dalb = 1.0 / (double)albedo;
    return (albedo * ORC_INV_PI_F) * cos_l;
}

/* GGX continuation in the local frame: visible-normal sample with alpha_s,
 * weight f_alpha cos / pdf_alpha_s.  With alpha_s == alpha (no frozen
 * proposal) the weight reduces to F G2(wo,wi) / G1(wo). */
static float ggx_sample_weight(v3 wol, float alpha, float alpha_s, float F, int frozen, float u0, float u1,
                               v3* wil_out)
{
    v3 wil;
    if (!(wol.z > 0.0f)) return 0.0f;
    wil = ggx_sample_vndf(wol, alpha_s, u0, u1);
    *wil_out = wil;
    if (!(wil.z > 0.0f)) return 0.0f;
    if (frozen) {
        float pdf = ggx_pdf(wol, wil, alpha_s);
        float f = ggx_f(wol, wil, alpha, F);
        if (!(pdf > 0.0f)) return 0.0f;
        return (f * wil.z) / pdf;
    } else {
        float a2 = alpha * alpha;
        float lo = ggx_lambda(wol, a2), li = ggx_lambda(wil, a2);
        return F * ((1.0f + lo) / ((1.0f + lo) + li));
    }
}

/* Continuation sample at a surface vertex; returns the weight (0 ends the
 * path) and the new direction. */
static float surface_sample(const struct orc_prepared* P, const orc_render* R, int k, v3 n, v3 wo,
                            const float u[4], v3* wi_out, double* dalb, double* drough)
{
    float albedo = R->albedo ? R->albedo[k] : P->albedo[k];
    v3 t, b;
    onb(n, &t, &b);
    *dalb = 1.0 / (double)albedo;
    *drough = 0.0;
    if (P->mat[k] == ORC_MAT_GGX) {
        float alpha = R->roughness ? R->roughness[k] : P->rough[k];
        float alpha_s = R->frozen_proposal ? P->rough[k] : alpha;
        v3 wol = mk(vdot(wo, t), vdot(wo, b), vdot(wo, n));
        v3 wil = mk(0.0f, 0.0f, 0.0f);
        float w = ggx_sample_weight(wol, alpha, alpha_s, albedo, R->frozen_proposal, u[0], u[1], &wil);
        if (!(w > 0.0f)) return 0.0f;
        *drough = ggx_dlogf_dalpha(wol, wil, (double)alpha);
        *wi_out = to_world(t, b, n, wil);
        return w;
    } else {
        float l[3];
        orc_cosine_sample(u[0], u[1], l);
        *wi_out = to_world(t, b, n, mk(l[0], l[1], l[2]));
        return albedo;
    }
}

/* Smooth dielectric interface between the space around the meshes (index
 * eta_amb) and the inside of triangle k's mesh (index eta_k), the inside
 * lying against the winding normal ng = e1 x e2.  wo is the direction back
 * along the arriving ray, n = ng or -ng on wo's side.  The event is
 * reflection with the unpolarised Fresnel reflectance F (1 beyond the
 * critical angle), else refraction by Snell's law, each sampled with its own
 * probability; the weight is 1 for reflection and (eta_i / eta_t)^2 for
 * refraction, since radiance divided by eta^2 is what crosses the interface
 * unchanged (times 1 - F).  u0 decides.  Sets the new direction, the
 * offset origin, the index of the medium the path continues in and whether
 * that is the inside; returns the weight. */
/* Unpolarised Fresnel reflectance of light arriving at cosine ci from the
 * side of index eta_i: the mean of the squared s and p amplitude ratios,
 * 1 beyond the critical angle; *ct = cosine of the refracted direction. */
static float fresnel_dielectric(float ci, float eta_i, float eta_t, float* ct)
{
    float eta_r = eta_i / eta_t;
    float st2 = (eta_r * eta_r) * (1.0f - ci * ci);
    float rs, rp;
    *ct = 0.0f;
    if (!(st2 < 1.0f)) return 1.0f;
    *ct = sqrtf(1.0f - st2);
    rs = (eta_i * ci - eta_t * *ct) / (eta_i * ci + eta_t * *ct);
    rp = (eta_t * ci - eta_i * *ct) / (eta_t * ci + eta_i * *ct);
    return 0.5f * (rs * rs + rp * rp);
}

float orc_fresnel(float ci, float eta_i, float eta_t)
{
    float ct;
    return fresnel_dielectric(ci, eta_i, eta_t, &ct);
}

static float dielectric_sample(v3 x, v3 ng, v3 n, v3 wo, float eta_amb, float eta_k, float u0, v3* wi, v3* o,
                               float* eta_out, int* inside_out)
{
    int entering = !(vdot(ng, wo) < 0.0f);
    float ci = vdot(n, wo);
    float eta_i = entering ? eta_amb : eta_k, eta_t = entering ? eta_k : eta_amb;
    float eta_r = eta_i / eta_t;
    float ct;
    float F = fresnel_dielectric(ci, eta_i, eta_t, &ct);
    if (u0 < F) {
        *wi = vnormalize(vsub(vscale(n, 2.0f * ci), wo));
        *o = offset_ray(x, n);
        *inside_out = !entering;
        *eta_out = eta_i;
        return 1.0f;
    }
    *wi = vnormalize(vadd(vscale(wo, -eta_r), vscale(n, eta_r * ci - ct)));
    *o = offset_ray(x, vneg(n));
    *inside_out = entering;
    *eta_out = eta_t;
    return eta_r * eta_r;
}

static void record(orc_path* rec, int tri, float c, float opl_c, const orc_scene* sc,
                   double dn_alb, double dn_rough)
{
    orc_vertex* v = &rec->v[rec->n_vert - 1];
    float q = (opl_c - sc->bin_start) / sc->bin_width;
    v->has_c = 1;
    v->c = c;
    v->opl_c = opl_c;
    v->bin = (q >= 0.0f && q < (float)sc->n_bins) ? (int)q : -1;
    v->tri = tri;
    v->dn_alb = dn_alb;
    v->dn_rough = dn_rough;
}

int orc_trace_path(const orc_prepared* P, const orc_render* R, uint32_t pix, uint32_t sample, orc_path* rec)
{
    const orc_scene* sc = &P->sc;
    int confocal = (sc->sensor == ORC_SENSOR_CONFOCAL);
    int has_medium = (sc->sigma_t > 0.0f);
    float u[4], beta, opl = 0.0f, u_ff, forced_t = 0.0f;
    v3 o, d, target, wall_n = vload(sc->wall_normal);
    int prev = -1, vmax, v, forced_k = -1;
    /* index of the medium the path is in (Eq. 3: a segment's time of flight
     * is its length times eta) and whether that is a dielectric's inside;
     * the participating medium fills only the space around the meshes */
    const float eta_amb = (sc->medium_ior > 0.0f) ? sc->medium_ior : 1.0f;
    float eta = eta_amb;
    int inside = 0;

    path_reset(rec);
    draw(R, pix, sample, 0, u);
    u_ff = u[2];
    if (!confocal) {
        int ix = (int)(pix % (uint32_t)sc->width), iy = (int)(pix / (uint32_t)sc->width);
        float jx = R->pixel_centre ? 0.5f : u[0], jy = R->pixel_centre ? 0.5f : u[1];
        float fx = (float)ix + jx, fy = (float)iy + jy;
        float sx = ((fx * 2.0f) / (float)sc->width - 1.0f) * sc->tan_x;
        float sy = (1.0f - (fy * 2.0f) / (float)sc->height) * sc->tan_y;
        v3 cr = vload(sc->cam_right), cu = vload(sc->cam_up), cf = vload(sc->cam_fwd);
        d = vnormalize(mk(fmaf(cu.x, sy, fmaf(cr.x, sx, cf.x)),
                          fmaf(cu.y, sy, fmaf(cr.y, sx, cf.y)),
                          fmaf(cu.z, sy, fmaf(cr.z, sx, cf.z))));
        o = vload(sc->cam_origin);
        beta = 1.0f;
        vmax = R->max_depth - 1;
        target = vload(sc->light_pos);
    } else if (!R->nlos_area) {
        /* the traced path starts at the scan point on the relay wall: a
         * Lambertian vertex whose cosine-sampling weight is its albedo */
        v3 xs = vload(P->scan + 3 * pix), t, b;
        float l[3];
        onb(wall_n, &t, &b);
        orc_cosine_sample(u[0], u[1], l);
        d = to_world(t, b, wall_n, mk(l[0], l[1], l[2]));
        o = offset_ray(xs, wall_n);
        beta = sc->wall_albedo;
        vmax = R->max_depth - 3;
        target = xs;
    } else {
        /* NLOS area sampling: the hidden vertex is a point drawn on the
         * sampling set (triangle by u0 through the prefix sums of the
         * weights, point uniformly within it by u1, u2), the first segment
         * joins it to the offset scan point; its throughput is
         * f_wall cos_s / p_w with the solid angle pdf p_w = p_A r^2 / cos_h,
         * p_A = w_k / (W A_k).  Its visibility is the shadow test of the
         * connection back to the scan point, which runs the same segment. */
        v3 xs = vload(P->scan + 3 * pix), e1, e2, v0, xh, dv, ng;
        const int region = P->pix_region[pix];
        const double* cdf = P->area_cdf + (size_t)region * (size_t)sc->n_tris;
        const double target_area = (double)u[0] * P->weight_total[region];
        int lo = 0, hi = sc->n_tris - 1;
        float su, b1, b2, r2, r, cos_s0, cos_h, g;
        if (!(P->weight_total[region] > 0.0)) return 0;
        while (lo < hi) { /* first triangle whose prefix sum exceeds the target */
            int mid = (lo + hi) / 2;
            if (cdf[mid] > target_area) hi = mid;
            else lo = mid + 1;
        }
        {
            const float* tr = P->tri + 9 * lo;
            v0 = vload(tr);
            e1 = vsub(vload(tr + 3), v0);
            e2 = vsub(vload(tr + 6), v0);
        }
        su = sqrtf(u[1]);
        b1 = su * (1.0f - u[2]);
        b2 = su * u[2];
        xh = mk(fmaf(b1, e1.x, fmaf(b2, e2.x, v0.x)), fmaf(b1, e1.y, fmaf(b2, e2.y, v0.y)),
                fmaf(b1, e1.z, fmaf(b2, e2.z, v0.z)));
        o = offset_ray(xs, wall_n);
        dv = vsub(xh, o);
        r2 = vdot(dv, dv);
        r = sqrtf(r2);
        d = vscale(dv, 1.0f / r);
        ng = vnormalize(vcross(e1, e2));
        cos_s0 = vdot(wall_n, d);
        cos_h = fabsf(vdot(ng, d));
        if (!(cos_s0 > 0.0f) || !(cos_h > 0.0f)) return 0;
        g = (cos_s0 * cos_h) / r2;
        beta = ((sc->wall_albedo * P->area_invp[(size_t)region * (size_t)sc->n_tris + lo]) * ORC_INV_PI_F) * g;
        vmax = R->max_depth - 3;
        target = xs;
        forced_k = lo;
        forced_t = r;
    }

    for (v = 1; v <= vmax; ++v) {
        ray_t ray = make_ray(o, d);
        float t_hit = INFINITY, seg, fcos, em, cos_s;
        int k = -1, hit, medium_event = 0;
        v3 x, n, wo, dl, wl, ng = mk(0.0f, 0.0f, 0.0f);
        double dn_alb = 0.0, dn_rough = 0.0;
        int first_blocked = 0;
        orc_vertex* vert;
        if (v == 1 && forced_k >= 0) {
            hit = 1;
            k = forced_k;
            t_hit = forced_t;
        } else {
            hit = closest(P, &ray, prev, &t_hit, &k);
        }
        if (has_medium && !inside) {
            float t_ff = -orc_log1m(u_ff) / sc->sigma_t;
            if (!hit || t_ff < t_hit) {
                medium_event = 1;
                t_hit = t_ff;
            }
        }
        if (!hit && !medium_event) break;
        seg = t_hit;
        x = vray(o, d, t_hit);
        if (!(sc->camera_unwarp && !confocal && v == 1)) opl = opl + seg * eta;
        wo = vneg(d);
        vert = &rec->v[rec->n_vert++];
        memset(vert, 0, sizeof(*vert));
        vert->tri = medium_event ? -1 : k;
        vert->bin = -1;

        dl = vsub(target, x);
        {
            float d2 = vdot(dl, dl);
            float dist = sqrtf(d2);
            wl = vscale(dl, 1.0f / dist);
            if (confocal) {
                cos_s = -vdot(wall_n, wl);
                em = (cos_s > 0.0f) ? ((sc->wall_albedo * sc->laser_power) * ORC_INV_PI_F) * cos_s : 0.0f;
            } else {
                em = sc->light_intensity;
            }
            if (medium_event) {
                beta = beta * sc->medium_albedo;
                n = mk(0.0f, 0.0f, 0.0f);
                if (em > 0.0f) {
                    ray_t sh = make_ray(x, wl);
                    if (!occluded(P, &sh, -1, dist * SHADOW_SHRINK)) {
                        float c = ((beta * ORC_INV_4PI_F) * em) / d2;
                        c = c * expf(-(sc->sigma_t * dist));
                        record(rec, -1, c, opl + dist * eta, sc, 0.0, 0.0);
                    }
                }
            } else {
                const float* tr = P->tri + 9 * k;
                v3 e1 = vsub(vload(tr + 3), vload(tr)), e2 = vsub(vload(tr + 6), vload(tr));
                ng = vnormalize(vcross(e1, e2));
                n = (vdot(ng, wo) < 0.0f) ? vneg(ng) : ng;
                if (!(vdot(n, wo) > 0.0f)) {
                    rec->n_vert--;
                    break;
                }
                /* scattering delay (Eq. 10): exponentially distributed with
                 * the triangle's mean, word 2 of the vertex's Philox block;
                 * it delays every contribution from this vertex on */
                if (P->delay && P->delay[k] > 0.0f) {
                    float ud[4];
                    draw(R, pix, sample, (uint32_t)v, ud);
                    opl = opl + P->delay[k] * -orc_log1m(ud[2]);
                }
                if (P->mat[k] != ORC_MAT_DIELECTRIC) {
                    fcos = surface_fcos(P, R, k, n, wo, wl, &dn_alb, &dn_rough);
                    if (fcos > 0.0f && em > 0.0f) {
                        ray_t sh = make_ray(offset_ray(x, n), wl);
                        if (!occluded(P, &sh, k, dist * SHADOW_SHRINK)) {
                            float c = ((beta * fcos) * em) / d2;
                            if (has_medium && !inside) c = c * expf(-(sc->sigma_t * dist));
                            record(rec, k, c, opl + dist * eta, sc, dn_alb, dn_rough);
                        }
                    }
                }
                if (forced_k >= 0 && v == 1 && v < vmax) {
                    /* a path continued from the drawn hidden vertex needs its
                     * first segment unoccluded: the shadow test back to the
                     * scan point runs along that segment */
                    ray_t sh = make_ray(offset_ray(x, n), wl);
                    first_blocked = occluded(P, &sh, k, dist * SHADOW_SHRINK);
                }
            }
        }
        if (v == vmax || first_blocked) break;
        draw(R, pix, sample, (uint32_t)v, u);
        if (medium_event) {
            float w[3];
            orc_phase_sample(u[0], u[1], w);
            d = mk(w[0], w[1], w[2]);
            prev = -1;
            o = x;
            vert->dc_alb = 0.0;
            vert->dc_rough = 0.0;
        } else if (P->mat[k] == ORC_MAT_DIELECTRIC) {
            /* a delta interface: no next-event connection above, no
             * parameter of the gradients */
            v3 wi, on;
            float w = dielectric_sample(x, ng, n, wo, eta_amb, P->ior[k], u[0], &wi, &on, &eta, &inside);
            vert->has_cont = 1;
            beta = beta * w;
            d = wi;
            o = on;
            prev = k;
        } else {
            v3 wi;
            double ca, cr;
            float w = surface_sample(P, R, k, n, wo, u, &wi, &ca, &cr);
            if (!(w > 0.0f)) break;
            vert->dc_alb = ca;
            vert->dc_rough = cr;
            vert->has_cont = 1;
            beta = beta * w;
            d = wi;
            o = offset_ray(x, n);
            prev = k;
        }
        u_ff = u[3];
    }
    return rec->n_vert;
}

/* ------------------------------------------------------------------------ */
/* Film render and adjoint, threaded over pixels.                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    const struct orc_prepared* P;
    const orc_render* R;
    const int32_t* pixels;
    int n_pix, tid, nthreads;
    double* film;  /* [n_pix][T] */
    double* steady;
    double* oow;
    /* forward-mode derivative */
    const double* v_alb;
    const double* v_rough;
    double* dfilm; /* [n_pix][T] */
    /* phasor film */
    const double* freqs;
    int n_freq;
    double* phasor; /* [n_pix][n_freq][2] */
    /* adjoint */
    const float* grad_film; /* full film layout [P][T] */
    double* g_alb;
    double* g_rough;
} job_t;

static void* render_worker(void* arg)
{
    job_t* J = (job_t*)arg;
    const orc_scene* sc = &J->P->sc;
    orc_path* rec = (orc_path*)malloc(sizeof(orc_path));
    int i;
    uint32_t s;
    int T = sc->n_bins;
    for (i = J->tid; i < J->n_pix; i += J->nthreads) {
        uint32_t pix = (uint32_t)J->pixels[i];
        double* row = J->film + (size_t)i * (size_t)T;
        for (s = 0; s < (uint32_t)J->R->spp; ++s) {
            int v;
            orc_trace_path(J->P, J->R, pix, J->R->sample_offset + s, rec);
            for (v = 0; v < rec->n_vert; ++v) {
                const orc_vertex* vx = &rec->v[v];
                if (!vx->has_c) continue;
                if (vx->bin >= 0) row[vx->bin] += (double)vx->c;
                else if (J->oow) J->oow[i] += (double)vx->c;
                if (J->steady) J->steady[i] += (double)vx->c;
            }
        }
    }
    free(rec);
    return NULL;
}

/* Sec. 4.3, Eq. 14: every contribution c of the pixel's paths adds
 * c exp(-2 pi i f tof) for each frequency f (cycles per metre of optical
 * path), with tof the optical path length of the connected path; there is
 * no window, the transform covers all times. */
static void* phasor_worker(void* arg)
{
    job_t* J = (job_t*)arg;
    orc_path* rec = (orc_path*)malloc(sizeof(orc_path));
    const double two_pi = 6.283185307179586476925286766559;
    int i, j;
    uint32_t s;
    for (i = J->tid; i < J->n_pix; i += J->nthreads) {
        uint32_t pix = (uint32_t)J->pixels[i];
        double* row = J->phasor + (size_t)i * (size_t)J->n_freq * 2;
        for (s = 0; s < (uint32_t)J->R->spp; ++s) {
            int v;
            orc_trace_path(J->P, J->R, pix, J->R->sample_offset + s, rec);
            for (v = 0; v < rec->n_vert; ++v) {
                const orc_vertex* vx = &rec->v[v];
                if (!vx->has_c) continue;
                for (j = 0; j < J->n_freq; ++j) {
                    const double ang = two_pi * J->freqs[j] * (double)vx->opl_c;
                    row[2 * j] += (double)vx->c * cos(ang);
                    row[2 * j + 1] -= (double)vx->c * sin(ang);
                }
                if (J->steady) J->steady[i] += (double)vx->c;
            }
        }
    }
    free(rec);
    return NULL;
}

/* Sec. 4.4, forward mode: at a fixed seed with the sampling held fixed, a
 * contribution c_j carries the product of the continuation weights of the
 * vertices before it and the connection factor at its own vertex, so its
 * derivative along the direction v is c_j times (the sum over earlier
 * vertices of d log w . v plus d log f_nee . v of its vertex). */
static double along(const job_t* J, int tri, double d_alb, double d_rough)
{
    double d = 0.0;
    if (tri < 0) return 0.0;
    if (J->v_alb) d += J->v_alb[tri] * d_alb;
    if (J->v_rough) d += J->v_rough[tri] * d_rough;
    return d;
}

static void* tangent_worker(void* arg)
{
    job_t* J = (job_t*)arg;
    const orc_scene* sc = &J->P->sc;
    orc_path* rec = (orc_path*)malloc(sizeof(orc_path));
    int i;
    uint32_t s;
    int T = sc->n_bins;
    for (i = J->tid; i < J->n_pix; i += J->nthreads) {
        uint32_t pix = (uint32_t)J->pixels[i];
        double* row = J->film + (size_t)i * (size_t)T;
        double* drow = J->dfilm + (size_t)i * (size_t)T;
        for (s = 0; s < (uint32_t)J->R->spp; ++s) {
            int v;
            double tang = 0.0;
            orc_trace_path(J->P, J->R, pix, J->R->sample_offset + s, rec);
            for (v = 0; v < rec->n_vert; ++v) {
                const orc_vertex* vx = &rec->v[v];
                if (vx->has_c) {
                    if (J->steady) J->steady[i] += (double)vx->c;
                    if (vx->bin >= 0) {
                        row[vx->bin] += (double)vx->c;
                        drow[vx->bin] += (double)vx->c * (tang + along(J, vx->tri, vx->dn_alb, vx->dn_rough));
                    }
                }
                if (vx->has_cont) tang += along(J, vx->tri, vx->dc_alb, vx->dc_rough);
            }
        }
    }
    free(rec);
    return NULL;
}

static void* backward_worker(void* arg)
{
    job_t* J = (job_t*)arg;
    const orc_scene* sc = &J->P->sc;
    orc_path* rec = (orc_path*)malloc(sizeof(orc_path));
    double a[ORC_MAX_VERT];
    int i;
    uint32_t s;
    int T = sc->n_bins;
    double inv_n = 1.0 / (double)J->R->spp;
    for (i = J->tid; i < J->n_pix; i += J->nthreads) {
        uint32_t pix = (uint32_t)J->pixels[i];
        const float* delta = J->grad_film + (size_t)pix * (size_t)T;
        double* row = J->film ? J->film + (size_t)i * (size_t)T : NULL;
        for (s = 0; s < (uint32_t)J->R->spp; ++s) {
            int v, nv;
            double suffix = 0.0;
            nv = orc_trace_path(J->P, J->R, pix, J->R->sample_offset + s, rec);
            for (v = 0; v < nv; ++v) {
                const orc_vertex* vx = &rec->v[v];
                a[v] = 0.0;
                if (vx->has_c && vx->bin >= 0) {
                    a[v] = (double)delta[vx->bin] * (double)vx->c * inv_n;
                    if (row) row[vx->bin] += (double)vx->c;
                }
            }
            /* contribution j depends on the continuation BSDF of every
             * earlier vertex and on the NEE BSDF of its own vertex */
            for (v = nv - 1; v >= 0; --v) {
                const orc_vertex* vx = &rec->v[v];
                if (vx->tri >= 0) {
                    double ga = a[v] * vx->dn_alb, gr = a[v] * vx->dn_rough;
                    if (vx->has_cont) {
                        ga += suffix * vx->dc_alb;
                        gr += suffix * vx->dc_rough;
                    }
                    J->g_alb[vx->tri] += ga;
                    J->g_rough[vx->tri] += gr;
                }
                suffix += a[v];
            }
        }
    }
    free(rec);
    return NULL;
}

static int run_jobs(job_t* base, int nthreads, void* (*fn)(void*))
{
    pthread_t th[256];
    job_t jobs[256];
    int t;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    for (t = 0; t < nthreads; ++t) {
        jobs[t] = *base;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
    }
    if (nthreads == 1) {
        fn(&jobs[0]);
        return 0;
    }
    for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, fn, &jobs[t]);
    for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* Area sampling of the hidden vertex is defined for confocal paths with at
 * least one hidden vertex (max_depth >= 4) without a participating medium. */
static int render_ok(const orc_prepared* P, const orc_render* R)
{
    if (!P || !R || R->spp <= 0 || R->max_depth < 1) return 0;
    if (!R->nlos_area) return 1;
    return P->sc.sensor == ORC_SENSOR_CONFOCAL && R->max_depth >= 4 && !(P->sc.sigma_t > 0.0f) &&
           P->area_total > 0.0;
}

int orc_render_film(const orc_prepared* P, const orc_render* R, const int32_t* pixels, int n_pix,
                    double* film, double* steady, double* oow, int nthreads)
{
    job_t J;
    int i;
    size_t T = (size_t)P->sc.n_bins;
    double inv_n;
    if (!render_ok(P, R)) return -1;
    memset(&J, 0, sizeof(J));
    J.P = P; J.R = R; J.pixels = pixels; J.n_pix = n_pix;
    J.film = film; J.steady = steady; J.oow = oow;
    memset(film, 0, sizeof(double) * T * (size_t)n_pix);
    if (steady) memset(steady, 0, sizeof(double) * (size_t)n_pix);
    if (oow) memset(oow, 0, sizeof(double) * (size_t)n_pix);
    run_jobs(&J, nthreads, render_worker);
    /* Monte Carlo normalisation 1/N of Eq. 9 */
    inv_n = 1.0 / (double)R->spp;
    for (i = 0; i < n_pix; ++i) {
        size_t b;
        for (b = 0; b < T; ++b) film[(size_t)i * T + b] *= inv_n;
        if (steady) steady[i] *= inv_n;
        if (oow) oow[i] *= inv_n;
    }
    return 0;
}

/* Every next-event contribution of the listed pixels' paths, one entry
 * per contribution (the terms that the histogram of Sec. 3, "Path reuse and
 * histogramming", sums): pixel, sample, vertex (1-based), bin (-1 outside
 * the window), value c (before the 1/N of Eq. 9), time of flight, triangle
 * (-1 for a medium vertex).  Pixel by pixel, sample by sample, vertex by
 * vertex; at most `cap` entries are written, the return value counts all
 * (-1 for an invalid render). */
int64_t orc_render_records(const orc_prepared* P, const orc_render* R, const int32_t* pixels, int n_pix,
                           orc_record* out, int64_t cap)
{
    orc_path* rec;
    int64_t n = 0;
    int i, v;
    uint32_t s;
    if (!render_ok(P, R)) return -1;
    rec = (orc_path*)malloc(sizeof(orc_path));
    if (!rec) return -1;
    for (i = 0; i < n_pix; ++i) {
        for (s = 0; s < (uint32_t)R->spp; ++s) {
            orc_trace_path(P, R, (uint32_t)pixels[i], R->sample_offset + s, rec);
            for (v = 0; v < rec->n_vert; ++v) {
                const orc_vertex* vx = &rec->v[v];
                if (!vx->has_c) continue;
                if (n < cap) {
                    orc_record* o = &out[n];
                    o->pixel = (uint32_t)pixels[i];
                    o->sample = R->sample_offset + s;
                    o->vertex = v + 1;
                    o->bin = vx->bin;
                    o->value = vx->c;
                    o->tof = vx->opl_c;
                    o->tri = vx->tri;
                    o->reserved = 0;
                }
                ++n;
            }
        }
    }
    free(rec);
    return n;
}

int orc_render_tangent(const orc_prepared* P, const orc_render* R, const int32_t* pixels, int n_pix,
                       const double* v_alb, const double* v_rough, double* film, double* dfilm, double* steady,
                       int nthreads)
{
    job_t J;
    int i;
    size_t b, T = (size_t)P->sc.n_bins;
    double inv_n;
    if (!render_ok(P, R) || !film || !dfilm) return -1;
    memset(&J, 0, sizeof(J));
    J.P = P; J.R = R; J.pixels = pixels; J.n_pix = n_pix;
    J.v_alb = v_alb; J.v_rough = v_rough; J.film = film; J.dfilm = dfilm; J.steady = steady;
    memset(film, 0, sizeof(double) * T * (size_t)n_pix);
    memset(dfilm, 0, sizeof(double) * T * (size_t)n_pix);
    if (steady) memset(steady, 0, sizeof(double) * (size_t)n_pix);
    run_jobs(&J, nthreads, tangent_worker);
    inv_n = 1.0 / (double)R->spp;
    for (i = 0; i < n_pix; ++i) {
        for (b = 0; b < T; ++b) {
            film[(size_t)i * T + b] *= inv_n;
            dfilm[(size_t)i * T + b] *= inv_n;
        }
        if (steady) steady[i] *= inv_n;
    }
    return 0;
}

int orc_render_phasor(const orc_prepared* P, const orc_render* R, const int32_t* pixels, int n_pix,
                      const double* freqs, int n_freq, double* phasor, double* steady, int nthreads)
{
    job_t J;
    int i;
    size_t k, n2 = 2 * (size_t)n_freq;
    double inv_n;
    if (!render_ok(P, R) || n_freq < 1 || !freqs || !phasor) return -1;
    memset(&J, 0, sizeof(J));
    J.P = P; J.R = R; J.pixels = pixels; J.n_pix = n_pix;
    J.freqs = freqs; J.n_freq = n_freq; J.phasor = phasor; J.steady = steady;
    memset(phasor, 0, sizeof(double) * n2 * (size_t)n_pix);
    if (steady) memset(steady, 0, sizeof(double) * (size_t)n_pix);
    run_jobs(&J, nthreads, phasor_worker);
    inv_n = 1.0 / (double)R->spp;
    for (i = 0; i < n_pix; ++i) {
        for (k = 0; k < n2; ++k) phasor[(size_t)i * n2 + k] *= inv_n;
        if (steady) steady[i] *= inv_n;
    }
    return 0;
}

int orc_backward(const orc_prepared* P, const orc_render* R, const int32_t* pixels, int n_pix,
                 const float* grad_film, double* g_alb, double* g_rough, double* primal_film, int nthreads)
{
    job_t J;
    int t, nt = P->sc.n_tris;
    double *ga_all, *gr_all;
    pthread_t th[256];
    job_t jobs[256];
    if (!render_ok(P, R)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    memset(&J, 0, sizeof(J));
    J.P = P; J.R = R; J.pixels = pixels; J.n_pix = n_pix; J.grad_film = grad_film;
    J.film = primal_film;
    if (primal_film) memset(primal_film, 0, sizeof(double) * (size_t)P->sc.n_bins * (size_t)n_pix);
    ga_all = (double*)calloc((size_t)nt * (size_t)nthreads, sizeof(double));
    gr_all = (double*)calloc((size_t)nt * (size_t)nthreads, sizeof(double));
    for (t = 0; t < nthreads; ++t) {
        jobs[t] = J;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
        jobs[t].g_alb = ga_all + (size_t)t * (size_t)nt;
        jobs[t].g_rough = gr_all + (size_t)t * (size_t)nt;
    }
    if (nthreads == 1) backward_worker(&jobs[0]);
    else {
        for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, backward_worker, &jobs[t]);
        for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    memset(g_alb, 0, sizeof(double) * (size_t)nt);
    memset(g_rough, 0, sizeof(double) * (size_t)nt);
    for (t = 0; t < nthreads; ++t) {
        int k;
        for (k = 0; k < nt; ++k) {
            g_alb[k] += ga_all[(size_t)t * (size_t)nt + k];
            g_rough[k] += gr_all[(size_t)t * (size_t)nt + k];
        }
    }
    if (primal_film) {
        size_t i, n = (size_t)P->sc.n_bins * (size_t)n_pix;
        double inv_n = 1.0 / (double)R->spp;
        for (i = 0; i < n; ++i) primal_film[i] *= inv_n;
    }
    free(ga_all);
    free(gr_all);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Batched entry points for the exhaustive numerics pins.                   */
/* ------------------------------------------------------------------------ */
void orc_sincos2pi_n(int64_t n, const float* u, float* s, float* c)
{
    int64_t i;
    for (i = 0; i < n; ++i) orc_sincos2pi(u[i], s + i, c + i);
}

void orc_log1m_n(int64_t n, const float* u, float* out)
{
    int64_t i;
    for (i = 0; i < n; ++i) out[i] = orc_log1m(u[i]);
}

void orc_philox_n(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    int64_t i;
    for (i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

void orc_ggx_eval_n(int64_t n, const float* wo, const float* wi, const float* alpha, const float* F,
                    float* f_out, float* pdf_out)
{
    int64_t i;
    for (i = 0; i < n; ++i) {
        v3 a = vload(wo + 3 * i), b = vload(wi + 3 * i);
        f_out[i] = ggx_f(a, b, alpha[i], F[i]);
        pdf_out[i] = ggx_pdf(a, b, alpha[i]);
    }
}

void orc_ggx_sample_n(int64_t n, const float* wo, const float* alpha, const float* alpha_s, const float* F,
                      int frozen, const float* u0, const float* u1, float* wi_out, float* w_out)
{
    int64_t i;
    for (i = 0; i < n; ++i) {
        v3 wil = mk(0.0f, 0.0f, 0.0f);
        w_out[i] = ggx_sample_weight(vload(wo + 3 * i), alpha[i], alpha_s[i], F[i], frozen, u0[i], u1[i], &wil);
        wi_out[3 * i] = wil.x; wi_out[3 * i + 1] = wil.y; wi_out[3 * i + 2] = wil.z;
    }
}

void orc_cosine_sample_n(int64_t n, const float* u0, const float* u1, float* out)
{
    int64_t i;
    for (i = 0; i < n; ++i) orc_cosine_sample(u0[i], u1[i], out + 3 * i);
}

void orc_phase_sample_n(int64_t n, const float* u0, const float* u1, float* out)
{
    int64_t i;
    for (i = 0; i < n; ++i) orc_phase_sample(u0[i], u1[i], out + 3 * i);
}
