// device_math.h -- FP32 device arithmetic of the transient path tracer.
//
// Every routine here follows one fixed operation order (separate roundings
// except where fmaf is written, correctly rounded division and square root)
// so that a hit/miss or a histogram-bin decision is reproducible bit for bit
// by any other implementation of the same order.  Build with
// -ffp-contract=off so that the compiler does not fuse what is written as a
// separate multiply and add.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trhip {

struct vec3 {
    float x, y, z;
};

__device__ __forceinline__ vec3 v3(float x, float y, float z) { return vec3{x, y, z}; }
__device__ __forceinline__ vec3 sub(vec3 a, vec3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ vec3 add(vec3 a, vec3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ vec3 scale(vec3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ vec3 neg(vec3 a) { return v3(-a.x, -a.y, -a.z); }
// dot = fma(x, x', fma(y, y', z*z'))
__device__ __forceinline__ float dot(vec3 a, vec3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ vec3 cross(vec3 a, vec3 b)
{
    return v3(fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)), fmaf(a.x, b.y, -(a.y * b.x)));
}
__device__ __forceinline__ vec3 normalize(vec3 a)
{
    const float inv = 1.0f / sqrtf(dot(a, a));
    return scale(a, inv);
}
// o + t d with one rounding per component
__device__ __forceinline__ vec3 along(vec3 o, vec3 d, float t)
{
    return v3(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z));
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): 10 rounds of two 32x32->64 multiplies with the
// key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 x, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32),
        // not separate high and low multiplies
        const uint64_t p0 = (uint64_t)kM0 * x.a, p1 = (uint64_t)kM1 * x.c;
        x = u32x4{(uint32_t)(p1 >> 32) ^ x.b ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ x.d ^ k1, (uint32_t)p0};
        k0 += kW0;
        k1 += kW1;
    }
    return x;
}

// 24 random bits -> [0, 1 - 2^-24], exact
__device__ __forceinline__ float unit24(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

struct rand4 {
    float u0, u1, u2, u3;
};

__device__ __forceinline__ rand4 draw4(uint32_t pixel, uint32_t sample, uint32_t block, uint32_t stream,
                                       uint32_t k0, uint32_t k1)
{
    const u32x4 r = philox4x32_10(u32x4{pixel, sample, block, stream}, k0, k1);
    return rand4{unit24(r.a), unit24(r.b), unit24(r.c), unit24(r.d)};
}

// ---------------------------------------------------------------------------
// sin and cos of 2 pi u for u = k 2^-24.  u*8 splits exactly into an octant
// and a fraction; the octant angle in [0, pi/4] goes through Taylor
// polynomials (to x^11 for sine, x^12 for cosine) evaluated by Horner with
// fma; octant symmetries are exact sign flips and swaps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_2pi(float u, float& s, float& c)
{
    constexpr float kQuarterPi = float(3.14159265358979323846 / 4.0);
    constexpr float kS3 = float(-1.0 / 6.0), kS5 = float(1.0 / 120.0), kS7 = float(-1.0 / 5040.0);
    constexpr float kS9 = float(1.0 / 362880.0), kS11 = float(-1.0 / 39916800.0);
    constexpr float kC4 = float(1.0 / 24.0), kC6 = float(-1.0 / 720.0), kC8 = float(1.0 / 40320.0);
    constexpr float kC10 = float(-1.0 / 3628800.0), kC12 = float(1.0 / 479001600.0);
    const float x8 = u * 8.0f;
    const int oct = (int)x8;
    const float fr = x8 - (float)oct;
    const bool odd = (oct & 1) != 0;
    const int quad = oct >> 1;
    const float th = (odd ? (1.0f - fr) : fr) * kQuarterPi;
    const float z = th * th;
    float p = fmaf(z, kS11, kS9);
    p = fmaf(z, p, kS7);
    p = fmaf(z, p, kS5);
    p = fmaf(z, p, kS3);
    const float sn = fmaf(th * z, p, th);
    float q = fmaf(z, kC12, kC10);
    q = fmaf(z, q, kC8);
    q = fmaf(z, q, kC6);
    q = fmaf(z, q, kC4);
    q = fmaf(z, q, -0.5f);
    const float cs = fmaf(z, q, 1.0f);
    const float s0 = odd ? cs : sn;
    const float c0 = odd ? sn : cs;
    // rotate by quad * pi/2
    s = (quad == 0) ? s0 : (quad == 1) ? c0 : (quad == 2) ? -s0 : -c0;
    c = (quad == 0) ? c0 : (quad == 1) ? -s0 : (quad == 2) ? -c0 : s0;
}

// ln(1 - u) for u = k 2^-24: y = 1 - u is exact; y = 2^e m with m folded
// into [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m-1)/(m+1), by its odd
// series to s^13; e ln 2 added in a high and a low part.
__device__ __forceinline__ float log_one_minus(float u)
{
    constexpr float kSqrt2 = float(1.41421356237309504880);
    constexpr float kL3 = float(1.0 / 3.0), kL5 = float(1.0 / 5.0), kL7 = float(1.0 / 7.0);
    constexpr float kL9 = float(1.0 / 9.0), kL11 = float(1.0 / 11.0), kL13 = float(1.0 / 13.0);
    constexpr float kLn2Hi = 0.693145751953125f;
    constexpr float kLn2Lo = float(0.693147180559945309417232 - 0.693145751953125);
    const float y = 1.0f - u;
    const uint32_t bits = __float_as_uint(y);
    int e = (int)((bits >> 23) & 0xffu) - 127;
    float m = __uint_as_float((bits & 0x007fffffu) | 0x3f800000u);
    if (m > kSqrt2) {
        m = m * 0.5f;
        e = e + 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = fmaf(z, kL13, kL11);
    p = fmaf(z, p, kL9);
    p = fmaf(z, p, kL7);
    p = fmaf(z, p, kL5);
    p = fmaf(z, p, kL3);
    float r = fmaf(s * z, p, s);
    r = r + r;
    const float ef = (float)e;
    return fmaf(ef, kLn2Hi, fmaf(ef, kLn2Lo, r));
}

// ---------------------------------------------------------------------------
// Frames and ray offsets
// ---------------------------------------------------------------------------
// branchless orthonormal basis around a unit normal (Duff, Burgess,
// Christensen, Hery, Kensler, Liani, Villemin, JCGT 2017)
__device__ __forceinline__ void basis(vec3 n, vec3& t, vec3& b)
{
    const float sg = copysignf(1.0f, n.z);
    const float a = -1.0f / (sg + n.z);
    const float bb = n.x * n.y * a;
    t = v3(1.0f + sg * n.x * n.x * a, sg * bb, -sg * n.x);
    b = v3(bb, sg + n.y * n.y * a, -n.y);
}

__device__ __forceinline__ vec3 local_to_world(vec3 t, vec3 b, vec3 n, vec3 l)
{
    return v3(fmaf(n.x, l.z, fmaf(b.x, l.y, t.x * l.x)), fmaf(n.y, l.z, fmaf(b.y, l.y, t.y * l.x)),
              fmaf(n.z, l.z, fmaf(b.z, l.y, t.z * l.x)));
}

// origin offset of a spawned ray by a few ulps along n (Waechter and Binder,
// "A Fast and Robust Method for Avoiding Self-Intersection", Ray Tracing
// Gems 2019); n points to the side the ray leaves toward
__device__ __forceinline__ float nudge(float p, float n)
{
    constexpr float kOrigin = 1.0f / 32.0f, kFloatScale = 1.0f / 65536.0f, kIntScale = 256.0f;
    if (fabsf(p) < kOrigin) return p + kFloatScale * n;
    const int of = (int)(kIntScale * n);
    const int pi = __float_as_int(p) + ((p < 0.0f) ? -of : of);
    return __int_as_float(pi);
}
__device__ __forceinline__ vec3 nudge(vec3 p, vec3 n) { return v3(nudge(p.x, n.x), nudge(p.y, n.y), nudge(p.z, n.z)); }

// cosine-weighted direction in the local frame (z up)
__device__ __forceinline__ vec3 cosine_dir(float u0, float u1)
{
    float s, c;
    sincos_2pi(u1, s, c);
    const float r = sqrtf(u0);
    return v3(r * c, r * s, sqrtf(1.0f - u0));
}

// ---------------------------------------------------------------------------
// GGX conductor: D, height-correlated Smith G2, reflectance F = albedo;
// visible-normal sampling (Heitz, JCGT 2018).
// ---------------------------------------------------------------------------
constexpr float kPi = float(3.14159265358979323846);
constexpr float kInvPi = float(1.0 / 3.14159265358979323846);
constexpr float kInv4Pi = float(1.0 / (4.0 * 3.14159265358979323846));

__device__ __forceinline__ float smith_lambda(vec3 w, float a2)
{
    const float tan2 = fmaf(w.x, w.x, w.y * w.y) / (w.z * w.z);
    return (sqrtf(fmaf(a2, tan2, 1.0f)) - 1.0f) * 0.5f;
}

__device__ __forceinline__ float ggx_ndf(float hz, float a2)
{
    const float c2 = hz * hz;
    const float den = fmaf(c2, a2 - 1.0f, 1.0f);
    return a2 / ((kPi * den) * den);
}

__device__ __forceinline__ float ggx_eval(vec3 wo, vec3 wi, float alpha, float F)
{
    if (!(wo.z > 0.0f) || !(wi.z > 0.0f)) return 0.0f;
    const vec3 h = normalize(v3(wo.x + wi.x, wo.y + wi.y, wo.z + wi.z));
    const float a2 = alpha * alpha;
    const float d = ggx_ndf(h.z, a2);
    const float lo = smith_lambda(wo, a2);
    const float li = smith_lambda(wi, a2);
    const float g2 = 1.0f / ((1.0f + lo) + li);
    return ((F * d) * g2) / ((4.0f * wo.z) * wi.z);
}

__device__ __forceinline__ float ggx_vndf_pdf(vec3 wo, vec3 wi, float alpha)
{
    const float a2 = alpha * alpha;
    const vec3 h = normalize(v3(wo.x + wi.x, wo.y + wi.y, wo.z + wi.z));
    const float g1 = 1.0f / (1.0f + smith_lambda(wo, a2));
    return (g1 * ggx_ndf(h.z, a2)) / (4.0f * wo.z);
}

__device__ __forceinline__ vec3 ggx_vndf_sample(vec3 wo, float alpha, float u0, float u1)
{
    const vec3 vh = normalize(v3(alpha * wo.x, alpha * wo.y, wo.z));
    const float lensq = fmaf(vh.x, vh.x, vh.y * vh.y);
    vec3 t1;
    if (lensq > 0.0f) {
        const float inv = 1.0f / sqrtf(lensq);
        t1 = v3(-vh.y * inv, vh.x * inv, 0.0f);
    } else {
        t1 = v3(1.0f, 0.0f, 0.0f);
    }
    const vec3 t2 = cross(vh, t1);
    float sn, cs;
    sincos_2pi(u1, sn, cs);
    const float r = sqrtf(u0);
    const float p1 = r * cs;
    float p2 = r * sn;
    const float s = 0.5f * (1.0f + vh.z);
    p2 = fmaf(1.0f - s, sqrtf(fmaxf(0.0f, 1.0f - p1 * p1)), s * p2);
    const float rest = sqrtf(fmaxf(0.0f, (1.0f - p1 * p1) - p2 * p2));
    const vec3 nh = v3(fmaf(vh.x, rest, fmaf(t2.x, p2, t1.x * p1)), fmaf(vh.y, rest, fmaf(t2.y, p2, t1.y * p1)),
                       fmaf(vh.z, rest, fmaf(t2.z, p2, t1.z * p1)));
    const vec3 ne = normalize(v3(alpha * nh.x, alpha * nh.y, fmaxf(0.0f, nh.z)));
    const float k = 2.0f * dot(wo, ne);
    return v3(fmaf(k, ne.x, -wo.x), fmaf(k, ne.y, -wo.y), fmaf(k, ne.z, -wo.z));
}

// d/d(alpha) of log f: d log D / d alpha + d log G2 / d alpha (values only,
// no bin decision depends on it)
__device__ __forceinline__ float ggx_dlog_dalpha(vec3 wo, vec3 wi, float alpha)
{
    const float hx = wo.x + wi.x, hy = wo.y + wi.y, hz = wo.z + wi.z;
    const float c2 = (hz * hz) / (hx * hx + hy * hy + hz * hz);
    const float a2 = alpha * alpha;
    const float dlogd = 2.0f / alpha - 4.0f * alpha * c2 / (c2 * (a2 - 1.0f) + 1.0f);
    const float to = (wo.x * wo.x + wo.y * wo.y) / (wo.z * wo.z);
    const float ti = (wi.x * wi.x + wi.y * wi.y) / (wi.z * wi.z);
    const float so = sqrtf(1.0f + a2 * to), si = sqrtf(1.0f + a2 * ti);
    const float lam = 0.5f * (so - 1.0f) + 0.5f * (si - 1.0f);
    const float dlam = 0.5f * alpha * (to / so + ti / si);
    return dlogd - dlam / (1.0f + lam);
}

}  // namespace trhip
