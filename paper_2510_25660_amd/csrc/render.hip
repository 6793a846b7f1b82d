// render.hip -- transient path tracing kernels for gfx950.
//
// One workgroup owns a tile of consecutive pixels (all their time bins) and
// traces every sample of those pixels, one path per lane at a time.  The
// tile's film rows live in LDS, so contributions are LDS atomics and the
// tile is written to HBM once, with coalesced stores, at the end: no film
// zero-fill pass and no HBM atomics.  (When the deferred form splits a
// tile's samples over several workgroups, the extra ones leave their partial
// tiles in a scratch film that a second pass adds, still without atomics.
// The path form on long films of large scenes is the exception: it adds
// into the film in HBM.)  The BVH traversal stack of each lane lives in LDS
// (stride = block size, so a wave's pushes are contiguous), with 16-bit
// links when the scene is small enough, 32-bit otherwise (then, in the
// HBM-film form, split between LDS and scratch).
//
// Path construction (arXiv 2510.25660, Sec. 3): paths are traced from the
// sensor (pinhole camera, or the scan point on the relay wall for the
// confocal NLOS sensor of Sec. 4.5); at each scattering vertex the point
// emitter is connected by next-event estimation (the G V terms of Eq. 8),
// the contribution lands in bin floor((opl - b_start) / b_width) of the
// path's pixel, where opl is the summed segment length (Eqs. 3-4) plus the
// connection; the continuation is importance sampled (cosine for
// Lambertian, visible normals for GGX; isotropic phase in a homogeneous
// medium, Sec. 4.1).  The film is the estimator of Eq. 9 (divided by N).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "device_math.h"

#include "internal.h"
#include "scene_view.h"

namespace trhip {

namespace {

struct Ray {
    vec3 o, d, inv, oi;
    uint32_t rx, ry, rz;  // 16 where the direction's component is negative, else 0
};

__device__ __forceinline__ float guard(float x) { return (fabsf(x) < 1e-30f) ? copysignf(1e-30f, x) : x; }

__device__ __forceinline__ Ray make_ray(vec3 o, vec3 d)
{
    Ray r;
    r.o = o;
    r.d = d;
    r.inv = v3(1.0f / guard(d.x), 1.0f / guard(d.y), 1.0f / guard(d.z));
    r.oi = v3(o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z);
    r.rx = (r.inv.x < 0.0f) ? 16u : 0u;
    r.ry = (r.inv.y < 0.0f) ? 16u : 0u;
    r.rz = (r.inv.z < 0.0f) ? 16u : 0u;
    return r;
}

// entry/exit of a box along the ray; planes at fma(bound, 1/d, -o/d)
__device__ __forceinline__ void slab(const Ray& r, float lx, float ly, float lz, float hx, float hy, float hz,
                                     float& tn, float& tf)
{
    const float ax = fmaf(lx, r.inv.x, -r.oi.x), bx = fmaf(hx, r.inv.x, -r.oi.x);
    const float ay = fmaf(ly, r.inv.y, -r.oi.y), by = fmaf(hy, r.inv.y, -r.oi.y);
    const float az = fmaf(lz, r.inv.z, -r.oi.z), bz = fmaf(hz, r.inv.z, -r.oi.z);
    tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
    tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
}

// Two-sided Moller-Trumbore on (v0, e1, e2), for a triangle other than
// `exclude`.  kEarly leaves at a zero determinant or at the excluded
// triangle before the division (records fetched by buffer loads, which the
// compiler issues together).  Otherwise those checks join the first test on
// u, which needs v0: an early exit that needs only the edges lets the
// compiler move v0's global load behind it, and the test then waits for two
// round trips to memory instead of one.  Both orders compute the same
// values; the division by a zero determinant is discarded.
template <bool kEarly>
__device__ __forceinline__ bool intersect_tri(const Ray& r, const TriRec& tr, int exclude, float& t)
{
    const vec3 e1 = v3(tr.e1x, tr.e1y, tr.e1z), e2 = v3(tr.e2x, tr.e2y, tr.e2z);
    const vec3 p = cross(r.d, e2);
    const float det = dot(e1, p);
    const bool skip = det == 0.0f || (int)tr.prim == exclude;
    if (kEarly && skip) return false;
    const float inv = 1.0f / det;
    const vec3 s = sub(r.o, v3(tr.v0x, tr.v0y, tr.v0z));
    const float u = dot(s, p) * inv;
    if ((!kEarly && skip) || u < 0.0f || u > 1.0f) return false;
    const vec3 q = cross(s, e1);
    const float v = dot(r.d, q) * inv;
    if (v < 0.0f || u + v > 1.0f) return false;
    t = dot(e2, q) * inv;
    return t > 0.0f;
}

// Scenes with 16-bit links (at most 32,768 triangles, so nodes and
// triangle records span a few MB) fetch them with buffer loads: a 32-bit
// byte offset against a descriptor held in scalar registers, where a global
// load needs a 64-bit address per lane (the 48-byte record stride costs a
// quarter-rate 64-bit multiply).  Larger scenes use global loads (and the
// compact layout).  The
// descriptor has stride 0 (raw, byte-addressed), `bytes` as its range (a
// load past it returns zeros instead of faulting) and 0x00020000 as its
// fourth word, the value for untyped 32-bit access on gfx9-family GPUs
// (gfx950 included).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float4 buffer_f4(__amdgpu_buffer_rsrc_t R, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(R, (int)off, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

__device__ __forceinline__ TriRec tri_of(float4 a, float4 b, float4 c)
{
    TriRec t;
    t.v0x = a.x; t.v0y = a.y; t.v0z = a.z; t.prim = __float_as_uint(a.w);
    t.e1x = b.x; t.e1y = b.y; t.e1z = b.z; t.unused0 = 0.0f;
    t.e2x = c.x; t.e2y = c.y; t.e2z = c.z; t.unused1 = 0.0f;
    return t;
}

// The record of a leaf test.  kBuf: the TriRec layout of scenes with 16-bit
// links, by buffer loads.  Otherwise the compact layout's TriRecBox: its
// first three 16-byte words hold what TriRec holds, the fourth (with the .w
// of the second and third) the triangle's padded box, returned in lo/hi.
template <bool kBuf>
__device__ __forceinline__ TriRec leaf_tri(const SceneView& S, int j, vec3& lo, vec3& hi)
{
    if constexpr (kBuf) {
        const __amdgpu_buffer_rsrc_t R = buffer_of(S.tris, S.n_tris * (uint32_t)sizeof(TriRec));
        const uint32_t off = (uint32_t)j * (uint32_t)sizeof(TriRec);
        return tri_of(buffer_f4(R, off), buffer_f4(R, off + 16u), buffer_f4(R, off + 32u));
    } else {
        const float4* p = reinterpret_cast<const float4*>(S.tris) + 4 * (size_t)j;
        const float4 a = p[0], b = p[1], c = p[2], d = p[3];
        lo = v3(b.w, c.w, d.x);
        hi = v3(d.y, d.z, d.w);
        return tri_of(a, b, c);
    }
}

__device__ __forceinline__ float half_lo(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)); }
__device__ __forceinline__ float half_hi(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)); }

// Entry and exit of a CompactNode child box whose axes are the (lo, hi) FP16
// pairs wx, wy, wz.  Rotating a pair by 16 bits where the ray's direction is
// negative puts that axis's entry plane in the low half: a correctly rounded
// fma is monotone in its first argument, so the planes come out already
// ordered, the same values the min/max of the two planes give (slab), with
// no ordering instructions.
__device__ __forceinline__ void slab_h(const Ray& r, uint32_t wx, uint32_t wy, uint32_t wz, float& tn, float& tf)
{
    wx = __builtin_rotateright32(wx, r.rx);
    wy = __builtin_rotateright32(wy, r.ry);
    wz = __builtin_rotateright32(wz, r.rz);
    const float nx = fmaf(half_lo(wx), r.inv.x, -r.oi.x), fx = fmaf(half_hi(wx), r.inv.x, -r.oi.x);
    const float ny = fmaf(half_lo(wy), r.inv.y, -r.oi.y), fy = fmaf(half_hi(wy), r.inv.y, -r.oi.y);
    const float nz = fmaf(half_lo(wz), r.inv.z, -r.oi.z), fz = fmaf(half_hi(wz), r.inv.z, -r.oi.z);
    tn = fmaxf(fmaxf(nx, ny), nz);
    tf = fminf(fminf(fx, fy), fz);
}

// The internal node n: entry and exit of both child boxes, and the links.
// kBuf: the 64-byte BvhNode by buffer loads; otherwise the 32-byte
// CompactNode.
template <bool kBuf>
__device__ __forceinline__ void node_boxes(const SceneView& S, const Ray& r, int n, float& tn0, float& tf0,
                                           float& tn1, float& tf1, int& c0, int& c1)
{
    if constexpr (kBuf) {
        const __amdgpu_buffer_rsrc_t R = buffer_of(S.nodes, S.n_tris * 64u);
        const uint32_t off = (uint32_t)n << 6;
        const float4 a = buffer_f4(R, off), b = buffer_f4(R, off + 16u), d = buffer_f4(R, off + 32u),
                     l = buffer_f4(R, off + 48u);
        slab(r, a.x, a.y, a.z, a.w, b.x, b.y, tn0, tf0);
        slab(r, b.z, b.w, d.x, d.y, d.z, d.w, tn1, tf1);
        c0 = __float_as_int(l.x);
        c1 = __float_as_int(l.y);
    } else {
        const uint4* q = reinterpret_cast<const uint4*>(S.nodes) + 2 * (size_t)n;
        const uint4 q0 = q[0], q1 = q[1];
        slab_h(r, q0.x, q0.y, q0.z, tn0, tf0);
        slab_h(r, q0.w, q1.x, q1.y, tn1, tf1);
        c0 = (int)q1.z;
        c1 = (int)q1.w;
    }
}

// a hit triangle's record (v0, edges, caller index), either layout
__device__ __forceinline__ TriRec load_tri(const SceneView& S, int j)
{
    const float4* p = reinterpret_cast<const float4*>(S.tris) + (size_t)j * (S.compact ? 4u : 3u);
    return tri_of(p[0], p[1], p[2]);
}

struct Hit {
    float t;
    int prim;    // caller index, -1 = miss
    int sorted;  // BVH-order index
};

// Work counters of the profiling build (compiled out otherwise): node
// visits, triangle tests, closest-hit rays, shadow rays, scattering
// vertices, Philox draws, contributions (per lane), then wave executions of
// node visits, triangle tests and vertices (once per wave, by its first
// active lane).  Same order as TRHIP_COUNT_*.
enum {
    kTallyNodes,
    kTallyTris,
    kTallyRays,
    kTallyShadow,
    kTallyVerts,
    kTallyDraws,
    kTallyContrib,
    kTallyWaveNodes,
    kTallyWaveTris,
    kTallyWaveVerts,
    kTallyN
};
static_assert(kTallyN == kWorkCounters, "one tally per work counter");

// Build of a kernel: plain, counting (the work counters above), or
// recording (every next-event contribution of the pixels marked in the
// launch's record mask appended to its record buffer, to compare bins and
// values one by one with the oracle).
enum { kPlain = 0, kCounting = 1, kRecording = 2 };

template <int kMode>
struct Tally {
    __device__ __forceinline__ void add(int, uint32_t = 1u) {}
    __device__ __forceinline__ void wave(int) {}
    __device__ __forceinline__ void flush(unsigned long long*) {}
    __device__ __forceinline__ void record(const LaunchArgs&, uint32_t, uint32_t, int, int, float, int, float) {}
};
template <>
struct Tally<kRecording> {
    __device__ __forceinline__ void add(int, uint32_t = 1u) {}
    __device__ __forceinline__ void wave(int) {}
    __device__ __forceinline__ void flush(unsigned long long*) {}
    __device__ __forceinline__ void record(const LaunchArgs& L, uint32_t pix, uint32_t sample, int v, int k, float c,
                                           int bin, float tof)
    {
        if (!L.record_mask[pix]) return;
        const unsigned long long i = atomicAdd(L.record_count, 1ull);
        if (i >= L.record_cap) return;
        uint4* dst = reinterpret_cast<uint4*>(L.records + i);
        dst[0] = make_uint4(pix, sample, (uint32_t)v, (uint32_t)bin);
        dst[1] = make_uint4(__float_as_uint(c), __float_as_uint(tof), (uint32_t)k, 0u);
    }
};
template <>
struct Tally<kCounting> {
    uint32_t n[kTallyN] = {};
    __device__ __forceinline__ void add(int i, uint32_t v = 1u) { n[i] += v; }
    __device__ __forceinline__ void wave(int i)
    {
        const uint64_t active = __builtin_amdgcn_read_exec();
        if (__lane_id() == (uint32_t)__builtin_ctzll(active)) n[i] += 1u;
    }
    __device__ __forceinline__ void flush(unsigned long long* out)
    {
        for (int i = 0; i < kTallyN; ++i) atomicAdd(out + i, (unsigned long long)n[i]);
    }
    __device__ __forceinline__ void record(const LaunchArgs&, uint32_t, uint32_t, int, int, float, int, float) {}
};

// A BVH link read back from a traversal stack: 32-bit words hold it as is,
// 16-bit words (scenes of at most 32,768 triangles, where every internal
// node index and every ~triangle index fits in an int16) are sign-extended.
__device__ __forceinline__ int link_of(uint32_t w) { return (int)w; }
__device__ __forceinline__ int link_of(uint16_t w) { return (int)(int16_t)w; }

// A lane's traversal stack: one BVH link per level, word i at p[i * stride]
// in LDS (a 24-bit product: a full-rate multiply, where a 32-bit one takes
// four passes).  16-bit words also select buffer loads for nodes and
// triangles (their offsets fit in 32 bits).
template <class W>
struct LdsStack {
    static constexpr bool kBuf = sizeof(W) == 2;
    W* p;
    int stride;
    __device__ __forceinline__ int cap(const SceneView& S) const { return (int)S.stack_depth; }
    __device__ __forceinline__ void put(int sp, int link) { p[__umul24((uint32_t)sp, (uint32_t)stride)] = (W)link; }
    __device__ __forceinline__ int get(int sp) const { return link_of(p[__umul24((uint32_t)sp, (uint32_t)stride)]); }
};

// The first kLds words in LDS, the deeper ones in a per-lane array in
// scratch memory.  A traversal's stack stays far below the tree's depth (the
// far children pending at one time), so the deep words are rarely touched,
// while the LDS a wave holds shrinks and more waves fit on a CU.  For trees
// of at most kLds + kDeep levels; cap() keeps every access inside both parts
// for any tree.
template <int kLds, int kDeep>
struct SplitStack {
    static constexpr bool kBuf = false;
    // The LDS part carries its address space in its type, so that the two
    // parts are never read through one generic (flat) pointer.
    __attribute__((address_space(3))) uint32_t* p;
    int stride;
    int* deep;  // kDeep words, a local array of the kernel (scratch)
    __device__ __forceinline__ int cap(const SceneView& S) const { return min((int)S.stack_depth, kLds + kDeep); }
    __device__ __forceinline__ void put(int sp, int link)
    {
        if (sp < kLds)
            p[__umul24((uint32_t)sp, (uint32_t)stride)] = (uint32_t)link;
        else
            deep[sp - kLds] = link;
    }
    __device__ __forceinline__ int get(int sp) const
    {
        return sp < kLds ? (int)p[__umul24((uint32_t)sp, (uint32_t)stride)] : deep[sp - kLds];
    }
};

// Closest accepted triangle: smallest t, then smallest caller index.  A
// triangle is accepted at t only if its padded box's slab interval is
// non-empty and reaches t >= 0 and t is not before the box's entry, which
// makes the result independent of the traversal order.  With 16-bit links
// the padded box is the one stored for the triangle in its parent, tested
// there (tn: its entry); in the compact layout the parent's FP16 box only
// admitted the triangle, and the padded box comes with the record.
template <bool kBuf, class TallyT>
__device__ __forceinline__ void leaf_closest(const SceneView& S, const Ray& r, int sorted, float tn, int exclude,
                                             Hit& h, TallyT& tally)
{
    tally.add(kTallyTris);
    tally.wave(kTallyWaveTris);
    vec3 lo, hi;
    const TriRec tr = leaf_tri<kBuf>(S, sorted, lo, hi);
    if constexpr (!kBuf) {
        float tf;
        slab(r, lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, tn, tf);
        if (!(tn <= tf && tf >= 0.0f && tn <= h.t)) return;
    }
    const int prim = (int)tr.prim;
    float t;
    if (!intersect_tri<kBuf>(r, tr, exclude, t) || tn > t) return;
    if (t < h.t || (t == h.t && prim < h.prim)) {
        h.t = t;
        h.prim = prim;
        h.sorted = sorted;
    }
}

// Closest-hit traversal as a resumable state machine: the state between
// two internal-node visits.
struct ClosestTrav {
    Hit h;
    int node;         // next internal node
    int sp;           // stack entries in use
    uint32_t visits;  // a tree visits each internal node at most once per ray
};

template <class TallyT>
__device__ __forceinline__ void closest_begin(const SceneView& S, const Ray& r, int exclude, ClosestTrav& c,
                                              TallyT& tally)
{
    tally.add(kTallyRays);
    c.h.t = __builtin_huge_valf();
    c.h.prim = -1;
    c.h.sorted = -1;
    c.node = S.root;
    c.sp = 0;
    c.visits = 0;
    if (S.root < 0) {  // a single triangle: no internal node to visit
        float tn, tf;
        slab(r, S.root_lo[0], S.root_lo[1], S.root_lo[2], S.root_hi[0], S.root_hi[1], S.root_hi[2], tn, tf);
        if (tn <= tf && tf >= 0.0f) leaf_closest<true>(S, r, ~S.root, tn, exclude, c.h, tally);
        c.visits = S.n_tris;
    }
}

// Visits one internal node; returns true once the traversal has finished.
template <class St, class TallyT>
__device__ __forceinline__ bool closest_step(const SceneView& S, const Ray& r, int exclude, St& stk,
                                             ClosestTrav& c, TallyT& tally)
{
    if (c.visits >= S.n_tris) return true;
    ++c.visits;
    tally.add(kTallyNodes);
    tally.wave(kTallyWaveNodes);
    constexpr bool kBuf = St::kBuf;
    float tn0, tf0, tn1, tf1;
    int c0, c1;
    node_boxes<kBuf>(S, r, c.node, tn0, tf0, tn1, tf1, c0, c1);
    bool h0 = tn0 <= tf0 && tf0 >= 0.0f && tn0 <= c.h.t;
    bool h1 = tn1 <= tf1 && tf1 >= 0.0f && tn1 <= c.h.t;
    // Leaf children: each lane tests its first pending leaf, then its
    // second, so that lanes whose leaves hang in different children share
    // one pass of the test instead of taking one each.  The closest hit
    // does not depend on the order of the tests.
    bool l0 = h0 && c0 < 0, l1 = h1 && c1 < 0;
    h0 = h0 && c0 >= 0;
    h1 = h1 && c1 >= 0;
    while (l0 || l1) {
        const bool first = l0;
        leaf_closest<kBuf>(S, r, first ? ~c0 : ~c1, first ? tn0 : tn1, exclude, c.h, tally);
        l1 = l1 && first;  // the second leaf stays pending only after the first
        l0 = false;
    }
    h0 = h0 && tn0 <= c.h.t;
    h1 = h1 && tn1 <= c.h.t;
    if (h0 && h1 && c.sp < stk.cap(S)) {
        const bool first0 = tn0 <= tn1;
        stk.put(c.sp, first0 ? c1 : c0);
        ++c.sp;
        c.node = first0 ? c0 : c1;
    } else if (h0) {
        c.node = c0;
    } else if (h1) {
        c.node = c1;
    } else {
        if (c.sp == 0) return true;
        --c.sp;
        c.node = stk.get(c.sp);
    }
    return false;
}

template <class St, class TallyT>
__device__ Hit closest_hit(const SceneView& S, const Ray& r, int exclude, St& stk, TallyT& tally)
{
    ClosestTrav c;
    closest_begin(S, r, exclude, c, tally);
    while (!closest_step(S, r, exclude, stk, c, tally)) {
    }
    return c.h;
}

template <bool kBuf, class TallyT>
__device__ __forceinline__ bool leaf_blocks(const SceneView& S, const Ray& r, int sorted, float tn, int exclude,
                                            float tmax, TallyT& tally)
{
    tally.add(kTallyTris);
    tally.wave(kTallyWaveTris);
    vec3 lo, hi;
    const TriRec tr = leaf_tri<kBuf>(S, sorted, lo, hi);
    if constexpr (!kBuf) {
        float tf;
        slab(r, lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, tn, tf);
        if (!(tn <= tf && tf >= 0.0f && tn <= tmax)) return false;
    }
    float t;
    return intersect_tri<kBuf>(r, tr, exclude, t) && !(tn > t) && t < tmax;
}

// any accepted triangle other than `exclude` with t < tmax
template <class St, class TallyT>
__device__ bool occluded(const SceneView& S, const Ray& r, int exclude, float tmax, St& stk, TallyT& tally)
{
    tally.add(kTallyShadow);
    if (S.root < 0) {
        float tn, tf;
        slab(r, S.root_lo[0], S.root_lo[1], S.root_lo[2], S.root_hi[0], S.root_hi[1], S.root_hi[2], tn, tf);
        return tn <= tf && tf >= 0.0f && tn <= tmax && leaf_blocks<true>(S, r, ~S.root, tn, exclude, tmax, tally);
    }
    int node = S.root;
    int sp = 0;
    constexpr bool kBuf = St::kBuf;
    const int max_sp = stk.cap(S);
    for (uint32_t visits = 0; visits < S.n_tris; ++visits) {
        float tn0, tf0, tn1, tf1;
        int c0, c1;
        node_boxes<kBuf>(S, r, node, tn0, tf0, tn1, tf1, c0, c1);
        tally.add(kTallyNodes);
        tally.wave(kTallyWaveNodes);
        bool h0 = tn0 <= tf0 && tf0 >= 0.0f && tn0 <= tmax;
        bool h1 = tn1 <= tf1 && tf1 >= 0.0f && tn1 <= tmax;
        // leaf children, one pass per pending leaf shared by the wave's
        // lanes (as in closest_step)
        bool l0 = h0 && c0 < 0, l1 = h1 && c1 < 0;
        h0 = h0 && c0 >= 0;
        h1 = h1 && c1 >= 0;
        while (l0 || l1) {
            const bool first = l0;
            if (leaf_blocks<kBuf>(S, r, first ? ~c0 : ~c1, first ? tn0 : tn1, exclude, tmax, tally)) return true;
            l1 = l1 && first;
            l0 = false;
        }
        if (h0 && h1 && sp < max_sp) {
            // large scenes (compact layout): the nearer child first
            // (1M-triangle scene: 1.5 % fewer wave node steps, +1.8 %);
            // small ones: child 0 first (box and glass rooms: 3-5 % faster
            // so).  An any-hit result does not depend on the order.
            const bool first0 = kBuf || tn0 <= tn1;
            stk.put(sp, first0 ? c1 : c0);
            ++sp;
            node = first0 ? c0 : c1;
        } else if (h0) {
            node = c0;
        } else if (h1) {
            node = c1;
        } else {
            if (sp == 0) return false;
            --sp;
            node = stk.get(sp);
        }
    }
    return false;
}

__device__ __forceinline__ vec3 ld3(const float* p) { return v3(p[0], p[1], p[2]); }

constexpr float kShadowShrink = 1.0f - 0x1p-10f;

// State of one path between two closest-hit queries.
struct PathState {
    vec3 o, d;     // next ray
    float beta;    // throughput
    float opl;     // optical path length so far
    float u_ff;    // uniform of the next free flight
    float eta;     // index of the medium the ray runs in; negative: inside a dielectric mesh
    int prev;      // caller index of the triangle the ray leaves (-1: none)
    int v;         // index of the vertex the next ray creates (1-based)
};

// A next-event connection waiting for its shadow ray.
struct Nee {
    vec3 so, sd;   // shadow ray
    float tmax;
    int excl;      // triangle excluded from the shadow test
    float c;       // contribution if unoccluded
    int bin;       // -1: outside the film window
    float tof;     // optical path length of the connected path
    int k;         // triangle of the vertex (-1: medium vertex)
    float g_alb, g_rough;  // d log f of the connection
    bool valid;
};

// Outcome of the continuation at a vertex.
struct Cont {
    bool alive;    // the path continues with ps.o, ps.d
    int k;         // triangle of the vertex (-1: medium)
    float g_alb, g_rough;  // d log f of the sampled direction (surface only)
};

__device__ __forceinline__ int last_vertex(const SceneView& S, const LaunchArgs& L)
{
    return (S.sensor == 1) ? (int)L.max_depth - 3 : (int)L.max_depth - 1;
}

// Generation (Philox block 0): the camera ray through the jittered pixel, or
// for the confocal sensor the cosine-sampled ray leaving the scan point of
// the relay wall (a Lambertian vertex whose sampling weight is its albedo).
__device__ __forceinline__ void begin_path(const SceneView& S, const LaunchArgs& L, uint32_t pix, uint32_t sample,
                                           PathState& ps)
{
    const rand4 u = draw4(pix, sample, 0u, L.stream_id, L.key0, L.key1);
    ps.u_ff = u.u2;
    if (S.sensor != 1) {
        const uint32_t ix = pix % S.width, iy = pix / S.width;
        const bool centre = (L.flags & kFlagPixelCentre) != 0;
        const float jx = centre ? 0.5f : u.u0, jy = centre ? 0.5f : u.u1;
        const float fx = (float)ix + jx, fy = (float)iy + jy;
        const float sx = ((fx * 2.0f) / (float)S.width - 1.0f) * S.tan_x;
        const float sy = (1.0f - (fy * 2.0f) / (float)S.height) * S.tan_y;
        ps.d = normalize(v3(fmaf(S.cam_u[0], sy, fmaf(S.cam_r[0], sx, S.cam_f[0])),
                            fmaf(S.cam_u[1], sy, fmaf(S.cam_r[1], sx, S.cam_f[1])),
                            fmaf(S.cam_u[2], sy, fmaf(S.cam_r[2], sx, S.cam_f[2]))));
        ps.o = ld3(S.cam_o);
        ps.beta = 1.0f;
    } else {
        const vec3 wall_n = ld3(S.wall_n);
        const vec3 xs = ld3(S.scan + 3ull * pix);
        vec3 t, b;
        basis(wall_n, t, b);
        ps.d = local_to_world(t, b, wall_n, cosine_dir(u.u0, u.u1));
        ps.o = nudge(xs, wall_n);
        ps.beta = S.wall_albedo;
    }
    ps.opl = 0.0f;
    ps.eta = S.eta0;
    ps.prev = -1;
    ps.v = 1;
}

// caller index of the area-sampled triangle for scan region r: the first
// whose prefix sum exceeds u0 * W_r, found by bisection between two
// guide-table entries (the cutpoint method).  With m = floor(u0 * M),
// m / M <= u0 < (m + 1) / M exactly, and FP64 rounding is monotone, so the
// thresholds of entries m and m + 1 bracket u0 * W_r and their first indices
// bracket the answer.  u0 is a multiple of 2^-24 and M a power of two
// <= 2^20: u0 * M is exact.
__device__ __forceinline__ uint32_t area_pick(const SceneView& S, uint32_t r, float u0)
{
    const double* cdf = S.area_cdf + (size_t)r * S.n_tris;
    const uint32_t* guide = S.area_guide + (size_t)r * ((uint32_t)S.guide_cells + 1u);
    const double target = (double)u0 * S.area_wtotal[r];
    const uint32_t m = (uint32_t)(u0 * S.guide_cells);
    uint32_t lo = guide[m], hi = guide[m + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cdf[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// NLOS area sampling (confocal; the NLOS-tailored sampling of Sec. 4.5):
// generation draws the hidden vertex itself -- triangle k of the sampling
// set (the triangles off the relay wall's plane) with probability w_k / W_r
// through the FP64 prefix sums of the weights of the scan point's region r
// (u0), the point uniformly within it by the square-root warp (u1, u2) --
// and joins it to the offset scan point.  The area density w_k / (W_r A_k)
// converted to solid angle at the scan point (times r^2 / cos_hidden) gives
// the weight f_wall cos_wall / p = wall_albedo / pi * (W_r A_k / w_k) *
// cos_wall cos_hidden / r^2.  The segment's visibility is left to the next-event
// shadow ray of the vertex, which tests the same segment back to the scan
// point.  Returns false when the pair faces away (no contribution);
// otherwise sets ps and the vertex's hit h (distance r, caller and
// BVH-order triangle).
__device__ __forceinline__ bool begin_area(const SceneView& S, const LaunchArgs& L, uint32_t pix, uint32_t sample,
                                           PathState& ps, Hit& h)
{
    const rand4 u = draw4(pix, sample, 0u, L.stream_id, L.key0, L.key1);
    ps.u_ff = u.u2;
    const uint32_t region = S.area_region[pix];
    const uint32_t lo = area_pick(S, region, u.u0);
    const uint32_t j = S.sorted_of[lo];
    const TriRec tr = load_tri(S, (int)j);
    const vec3 e1 = v3(tr.e1x, tr.e1y, tr.e1z), e2 = v3(tr.e2x, tr.e2y, tr.e2z);
    const float su = sqrtf(u.u1);
    const float b1 = su * (1.0f - u.u2), b2 = su * u.u2;
    const vec3 x = v3(fmaf(b1, e1.x, fmaf(b2, e2.x, tr.v0x)), fmaf(b1, e1.y, fmaf(b2, e2.y, tr.v0y)),
                      fmaf(b1, e1.z, fmaf(b2, e2.z, tr.v0z)));
    const vec3 wall_n = ld3(S.wall_n);
    const vec3 o = nudge(ld3(S.scan + 3ull * pix), wall_n);
    const vec3 dv = sub(x, o);
    const float r2 = dot(dv, dv);
    const float r = sqrtf(r2);
    const vec3 d = scale(dv, 1.0f / r);
    const vec3 ng = normalize(cross(e1, e2));
    const float cos_s = dot(wall_n, d);
    const float cos_h = fabsf(dot(ng, d));
    if (!(cos_s > 0.0f) || !(cos_h > 0.0f)) return false;
    const float g = (cos_s * cos_h) / r2;
    ps.beta = ((S.wall_albedo * S.area_invp[(size_t)region * S.n_tris + lo]) * kInvPi) * g;
    ps.o = o;
    ps.d = d;
    ps.opl = 0.0f;
    ps.eta = S.eta0;
    ps.prev = -1;
    ps.v = 1;
    h.t = r;
    h.prim = (int)lo;
    h.sorted = (int)j;
    return true;
}

// Free flight in the medium against the surface hit: returns whether a
// vertex exists and sets its distance and kind.
__device__ __forceinline__ bool resolve_event(const SceneView& S, const PathState& ps, const Hit& h, float& t_hit,
                                              bool& med)
{
    const bool hit = h.prim >= 0;
    t_hit = h.t;
    med = false;
    if (S.sigma_t > 0.0f && ps.eta > 0.0f) {  // the medium fills the space around the meshes
        const float t_ff = -log_one_minus(ps.u_ff) / S.sigma_t;
        if (!hit || t_ff < t_hit) {
            med = true;
            t_hit = t_ff;
        }
    }
    return hit || med;
}

// Smooth dielectric interface (Eq. 3 with an index per medium): the mesh of
// triangle k has index S.ior[k] inside, the side against its winding normal
// ng = e1 x e2, and the surrounding space S.eta0 outside.  Reflection with
// the unpolarised Fresnel reflectance F (1 beyond the critical angle), else
// refraction by Snell's law, each with its own probability (u0 decides);
// radiance over eta^2 is what crosses the interface (times 1 - F), so a
// refraction weighs (eta_i / eta_t)^2 and a reflection 1.  Updates the
// direction, offset origin, throughput and the medium of ps.
__device__ __forceinline__ void dielectric_event(const SceneView& S, int k, const vec3& x, const vec3& ng,
                                                 const vec3& n, const vec3& wo, float u0, PathState& ps)
{
    const bool entering = !(dot(ng, wo) < 0.0f);
    const float ci = dot(n, wo);
    const float eta_k = S.ior[k];
    const float eta_i = entering ? S.eta0 : eta_k, eta_t = entering ? eta_k : S.eta0;
    const float eta_r = eta_i / eta_t;
    const float st2 = (eta_r * eta_r) * (1.0f - ci * ci);
    float F = 1.0f, ct = 0.0f;
    if (st2 < 1.0f) {
        ct = sqrtf(1.0f - st2);
        const float rs = (eta_i * ci - eta_t * ct) / (eta_i * ci + eta_t * ct);
        const float rp = (eta_t * ci - eta_i * ct) / (eta_t * ci + eta_i * ct);
        F = 0.5f * (rs * rs + rp * rp);
    }
    if (u0 < F) {
        ps.d = normalize(sub(scale(n, 2.0f * ci), wo));
        ps.o = nudge(x, n);
        ps.eta = entering ? eta_i : -eta_i;
    } else {
        ps.d = normalize(add(scale(wo, -eta_r), scale(n, eta_r * ci - ct)));
        ps.o = nudge(x, neg(n));
        ps.beta = ps.beta * (eta_r * eta_r);
        ps.eta = entering ? -eta_t : eta_t;
    }
}

// Everything at one vertex except the two traversals: the next-event
// connection (value, bin, shadow ray) and the continuation (Philox block v),
// which updates ps in place.
template <bool kGrad, class TallyT>
__device__ __forceinline__ void shade_vertex(const SceneView& S, const LaunchArgs& L, uint32_t pix, uint32_t sample,
                                             PathState& ps, const Hit& h, float t_hit, bool med, Nee& nee,
                                             Cont& cont, TallyT& tally)
{
    const bool confocal = S.sensor == 1;
    const bool medium = S.sigma_t > 0.0f;
    const int vmax = last_vertex(S, L);
    const int v = ps.v;
    tally.add(kTallyVerts);
    tally.wave(kTallyWaveVerts);
    nee.valid = false;
    cont.alive = false;
    cont.k = med ? -1 : h.prim;
    cont.g_alb = 0.0f;
    cont.g_rough = 0.0f;
    const vec3 target = confocal ? ld3(S.scan + 3ull * pix) : ld3(S.light);
    const vec3 x = along(ps.o, ps.d, t_hit);
    // Eq. 3: a segment's time of flight is its length times the index
    const float eta = fabsf(ps.eta);
    const bool outside = ps.eta > 0.0f;
    if (!(S.unwarp && !confocal && v == 1)) ps.opl = ps.opl + t_hit * eta;
    const vec3 wo = neg(ps.d);
    const vec3 dl = sub(target, x);
    const float d2 = dot(dl, dl);
    const float dist = sqrtf(d2);
    const vec3 wl = scale(dl, 1.0f / dist);
    float em;
    if (confocal) {
        const float cos_s = -dot(ld3(S.wall_n), wl);
        em = (cos_s > 0.0f) ? ((S.wall_albedo * S.laser_power) * kInvPi) * cos_s : 0.0f;
    } else {
        em = S.intensity;
    }
    nee.sd = wl;
    nee.tmax = dist * kShadowShrink;
    // time of the connected path and its bin (after this vertex's delay)
    auto bin_of = [&]() {
        const float opl_c = ps.opl + dist * eta;
        const float q = (opl_c - S.bin_start) / S.bin_width;
        nee.bin = (q >= 0.0f && q < (float)S.n_bins) ? (int)q : -1;
        nee.tof = opl_c;
    };
    if (med) {
        bin_of();
        ps.beta = ps.beta * S.medium_albedo;
        if (em > 0.0f) {
            float c = ((ps.beta * kInv4Pi) * em) / d2;
            c = c * expf(-(S.sigma_t * dist));
            nee.valid = true;
            nee.so = x;
            nee.excl = -1;
            nee.c = c;
            nee.k = -1;
            nee.g_alb = 0.0f;
            nee.g_rough = 0.0f;
        }
        if (v == vmax) return;
        tally.add(kTallyDraws);
        const rand4 u = draw4(pix, sample, (uint32_t)v, L.stream_id, L.key0, L.key1);
        const float z = 1.0f - (u.u0 + u.u0);
        const float rr = sqrtf(fmaxf(0.0f, 1.0f - z * z));
        float sn, cs;
        sincos_2pi(u.u1, sn, cs);
        ps.d = v3(rr * cs, rr * sn, z);
        ps.o = x;
        ps.prev = -1;
        ps.u_ff = u.u3;
        ps.v = v + 1;
        cont.alive = true;
        return;
    }
    // surface vertex: two-sided, shading normal = geometric normal flipped
    // toward wo
    const TriRec tr = load_tri(S, h.sorted);
    const vec3 ng = normalize(cross(v3(tr.e1x, tr.e1y, tr.e1z), v3(tr.e2x, tr.e2y, tr.e2z)));
    const vec3 n = (dot(ng, wo) < 0.0f) ? neg(ng) : ng;
    if (!(dot(n, wo) > 0.0f)) return;
    const int k = h.prim;
    nee.so = nudge(x, n);
    nee.excl = k;
    // Eq. 10: a scattering delay, exponential with the triangle's mean, from
    // word 2 of the vertex's Philox block; it delays this vertex's
    // contribution and every later one
    rand4 u;
    bool have_u = false;
    if (S.delay) {
        const float tau = S.delay[k];
        if (tau > 0.0f) {
            tally.add(kTallyDraws);
            u = draw4(pix, sample, (uint32_t)v, L.stream_id, L.key0, L.key1);
            have_u = true;
            ps.opl = ps.opl + tau * -log_one_minus(u.u2);
        }
    }
    bin_of();
    const uint32_t mat = S.mat[k];
    if (mat == kMatDielectric) {
        // a delta interface: no next-event connection, no gradient factor
        if (v == vmax) return;
        if (!have_u) {
            tally.add(kTallyDraws);
            u = draw4(pix, sample, (uint32_t)v, L.stream_id, L.key0, L.key1);
        }
        dielectric_event(S, k, x, ng, n, wo, u.u0, ps);
        cont.alive = true;
        ps.prev = k;
        ps.u_ff = u.u3;
        ps.v = v + 1;
        return;
    }
    const bool ggx = mat == 1;
    const float albedo = L.albedo[k];
    vec3 tb, bb;
    basis(n, tb, bb);
    const vec3 wol = v3(dot(wo, tb), dot(wo, bb), dot(wo, n));
    float fcos = 0.0f, g_rough = 0.0f;
    {
        const float cos_l = dot(n, wl);
        if (cos_l > 0.0f) {
            if (ggx) {
                const float alpha = L.rough_eval[k];
                const vec3 wll = v3(dot(wl, tb), dot(wl, bb), dot(wl, n));
                const float f = ggx_eval(wol, wll, alpha, albedo);
                if (f > 0.0f) {
                    fcos = f * wll.z;
                    if (kGrad) g_rough = ggx_dlog_dalpha(wol, wll, alpha);
                }
            } else {
                fcos = (albedo * kInvPi) * cos_l;
            }
        }
    }
    if (fcos > 0.0f && em > 0.0f) {
        float c = ((ps.beta * fcos) * em) / d2;
        if (medium && outside) c = c * expf(-(S.sigma_t * dist));
        nee.valid = true;
        nee.c = c;
        nee.k = k;
        nee.g_alb = 1.0f / albedo;
        nee.g_rough = g_rough;
    }
    if (v == vmax) return;
    if (!have_u) {
        tally.add(kTallyDraws);
        u = draw4(pix, sample, (uint32_t)v, L.stream_id, L.key0, L.key1);
    }
    vec3 wi;
    float w;
    float gc_rough = 0.0f;
    if (ggx) {
        const float alpha = L.rough_eval[k];
        const float alpha_s = L.rough_sample[k];
        if (!(wol.z > 0.0f)) return;
        const vec3 wil = ggx_vndf_sample(wol, alpha_s, u.u0, u.u1);
        if (!(wil.z > 0.0f)) return;
        if (L.flags & kFlagFrozen) {
            const float pdf = ggx_vndf_pdf(wol, wil, alpha_s);
            const float f = ggx_eval(wol, wil, alpha, albedo);
            if (!(pdf > 0.0f)) return;
            w = (f * wil.z) / pdf;
        } else {
            const float a2 = alpha * alpha;
            const float lo = smith_lambda(wol, a2), li = smith_lambda(wil, a2);
            w = albedo * ((1.0f + lo) / ((1.0f + lo) + li));
        }
        if (!(w > 0.0f)) return;
        if (kGrad) gc_rough = ggx_dlog_dalpha(wol, wil, alpha);
        wi = local_to_world(tb, bb, n, wil);
    } else {
        wi = local_to_world(tb, bb, n, cosine_dir(u.u0, u.u1));
        w = albedo;
    }
    cont.alive = true;
    cont.g_alb = 1.0f / albedo;
    cont.g_rough = gc_rough;
    ps.beta = ps.beta * w;
    ps.d = wi;
    ps.o = nudge(x, n);
    ps.prev = k;
    ps.u_ff = u.u3;
    ps.v = v + 1;
}

// Continues a path whose next closest hit h is known, and reports through
// the sink every next-event contribution (vertex index, triangle, value,
// bin, d log f factors of the connection) and every continuation (triangle,
// d log f factors of the sampled direction).  Triangles are caller indices;
// -1 marks a medium vertex.
template <class Sink, class St, class TallyT>
__device__ void continue_path(const SceneView& S, const LaunchArgs& L, uint32_t pix, uint32_t sample, PathState& ps,
                              Hit h, St& stk, Sink& sink, TallyT& tally)
{
    const int vmax = last_vertex(S, L);
    while (true) {
        const int v = ps.v;
        float t_hit;
        bool med;
        if (!resolve_event(S, ps, h, t_hit, med)) break;
        Nee nee;
        Cont cont;
        shade_vertex<Sink::kWantsGradients>(S, L, pix, sample, ps, h, t_hit, med, nee, cont, tally);
        // A path drawn by NLOS area sampling continues from its hidden vertex
        // only if the first segment is unoccluded: the shadow test back to
        // the scan point runs along it, so a lane needs that test for its
        // contribution, its continuation or both.  One call serves both, so
        // the lanes of a wave share one traversal.
        const bool area_first = v == 1 && (L.flags & kFlagNlosArea) && cont.alive;
        bool blocked = true;
        if (nee.valid || area_first) blocked = occluded(S, make_ray(nee.so, nee.sd), nee.excl, nee.tmax, stk, tally);
        if (nee.valid && !blocked) {
            tally.add(kTallyContrib);
            tally.record(L, pix, sample, v, nee.k, nee.c, nee.bin, nee.tof);
            sink.contribution(v, nee.k, nee.c, nee.bin, nee.tof, nee.g_alb, nee.g_rough);
        }
        if (!cont.alive) break;
        if (area_first && blocked) break;
        if (cont.k >= 0) sink.continuation(v, cont.k, cont.g_alb, cont.g_rough);
        if (ps.v > vmax) break;
        h = closest_hit(S, make_ray(ps.o, ps.d), ps.prev, stk, tally);
    }
}

// Traces one whole path (Philox block 0 generation, then vertex by vertex).
template <class Sink, class St, class TallyT>
__device__ void trace_path(const SceneView& S, const LaunchArgs& L, uint32_t pix, uint32_t sample, St& stk,
                           Sink& sink, TallyT& tally)
{
    tally.add(kTallyDraws);
    PathState ps;
    if (L.flags & kFlagNlosArea) {
        Hit h;
        if (begin_area(S, L, pix, sample, ps, h)) continue_path(S, L, pix, sample, ps, h, stk, sink, tally);
        return;
    }
    begin_path(S, L, pix, sample, ps);
    if (last_vertex(S, L) < 1) return;
    const Hit h = closest_hit(S, make_ray(ps.o, ps.d), ps.prev, stk, tally);
    continue_path(S, L, pix, sample, ps, h, stk, sink, tally);
}

// ---------------------------------------------------------------------------
// forward render
// ---------------------------------------------------------------------------
// floats of one pixel's film: the time bins, or (re, im) per frequency
__device__ __forceinline__ uint32_t film_words(const SceneView& S, const LaunchArgs& L)
{
    return L.n_freq ? 2 * L.n_freq : S.n_bins;
}

// the frequencies of a phasor film into LDS (constant indices only, so
// the kernel argument array stays in registers / the argument segment)
__device__ __forceinline__ void load_freqs(const LaunchArgs& L, float* s_freq)
{
    if (threadIdx.x == 0) {
#pragma unroll
        for (uint32_t j = 0; j < kMaxFreq; ++j) s_freq[j] = L.freq[j];
    }
}

struct FilmSink {
    static constexpr bool kWantsGradients = false;
    float* row;     // LDS film row of the current pixel
    float steady;   // register partial sums of the current pixel
    float oow;
    const float* freq;  // LDS frequencies of a phasor film
    uint32_t n_freq;    // 0: time histogram
    __device__ __forceinline__ void contribution(int, int, float c, int bin, float tof, float, float)
    {
        if (n_freq) {
            // Sec. 4.3, Eq. 14: the contribution times exp(-2 pi i f tof);
            // the phase in cycles is reduced to [0, 1) exactly
            for (uint32_t j = 0; j < n_freq; ++j) {
                const float cyc = freq[j] * tof;
                float fr = cyc - floorf(cyc);
                if (fr >= 1.0f) fr = 0.0f;
                float sn, cs;
                sincos_2pi(fr, sn, cs);
                atomicAdd(row + 2 * j, c * cs);
                atomicAdd(row + 2 * j + 1, -(c * sn));
            }
        } else if (bin >= 0) {
            atomicAdd(row + bin, c);
        } else {
            oow += c;
        }
        steady += c;
    }
    __device__ __forceinline__ void continuation(int, int, float, float) {}
};

// ---------------------------------------------------------------------------
// Deterministic accumulation (TRHIP_FLAG_DETERMINISTIC).  Every film
// contribution and every gradient term is added as a 128-bit two's-complement
// fixed-point number with 64 fraction bits, held in two 64-bit words: the low
// words' atomic add returns the old value, and a wrap-around carries 1 into
// the high word.  Integer addition is associative and the number of
// wrap-arounds of the low word is fixed by the total, so the final sums do
// not depend on the order of the atomics, the launch shape or the kernel's
// scheduling.  A film bin is then the exact sum of its FP32 contributions
// (exact for contributions of at least 2^-41; smaller ones are truncated to
// multiples of 2^-64), rounded once; values and sums must stay below 2^63.
// ---------------------------------------------------------------------------
struct Fixed128 {
    uint64_t lo, hi;
};

// x * 2^64 truncated toward zero (saturated at |x| >= 2^63; NaN gives 0)
__device__ __forceinline__ Fixed128 to_fixed(double x)
{
    Fixed128 f{0ull, 0ull};
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const int e = (int)((b >> 52) & 0x7ffu);
    if (e == 0 || x != x) return f;
    const uint64_t m = (b & 0xfffffffffffffull) | 0x10000000000000ull;  // |x| = m 2^(e - 1075)
    const int s = e - 1075 + 64;                                          // |x| 2^64 = m 2^s
    if (s > 74) {
        f.lo = ~0ull;
        f.hi = 0x7fffffffffffffffull;
    } else if (s >= 64) {
        f.hi = m << (s - 64);
    } else if (s > 0) {
        f.lo = m << s;
        f.hi = m >> (64 - s);
    } else if (s > -53) {
        f.lo = m >> (-s);
    }
    if (b >> 63) {
        f.lo = ~f.lo + 1ull;
        f.hi = ~f.hi + (f.lo == 0ull ? 1ull : 0ull);
    }
    return f;
}

__device__ __forceinline__ double from_fixed(uint64_t lo, uint64_t hi)
{
    return (double)(int64_t)hi + (double)lo * 0x1p-64;
}

// cell[0], cell[1]: low and high word (LDS or global memory)
__device__ __forceinline__ void fixed_add(unsigned long long* cell, Fixed128 f)
{
    if ((f.lo | f.hi) == 0ull) return;
    const unsigned long long old = atomicAdd(cell, (unsigned long long)f.lo);
    const uint64_t h = f.hi + ((old + f.lo < old) ? 1ull : 0ull);
    if (h) atomicAdd(cell + 1, (unsigned long long)h);
}

struct FixedFilmSink {
    static constexpr bool kWantsGradients = false;
    unsigned long long* row;     // LDS film row of the pixel, two words per bin
    unsigned long long* steady;  // two words
    unsigned long long* oow;
    __device__ __forceinline__ void contribution(int, int, float c, int bin, float, float, float)
    {
        const Fixed128 f = to_fixed((double)c);
        if (bin >= 0) fixed_add(row + 2 * bin, f);
        else fixed_add(oow, f);
        fixed_add(steady, f);
    }
    __device__ __forceinline__ void continuation(int, int, float, float) {}
};

// The HBM fixed-point film: film and out-of-window sums by 64-bit atomics,
// the pixel's steady sum exact in a register pair (two's complement, the
// carry taken by hand) until the lane moves to another pixel.
// The HBM form's sums: three 64-bit words per sum, word k adding up the
// 43-bit limbs k (bits 43k and up) of the 128-bit values, so that every
// atomic is a plain add whose old value no lane waits for (the LDS form's
// carry needs it).  The value of one FP32 contribution has at most 24
// significant bits and so touches at most two limbs (three if negative).
// The words stay exact for fewer than 2^21 adds per sum, and the sum is the
// value of the words below, modulo 2^128: the same integer as the two-word
// form's.
constexpr uint32_t kLimbWords = 3;
constexpr uint64_t kLimbMask = (1ull << 43) - 1ull;

__device__ __forceinline__ void limb_add(unsigned long long* cell, Fixed128 f)
{
    const uint64_t l0 = f.lo & kLimbMask;
    const uint64_t l1 = (f.lo >> 43) | ((f.hi & ((1ull << 22) - 1ull)) << 21);
    const uint64_t l2 = f.hi >> 22;
    if (l0) atomicAdd(cell, (unsigned long long)l0);
    if (l1) atomicAdd(cell + 1, (unsigned long long)l1);
    if (l2) atomicAdd(cell + 2, (unsigned long long)l2);
}

// w0 + w1 2^43 + w2 2^86 modulo 2^128
__device__ __forceinline__ Fixed128 limb_value(uint64_t w0, uint64_t w1, uint64_t w2)
{
    Fixed128 f;
    const uint64_t t = w1 << 43;
    f.lo = w0 + t;
    f.hi = (f.lo < t ? 1ull : 0ull) + (w1 >> 21) + (w2 << 22);
    return f;
}

struct FixedHbmSink {
    static constexpr bool kWantsGradients = false;
    unsigned long long* row;  // HBM fixed-point film row of the pixel, kLimbWords words per bin
    unsigned long long* oow;  // kLimbWords words
    unsigned long long steady_lo, steady_hi;
    __device__ __forceinline__ void contribution(int, int, float c, int bin, float, float, float)
    {
        const Fixed128 f = to_fixed((double)c);
        if (bin >= 0) limb_add(row + kLimbWords * bin, f);
        else limb_add(oow, f);
        const unsigned long long lo = steady_lo + f.lo;
        steady_hi += f.hi + (lo < steady_lo ? 1ull : 0ull);
        steady_lo = lo;
    }
    __device__ __forceinline__ void continuation(int, int, float, float) {}
};

// Deterministic form of render_tile (path per lane): the tile's film,
// steady and out-of-window sums in fixed point in LDS ([TP][T][2], [TP][2],
// [TP][2] words), each written as sum / norm_spp rounded to FP32.
template <class St, class TallyT>
__device__ __forceinline__ void render_tile_fixed(const SceneView& S, const LaunchArgs& L, uint32_t p0,
                                                  unsigned long long* q, St& stk, TallyT& tally)
{
    const uint32_t T = S.n_bins;
    const uint32_t TP = L.tile_pixels;
    unsigned long long* qfilm = q;
    unsigned long long* qsteady = q + 2ull * TP * T;
    unsigned long long* qoow = qsteady + 2 * TP;
    const uint32_t npix = min(TP, L.n_pixels - p0);
    for (uint32_t i = threadIdx.x; i < 2 * (TP * T + 2 * TP); i += blockDim.x) q[i] = 0ull;
    __syncthreads();
    const uint32_t work = npix * L.spp;
    for (uint32_t w = threadIdx.x; w < work; w += blockDim.x) {
        const uint32_t pl = w / L.spp;
        const uint32_t s = w - pl * L.spp;
        FixedFilmSink sink{qfilm + 2ull * pl * T, qsteady + 2 * pl, qoow + 2 * pl};
        trace_path(S, L, p0 + pl, L.sample_offset + s, stk, sink, tally);
    }
    __syncthreads();
    const bool acc = (L.flags & kFlagAccumulate) != 0;
    const double n = (double)L.norm_spp;
    auto value = [&](const unsigned long long* c) { return (float)(from_fixed(c[0], c[1]) / n); };
    const size_t base = (size_t)p0 * T;
    for (uint32_t i = threadIdx.x; i < npix * T; i += blockDim.x) {
        const float v = value(qfilm + 2 * i);
        L.film[base + i] = acc ? L.film[base + i] + v : v;
    }
    if (threadIdx.x < npix) {
        const uint32_t p = p0 + threadIdx.x;
        if (L.steady) {
            const float v = value(qsteady + 2 * threadIdx.x);
            L.steady[p] = acc ? L.steady[p] + v : v;
        }
        if (L.oow) {
            const float v = value(qoow + 2 * threadIdx.x);
            L.oow[p] = acc ? L.oow[p] + v : v;
        }
    }
}

// Deterministic form with the film in HBM (long films of large scenes,
// where a fixed-point LDS row of 16 bytes per bin would leave few waves per
// CU): the fixed-point sums of the whole launch live in L.fixed_film
// (zeroed beforehand) as limb words (limb_add), and a second pass
// (k_fixed_film_out) rounds each once, as render_tile_fixed does.  For
// spp * max_depth < 2^21 (the adds one sum can receive).
template <class St, class TallyT>
__device__ __forceinline__ void render_tile_fixed_hbm(const SceneView& S, const LaunchArgs& L, uint32_t p0, St& stk,
                                                      TallyT& tally)
{
    const uint32_t T = S.n_bins;
    unsigned long long* qfilm = L.fixed_film;
    unsigned long long* qsteady = qfilm + (size_t)kLimbWords * L.n_pixels * T;
    unsigned long long* qoow = qsteady + (size_t)kLimbWords * L.n_pixels;
    const uint32_t npix = min(L.tile_pixels, L.n_pixels - p0);
    const uint32_t work = npix * L.spp;
    uint32_t cur = 0xffffffffu;
    FixedHbmSink sink{nullptr, nullptr, 0ull, 0ull};
    auto flush = [&]() {
        if (cur != 0xffffffffu)
            limb_add(qsteady + kLimbWords * ((size_t)p0 + cur), Fixed128{sink.steady_lo, sink.steady_hi});
    };
    for (uint32_t w = threadIdx.x; w < work; w += blockDim.x) {
        const uint32_t pl = w / L.spp;
        const uint32_t s = w - pl * L.spp;
        const size_t p = (size_t)p0 + pl;
        if (pl != cur) {
            flush();
            cur = pl;
            sink.row = qfilm + kLimbWords * p * T;
            sink.oow = qoow + kLimbWords * p;
            sink.steady_lo = 0ull;
            sink.steady_hi = 0ull;
        }
        trace_path(S, L, (uint32_t)p, L.sample_offset + s, stk, sink, tally);
    }
    flush();
}

// Renders one tile of pixels [p0, p0 + tile_pixels) with all their samples:
// LDS film rows (zeroed here), paths traced one per lane, then one
// coalesced write (or accumulate) of the tile to HBM.  lds_film holds
// tile_pixels * n_bins + 2 * tile_pixels floats; stk is the lane's stack.
template <class St, class TallyT>
__device__ __forceinline__ void render_tile(const SceneView& S, const LaunchArgs& L, uint32_t p0, float* lds_film,
                                            const float* freq, St& stk, TallyT& tally)
{
    const uint32_t T = film_words(S, L);
    const uint32_t TP = L.tile_pixels;
    float* tfilm = lds_film;
    float* tsteady = lds_film + (size_t)TP * T;
    float* toow = tsteady + TP;
    const uint32_t npix = min(TP, L.n_pixels - p0);
    for (uint32_t i = threadIdx.x; i < TP * T + 2 * TP; i += blockDim.x) lds_film[i] = 0.0f;
    __syncthreads();

    const uint32_t work = npix * L.spp;
    uint32_t cur = 0xffffffffu;
    FilmSink sink{nullptr, 0.0f, 0.0f, freq, L.n_freq};
    for (uint32_t w = threadIdx.x; w < work; w += blockDim.x) {
        const uint32_t pl = w / L.spp;
        const uint32_t s = w - pl * L.spp;
        if (pl != cur) {
            if (cur != 0xffffffffu) {
                atomicAdd(tsteady + cur, sink.steady);
                atomicAdd(toow + cur, sink.oow);
            }
            cur = pl;
            sink.row = tfilm + (size_t)pl * T;
            sink.steady = 0.0f;
            sink.oow = 0.0f;
        }
        trace_path(S, L, p0 + pl, L.sample_offset + s, stk, sink, tally);
    }
    if (cur != 0xffffffffu) {
        atomicAdd(tsteady + cur, sink.steady);
        atomicAdd(toow + cur, sink.oow);
    }
    __syncthreads();

    const bool acc = (L.flags & kFlagAccumulate) != 0;
    const size_t base = (size_t)p0 * T;
    const uint32_t nvals = npix * T;
    for (uint32_t i = threadIdx.x; i < nvals; i += blockDim.x) {
        const float v = tfilm[i] * L.norm;
        L.film[base + i] = acc ? L.film[base + i] + v : v;
    }
    if (threadIdx.x < npix) {
        const uint32_t p = p0 + threadIdx.x;
        if (L.steady) {
            const float v = tsteady[threadIdx.x] * L.norm;
            L.steady[p] = acc ? L.steady[p] + v : v;
        }
        if (L.oow) {
            const float v = toow[threadIdx.x] * L.norm;
            L.oow[p] = acc ? L.oow[p] + v : v;
        }
    }
}

// Path per lane with the film in HBM: every contribution, scaled by 1/N, is
// a float atomic add into the film itself (zeroed beforehand unless
// accumulating), so the workgroup keeps no film in LDS, only its lanes'
// stacks.  For long films (1,024 bins of a 1M-triangle scene: 4 KB per
// pixel) the LDS film is what limits the workgroups a CU holds; a pixel's
// row stays in L2 while its tile renders, so its atomics are served there.
struct HbmFilmSink {
    static constexpr bool kWantsGradients = false;
    float* row;  // HBM film row of the current pixel
    float norm;
    float steady, oow;  // register partial sums of the current pixel (unnormalised)
    __device__ __forceinline__ void contribution(int, int, float c, int bin, float, float, float)
    {
        if (bin >= 0) unsafeAtomicAdd(row + bin, c * norm);
        else oow += c;
        steady += c;
    }
    __device__ __forceinline__ void continuation(int, int, float, float) {}
};

template <class St, class TallyT>
__device__ __forceinline__ void render_tile_hbm(const SceneView& S, const LaunchArgs& L, uint32_t p0, St& stk,
                                                TallyT& tally)
{
    const uint32_t T = S.n_bins;
    const uint32_t npix = min(L.tile_pixels, L.n_pixels - p0);
    const uint32_t work = npix * L.spp;
    uint32_t cur = 0xffffffffu;
    HbmFilmSink sink{nullptr, L.norm, 0.0f, 0.0f};
    auto flush = [&]() {
        if (cur == 0xffffffffu) return;
        if (L.steady) unsafeAtomicAdd(L.steady + p0 + cur, sink.steady * L.norm);
        if (L.oow) unsafeAtomicAdd(L.oow + p0 + cur, sink.oow * L.norm);
    };
    for (uint32_t w = threadIdx.x; w < work; w += blockDim.x) {
        const uint32_t pl = w / L.spp;
        const uint32_t s = w - pl * L.spp;
        if (pl != cur) {
            flush();
            cur = pl;
            sink.row = L.film + (size_t)(p0 + pl) * T;
            sink.steady = 0.0f;
            sink.oow = 0.0f;
        }
        trace_path(S, L, p0 + pl, L.sample_offset + s, stk, sink, tally);
    }
    flush();
}

// Same tile, deferred form.  Phase 1 takes the tile's samples in batches
// of kSortPerLane * block: the batch is counting-sorted in LDS by a cell of
// its first rays' directions, and the waves then trace the first rays in
// sorted order, each lane taking the next ray of the order as soon as its
// own has finished (in groups, see trace_first_hits), and append every
// first vertex (work index, t, triangle) to an LDS buffer.  Sorting keeps
// rays of similar direction (similar traversals) in the same wave; the
// refill keeps the waves full while the few rays that reach the scene
// traverse deep.  Whenever the buffer holds a block's worth, phase 2
// drains it: each lane regenerates its entry's path state (Philox block
// 0), then shades, tests the shadow ray and follows the rest of the path,
// on densely packed lanes.  Redrawing a first ray costs less than keeping
// it: four LDS words per sample would cost the kernel a workgroup per CU.
//
// The sort cell needs no direction: for a given pixel the first ray's
// direction is a continuous function of the two uniforms (u0, u1) of
// Philox block 0 (the cosine map in the relay wall's frame, which is the
// same for every scan point, or the jitter inside a pinhole pixel), so a
// Morton-ordered cell of the (u0, u1) square is a compact cell of
// directions, and equally probable.
constexpr uint32_t kSortPerLane = 8;
constexpr uint32_t kCellBits = 4;  // per axis: 256 cells
constexpr uint32_t kDirCells = 1u << (2 * kCellBits);
static_assert(kDirCells % 64 == 0, "one wave scans the cell counts");

struct DeferredLds {
    uint32_t* work;    // first-hit buffer, capacity 2 * block
    float* t;
    int* prim;
    int* sorted;
    uint32_t* count;   // [0] buffer fill, [1] sorted batch size, [2] next sorted ray, [3] reserved slots
    uint32_t* order;   // [block * kSortPerLane] work indices in cell order
    uint32_t* start;   // [kDirCells] first slot of each cell
    uint32_t* fill;    // [kDirCells]
};

// 32-bit words of LDS the deferred form adds per block of nb lanes
__host__ __device__ constexpr size_t deferred_words(uint32_t nb)
{
    return 8ull * nb + 4 + (size_t)nb * kSortPerLane + 2ull * kDirCells;
}

__device__ __forceinline__ DeferredLds carve_deferred(float* base, uint32_t nb)
{
    const uint32_t cap = 2 * nb;
    DeferredLds f;
    uint32_t* u = reinterpret_cast<uint32_t*>(base);
    f.work = u;
    f.t = reinterpret_cast<float*>(u + cap);
    f.prim = reinterpret_cast<int*>(u + 2 * cap);
    f.sorted = reinterpret_cast<int*>(u + 3 * cap);
    f.count = u + 4 * cap;
    f.order = u + 4 * cap + 4;
    f.start = f.order + nb * kSortPerLane;
    f.fill = f.start + kDirCells;
    return f;
}

// sort cell of a sample's first ray: Morton index of (u0, u1) on a
// 2^kCellBits square grid
__device__ __forceinline__ uint32_t first_ray_cell(const LaunchArgs& L, uint32_t pix, uint32_t sample)
{
    const rand4 u = draw4(pix, sample, 0u, L.stream_id, L.key0, L.key1);
    constexpr float kRes = (float)(1u << kCellBits);
    uint32_t qx = (uint32_t)(u.u0 * kRes), qy = (uint32_t)(u.u1 * kRes);
    uint32_t m = 0;
#pragma unroll
    for (uint32_t b = 0; b < kCellBits; ++b) m |= (((qx >> b) & 1u) << (2 * b)) | (((qy >> b) & 1u) << (2 * b + 1));
    return m;
}

// sort cell of an area-sampled path: the BVH-order (Morton) position of its
// hidden triangle, so that a wave's shadow rays leave one patch of the
// hidden surface toward the same scan point
__device__ __forceinline__ uint32_t area_cell(const SceneView& S, const LaunchArgs& L, uint32_t pix,
                                              uint32_t sample)
{
    const rand4 u = draw4(pix, sample, 0u, L.stream_id, L.key0, L.key1);
    const uint32_t j = S.sorted_of[area_pick(S, S.area_region[pix], u.u0)];
    return (uint32_t)(((uint64_t)j * kDirCells) / S.n_tris);
}

constexpr int kRefill = 32;

// Closest hits of the sorted first rays [0, nvalid) of a batch, appended
// to the first-hit buffer.  Each wave keeps its lanes busy: once kRefill
// of its lanes have finished their rays, those lanes take the next rays of
// the order, so the long traversals of rays that reach the scene run side
// by side instead of each holding a mostly idle wave.  A ray starts only
// with a reserved buffer slot (released if it leaves the scene), so the
// buffer never overflows; a wave returns once it can start no ray and has
// none in flight.  No barrier inside.
template <class St, class TallyT>
__device__ __forceinline__ void trace_first_hits(const SceneView& S, const LaunchArgs& L, uint32_t p0,
                                                 const DeferredLds& fh, uint32_t nvalid, St& stk,
                                                 TallyT& tally)
{
    const uint32_t cap = 2 * blockDim.x;
    bool active = false;
    bool fetch = true;  // wave-uniform
    uint32_t w = 0;
    PathState ps;
    Ray r;
    ClosestTrav c;
    for (;;) {
        if (fetch && __popcll(__ballot(!active)) >= kRefill) {
            bool failed = false;
            if (!active) {
                const uint32_t rs = atomicAdd(fh.count + 3, 1u);
                const uint32_t j = rs < cap ? atomicAdd(fh.count + 2, 1u) : 0xffffffffu;
                if (j < nvalid) {
                    w = fh.order[j];
                    const uint32_t pl = w / L.spp;
                    begin_path(S, L, p0 + pl, L.sample_offset + (w - pl * L.spp), ps);
                    r = make_ray(ps.o, ps.d);
                    closest_begin(S, r, ps.prev, c, tally);
                    active = true;
                } else {
                    atomicSub(fh.count + 3, 1u);
                    failed = true;
                }
            }
            if (__any(failed)) fetch = false;
        }
        if (!__any(active)) break;
        while (active) {
            if (closest_step(S, r, ps.prev, stk, c, tally)) {
                float t_hit;
                bool med;
                if (resolve_event(S, ps, c.h, t_hit, med)) {
                    const uint32_t q = atomicAdd(fh.count, 1u);
                    fh.work[q] = w;
                    fh.t[q] = c.h.t;
                    fh.prim[q] = c.h.prim;
                    fh.sorted[q] = c.h.sorted;
                } else {
                    atomicSub(fh.count + 3, 1u);
                }
                active = false;
            }
            if (fetch && __popcll(__ballot(active)) <= 64 - kRefill) break;
        }
    }
}

// kArea: NLOS area sampling, whose first vertex needs no traversal; the
// batch is sorted by area_cell and each lane follows the sorted paths
// directly (phase 1b and 2 in one).
template <bool kArea, class St, class TallyT>
__device__ __forceinline__ void render_tile_deferred(const SceneView& S, const LaunchArgs& L, uint32_t tile,
                                                     uint32_t chunk, float* lds_film, const float* freq,
                                                     const DeferredLds& fh, St& stk, TallyT& tally)
{
    const uint32_t p0 = tile * L.tile_pixels;
    const uint32_t T = film_words(S, L);
    const uint32_t TP = L.tile_pixels;
    float* tfilm = lds_film;
    float* tsteady = lds_film + (size_t)TP * T;
    float* toow = tsteady + TP;
    const uint32_t npix = min(TP, L.n_pixels - p0);
    const uint32_t nb = blockDim.x;
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < TP * T + 2 * TP; i += nb) lds_film[i] = 0.0f;
    if (tid == 0) {
        fh.count[0] = 0u;
        fh.count[3] = 0u;
    }
    __syncthreads();

    const uint32_t work = npix * L.spp;
    const bool has_vertex = last_vertex(S, L) >= 1;
    const uint32_t batch = nb * kSortPerLane;
    uint32_t cur = 0xffffffffu;
    FilmSink sink{nullptr, 0.0f, 0.0f, freq, L.n_freq};
    for (uint32_t base = 0; base < work; base += batch) {
        // phase 1a: counting sort of the batch by first-ray cell
        for (uint32_t i = tid; i < kDirCells; i += nb) {
            fh.start[i] = 0u;
            fh.fill[i] = 0u;
        }
        __syncthreads();
        uint32_t cell[kSortPerLane];
#pragma unroll
        for (uint32_t k = 0; k < kSortPerLane; ++k) {
            const uint32_t w = base + k * nb + tid;
            cell[k] = 0xffffffffu;
            if (w < work && has_vertex) {
                const uint32_t pl = w / L.spp;
                tally.add(kTallyDraws);
                const uint32_t sample = L.sample_offset + (w - pl * L.spp);
                cell[k] = kArea ? area_cell(S, L, p0 + pl, sample) : first_ray_cell(L, p0 + pl, sample);
                atomicAdd(fh.start + cell[k], 1u);
            }
        }
        __syncthreads();
        if (tid < 64) {  // exclusive scan of the cell counts by the first wave
            constexpr uint32_t kPerLane = kDirCells / 64;
            uint32_t c[kPerLane];
            uint32_t sum = 0;
#pragma unroll
            for (uint32_t i = 0; i < kPerLane; ++i) {
                c[i] = fh.start[tid * kPerLane + i];
                sum += c[i];
            }
            uint32_t x = sum;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off, 64);
                if ((int)tid >= off) x += y;
            }
            uint32_t run = x - sum;
#pragma unroll
            for (uint32_t i = 0; i < kPerLane; ++i) {
                fh.start[tid * kPerLane + i] = run;
                run += c[i];
            }
            if (tid == 63) {
                fh.count[1] = x;
                fh.count[2] = 0u;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < kSortPerLane; ++k)
            if (cell[k] != 0xffffffffu)
                fh.order[fh.start[cell[k]] + atomicAdd(fh.fill + cell[k], 1u)] = base + k * nb + tid;
        __syncthreads();
        const uint32_t nvalid = fh.count[1];
        if (kArea) {
            for (uint32_t jj = tid; jj < nvalid; jj += nb) {
                const uint32_t wj = fh.order[jj];
                const uint32_t pl = wj / L.spp;
                const uint32_t sample = L.sample_offset + (wj - pl * L.spp);
                if (pl != cur) {
                    if (cur != 0xffffffffu) {
                        atomicAdd(tsteady + cur, sink.steady);
                        atomicAdd(toow + cur, sink.oow);
                    }
                    cur = pl;
                    sink.row = tfilm + (size_t)pl * T;
                    sink.steady = 0.0f;
                    sink.oow = 0.0f;
                }
                PathState ps;
                Hit h;
                if (begin_area(S, L, p0 + pl, sample, ps, h))
                    continue_path(S, L, p0 + pl, sample, ps, h, stk, sink, tally);
            }
            __syncthreads();  // the next batch reuses the order
            continue;
        }
        // phase 1b: first rays in cell order; phase 2 whenever the buffer
        // holds a block's worth (or at the end of the tile)
        const bool last_batch = base + batch >= work;
        for (;;) {
            trace_first_hits(S, L, p0, fh, nvalid, stk, tally);
            __syncthreads();
            const uint32_t n = fh.count[0];
            const bool exhausted = fh.count[2] >= nvalid;
            if (n >= nb || (last_batch && exhausted)) {
                for (uint32_t jj = tid; jj < n; jj += nb) {
                    const uint32_t wj = fh.work[jj];
                    const uint32_t pl = wj / L.spp;
                    const uint32_t sample = L.sample_offset + (wj - pl * L.spp);
                    if (pl != cur) {
                        if (cur != 0xffffffffu) {
                            atomicAdd(tsteady + cur, sink.steady);
                            atomicAdd(toow + cur, sink.oow);
                        }
                        cur = pl;
                        sink.row = tfilm + (size_t)pl * T;
                        sink.steady = 0.0f;
                        sink.oow = 0.0f;
                    }
                    PathState ps;
                    begin_path(S, L, p0 + pl, sample, ps);
                    Hit h;
                    h.t = fh.t[jj];
                    h.prim = fh.prim[jj];
                    h.sorted = fh.sorted[jj];
                    continue_path(S, L, p0 + pl, sample, ps, h, stk, sink, tally);
                }
                __syncthreads();
                if (tid == 0) {
                    fh.count[0] = 0u;
                    fh.count[3] = 0u;
                }
                __syncthreads();
            }
            if (exhausted) break;
        }
    }
    if (cur != 0xffffffffu) {
        atomicAdd(tsteady + cur, sink.steady);
        atomicAdd(toow + cur, sink.oow);
    }
    __syncthreads();

    const size_t fbase = (size_t)p0 * T;
    const uint32_t nvals = npix * T;
    const bool acc = (L.flags & kFlagAccumulate) != 0;
    if (chunk > 0) {
        // Other workgroups hold other samples of these pixels.  Chunk 0
        // writes the film as a single workgroup would; chunk c > 0 leaves
        // its normalised partial tile in plane c - 1 of the scratch (the
        // film's layout, then steady and oow), which a second pass adds to
        // the film in chunk order.  (Adding the partials into the film with
        // device-scope atomics cost one 64-byte memory write per atomic,
        // 10x the film's bytes; a last-finisher reduction inside the kernel
        // needs device-scope fences, which write back and invalidate the
        // XCD's whole L2 and with it the BVH.)
        const size_t film_n = (size_t)L.n_pixels * T;
        float* plane = L.chunk_scratch + (size_t)(chunk - 1) * (film_n + 2ull * L.n_pixels);
        for (uint32_t i = tid; i < nvals; i += nb) plane[fbase + i] = tfilm[i] * L.norm;
        if (tid < npix) {
            plane[film_n + p0 + tid] = tsteady[tid] * L.norm;
            plane[film_n + L.n_pixels + p0 + tid] = toow[tid] * L.norm;
        }
        return;
    }
    for (uint32_t i = tid; i < nvals; i += nb) {
        const float v = tfilm[i] * L.norm;
        L.film[fbase + i] = acc ? L.film[fbase + i] + v : v;
    }
    if (tid < npix) {
        const uint32_t p = p0 + tid;
        if (L.steady) {
            const float v = tsteady[tid] * L.norm;
            L.steady[p] = acc ? L.steady[p] + v : v;
        }
        if (L.oow) {
            const float v = toow[tid] * L.norm;
            L.oow[p] = acc ? L.oow[p] + v : v;
        }
    }
}

// Five waves per SIMD (at most 96 VGPRs, a few spilled outside the
// traversal loops) beat four without spills by 15% on confocal scans.
// Workgroups go to the 8 XCDs in turn (workgroup b runs on XCD b mod 8),
// and each XCD has its own L2.  The launch index is remapped so that, within
// every run of 8 * kXcdGroup workgroups, XCD x takes kXcdGroup consecutive
// tiles: the tiles an XCD holds at once are neighbours, whose rays meet the
// same part of the scene in its L2, while all XCDs still sweep the image
// together.  Workgroups past the last full run keep their index.
constexpr uint32_t kXcds = 8, kXcdGroup = 64;
__device__ __forceinline__ uint32_t xcd_block()
{
    const uint32_t b = blockIdx.x, n = gridDim.x;
    constexpr uint32_t run = kXcds * kXcdGroup;
    if (b >= (n / run) * run) return b;
    const uint32_t x = b % kXcds, k = b / kXcds;  // the k-th workgroup of XCD x
    return (k / kXcdGroup) * run + x * kXcdGroup + k % kXcdGroup;
}

// First pixel of this workgroup's tile (tiles of TP consecutive pixels, in
// the XCD-aware order).  In scenes too large for an XCD's L2 (more than
// 32,768 triangles: 3.7 MB of nodes and triangle records), one-pixel tiles
// of a camera image walk it in 16 x 16 pixel blocks (8 x 8 when its sides
// are multiples of 8 but not of 16) instead of rows, so the tiles the XCDs
// take at a time are compact patches of pixels, whose rays share more of
// the scene than row segments' (1M-triangle scene: 8 x 8 blocks +2 % over
// rows, 16 x 16 blocks +1.2 % over 8 x 8, 32 x 32 the same; on a
// 9,826-triangle scene that fits in L2 the blocks only cost, -5 % forward).
__device__ __forceinline__ uint32_t tile_first_pixel(const SceneView& S, const LaunchArgs& L, uint32_t TP)
{
    const uint32_t t = xcd_block();
    if (TP == 1 && S.sensor == 0 && S.n_tris > 32768u && L.n_pixels == S.width * S.height) {
        if ((S.width & 15u) == 0 && (S.height & 15u) == 0) {
            const uint32_t blk = t >> 8, in = t & 255u, bw = S.width >> 4;
            return ((blk / bw) * 16u + (in >> 4)) * S.width + (blk % bw) * 16u + (in & 15u);
        }
        if ((S.width & 7u) == 0 && (S.height & 7u) == 0) {
            const uint32_t blk = t >> 6, in = t & 63u, bw = S.width >> 3;
            return ((blk / bw) * 8u + (in >> 3)) * S.width + (blk % bw) * 8u + (in & 7u);
        }
    }
    return t * TP;
}

template <int kMode, class W, bool kArea>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_render_deferred(SceneView S, LaunchArgs L, unsigned long long* counts)
{
    Tally<kMode> tally;
    extern __shared__ float lds[];
    const uint32_t TP = L.tile_pixels;
    // workgroup -> (tile, chunk of the tile's samples)
    const uint32_t wg = xcd_block();
    const uint32_t tile = wg / L.chunks, chunk = wg - tile * L.chunks;
    LaunchArgs Lc = L;
    Lc.sample_offset = L.sample_offset + chunk * L.chunk_spp;
    Lc.spp = min(L.chunk_spp, L.spp - chunk * L.chunk_spp);
    __shared__ float s_freq[kMaxFreq];
    load_freqs(L, s_freq);
    float* after_film = lds + (size_t)TP * film_words(S, L) + 2 * TP;
    const DeferredLds fh = carve_deferred(after_film, blockDim.x);
    LdsStack<W> stk{reinterpret_cast<W*>(after_film + deferred_words(blockDim.x)) + threadIdx.x, (int)blockDim.x};
    render_tile_deferred<kArea>(S, Lc, tile, chunk, lds, s_freq, fh, stk, tally);
    tally.flush(counts);
}

template <int kMode, class W>
__global__ void __launch_bounds__(256) k_render(SceneView S, LaunchArgs L, unsigned long long* counts)
{
    Tally<kMode> tally;
    extern __shared__ float lds[];
    const uint32_t TP = L.tile_pixels;
    __shared__ float s_freq[kMaxFreq];
    load_freqs(L, s_freq);
    LdsStack<W> stk{reinterpret_cast<W*>(lds + (size_t)TP * film_words(S, L) + 2 * TP) + threadIdx.x, (int)blockDim.x};
    render_tile(S, L, tile_first_pixel(S, L, TP), lds, s_freq, stk, tally);
    tally.flush(counts);
}

// Five waves per SIMD (at most 96 VGPRs, a few spills): with no LDS film a
// CU holds the whole stacks of 20 waves.
template <int kMode, class W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_render_hbm(SceneView S, LaunchArgs L, unsigned long long* counts)
{
    Tally<kMode> tally;
    extern __shared__ float lds[];
    LdsStack<W> stk{reinterpret_cast<W*>(lds) + threadIdx.x, (int)blockDim.x};
    render_tile_hbm(S, L, tile_first_pixel(S, L, L.tile_pixels), stk, tally);
    tally.flush(counts);
}

// 32-bit links with the split stack: 4 KB of LDS per 64-lane workgroup, so
// eight waves per SIMD fit (at most 64 VGPRs, more spills; 1M-triangle
// scene: +21 % over five waves with whole stacks in LDS).
template <int kMode>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_render_hbm_split(SceneView S, LaunchArgs L, unsigned long long* counts)
{
    Tally<kMode> tally;
    extern __shared__ float lds[];
    int deep[kSplitStackDeep];
    SplitStack<(int)kSplitStackLds, (int)kSplitStackDeep> stk{
        (__attribute__((address_space(3))) uint32_t*)(reinterpret_cast<uint32_t*>(lds) + threadIdx.x),
        (int)blockDim.x, deep};
    render_tile_hbm(S, L, tile_first_pixel(S, L, L.tile_pixels), stk, tally);
    tally.flush(counts);
}

// the deterministic HBM-film form: split stacks at eight waves per SIMD, or
// whole stacks in LDS (deeper trees) at five, as k_render_hbm_split and
// k_render_hbm
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_render_fixed_hbm_split(SceneView S, LaunchArgs L)
{
    Tally<kPlain> tally;
    extern __shared__ float lds[];
    int deep[kSplitStackDeep];
    SplitStack<(int)kSplitStackLds, (int)kSplitStackDeep> stk{
        (__attribute__((address_space(3))) uint32_t*)(reinterpret_cast<uint32_t*>(lds) + threadIdx.x),
        (int)blockDim.x, deep};
    render_tile_fixed_hbm(S, L, tile_first_pixel(S, L, L.tile_pixels), stk, tally);
}

template <class W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_render_fixed_hbm(SceneView S, LaunchArgs L)
{
    Tally<kPlain> tally;
    extern __shared__ float lds[];
    LdsStack<W> stk{reinterpret_cast<W*>(lds) + threadIdx.x, (int)blockDim.x};
    render_tile_fixed_hbm(S, L, tile_first_pixel(S, L, L.tile_pixels), stk, tally);
}

// each film, steady and oow sum of L.fixed_film / norm_spp, rounded to FP32
// once, written (or added, when accumulating) to the outputs
__global__ void k_fixed_film_out(LaunchArgs L, uint32_t T)
{
    const size_t nf = (size_t)L.n_pixels * T;
    const size_t n = nf + 2ull * L.n_pixels;
    const bool acc = (L.flags & kFlagAccumulate) != 0;
    const double norm = (double)L.norm_spp;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float* dst;
        if (i < nf) dst = L.film + i;
        else if (i < nf + L.n_pixels) dst = L.steady ? L.steady + (i - nf) : nullptr;
        else dst = L.oow ? L.oow + (i - nf - L.n_pixels) : nullptr;
        if (!dst) continue;
        const unsigned long long* w = L.fixed_film + kLimbWords * i;
        const Fixed128 f = limb_value(w[0], w[1], w[2]);
        const float v = (float)(from_fixed(f.lo, f.hi) / norm);
        *dst = acc ? *dst + v : v;
    }
}

template <class W>
__global__ void __launch_bounds__(256) k_render_fixed(SceneView S, LaunchArgs L)
{
    Tally<kPlain> tally;
    extern __shared__ float lds[];
    const uint32_t TP = L.tile_pixels;
    unsigned long long* q = reinterpret_cast<unsigned long long*>(lds);
    LdsStack<W> stk{reinterpret_cast<W*>(q + 2ull * (TP * S.n_bins + 2 * TP)) + threadIdx.x, (int)blockDim.x};
    render_tile_fixed(S, L, tile_first_pixel(S, L, TP), q, stk, tally);
}

// ---------------------------------------------------------------------------
// batched persistent form: many scenes, one launch
// ---------------------------------------------------------------------------
// Work items are (scene, pixel tile) pairs numbered scene by scene in the
// processing order; a workgroup pops items from a global cursor until they
// run out, so scenes of very different cost balance themselves.  One launch
// serves scenes of one stack-link width W (the batch splits its scenes into
// classes); the tile width is each scene's own.
template <bool kDeferred, class W>
__global__ void __launch_bounds__(256) k_batch(BatchTables B)
{
    extern __shared__ float lds[];
    __shared__ uint32_t s_item;
    Tally<kPlain> tally;
    const DeferredLds fh = carve_deferred(lds + B.film_words, blockDim.x);
    LdsStack<W> stk{reinterpret_cast<W*>(lds + B.film_words + (kDeferred ? deferred_words(blockDim.x) : 0)) + threadIdx.x,
                    (int)blockDim.x};
    while (true) {
        if (threadIdx.x == 0) s_item = atomicAdd(B.cursor, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= B.n_items) break;
        uint32_t lo = 0, hi = B.n_scenes;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (B.item_start[mid] <= item) lo = mid;
            else hi = mid;
        }
        const uint32_t scene = __builtin_amdgcn_readfirstlane(B.order[lo]);
        const uint32_t tile = item - B.item_start[lo];
        const SceneView* __restrict__ views = B.views;
        const LaunchArgs* __restrict__ args = B.args;
        // NLOS area sampling needs no first-hit traversal to defer: such
        // scenes take the path-per-lane tile (same LDS film and stacks)
        if (kDeferred && !(args[scene].flags & kFlagNlosArea))
            render_tile_deferred<false>(views[scene], args[scene], tile, 0u, lds, nullptr, fh, stk,
                                        tally);
        else
            render_tile(views[scene], args[scene], tile * args[scene].tile_pixels, lds, nullptr, stk, tally);
        __syncthreads();
    }
}

__global__ void k_reset_cursor(uint32_t* cursor)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *cursor = 0u;
}

// ---------------------------------------------------------------------------
// forward render, wavefront form: one workgroup runs the stages of its
// tile's paths over queues kept in LDS
// ---------------------------------------------------------------------------
// Each lane owns one path slot (SoA arrays in LDS).  A round is
//   GEN       dead slots take the next (pixel, sample) of the tile,
//   INTERSECT closest hit + free flight for every live ray (ray queue),
//   SHADE     next-event geometry and continuation for every vertex (hit
//             queue), producing shadow records (shadow queue) and the
//             continuing rays (ray queue of the next round),
//   SHADOW    any-hit for every shadow record, accumulation into the tile
//             film in LDS,
// with a barrier between stages.  Compaction into queues keeps the costly
// stages dense: a wave that has no entry in a queue skips that stage and
// leaves its SIMD to other waves.
constexpr int kWfWords = 34;  // 32-bit words of LDS per slot

struct WfSlots {
    float *ox, *oy, *oz, *dx, *dy, *dz, *beta, *opl, *uff, *eta;
    int *prev, *v, *pl, *live;
    uint32_t* sample;
    float* ht;
    int *hprim, *hsorted, *hmed;
    float *sox, *soy, *soz, *sdx, *sdy, *sdz, *stmax, *sc, *stof;
    int *sexcl, *sbin, *sv;
    int *ray_q, *hit_q, *sh_q;
};

__device__ __forceinline__ WfSlots carve_slots(float* base, int ns)
{
    WfSlots w;
    float* f = base;
    auto take_f = [&]() { float* r = f; f += ns; return r; };
    auto take_i = [&]() { int* r = reinterpret_cast<int*>(f); f += ns; return r; };
    w.ox = take_f(); w.oy = take_f(); w.oz = take_f();
    w.dx = take_f(); w.dy = take_f(); w.dz = take_f();
    w.beta = take_f(); w.opl = take_f(); w.uff = take_f(); w.eta = take_f();
    w.prev = take_i(); w.v = take_i(); w.pl = take_i(); w.live = take_i();
    w.sample = reinterpret_cast<uint32_t*>(take_i());
    w.ht = take_f(); w.hprim = take_i(); w.hsorted = take_i(); w.hmed = take_i();
    w.sox = take_f(); w.soy = take_f(); w.soz = take_f();
    w.sdx = take_f(); w.sdy = take_f(); w.sdz = take_f();
    w.stmax = take_f(); w.sc = take_f(); w.stof = take_f();
    w.sexcl = take_i(); w.sbin = take_i(); w.sv = take_i();
    w.ray_q = take_i(); w.hit_q = take_i(); w.sh_q = take_i();
    return w;
}

__device__ __forceinline__ void store_state(const WfSlots& w, int i, const PathState& ps)
{
    w.ox[i] = ps.o.x; w.oy[i] = ps.o.y; w.oz[i] = ps.o.z;
    w.dx[i] = ps.d.x; w.dy[i] = ps.d.y; w.dz[i] = ps.d.z;
    w.beta[i] = ps.beta; w.opl[i] = ps.opl; w.uff[i] = ps.u_ff; w.eta[i] = ps.eta;
    w.prev[i] = ps.prev; w.v[i] = ps.v;
}

__device__ __forceinline__ PathState load_state(const WfSlots& w, int i)
{
    PathState ps;
    ps.o = v3(w.ox[i], w.oy[i], w.oz[i]);
    ps.d = v3(w.dx[i], w.dy[i], w.dz[i]);
    ps.beta = w.beta[i]; ps.opl = w.opl[i]; ps.u_ff = w.uff[i]; ps.eta = w.eta[i];
    ps.prev = w.prev[i]; ps.v = w.v[i];
    return ps;
}

template <int kMode, class W>
__global__ void __launch_bounds__(256) k_render_wf(SceneView S, LaunchArgs L, unsigned long long* counts)
{
    extern __shared__ float lds[];
    __shared__ uint32_t ctr[4];  // ray queue, hit queue, shadow queue, next work item
    Tally<kMode> tally;
    const uint32_t T = S.n_bins;
    const uint32_t TP = L.tile_pixels;
    const int nb = (int)blockDim.x;
    const int tid = (int)threadIdx.x;
    float* tfilm = lds;
    float* tsteady = lds + (size_t)TP * T;
    float* toow = tsteady + TP;
    const WfSlots w = carve_slots(toow + TP, nb);
    LdsStack<W> stk{reinterpret_cast<W*>(toow + TP + (size_t)kWfWords * nb) + tid, nb};
    const uint32_t p0 = tile_first_pixel(S, L, TP);
    const uint32_t npix = min(TP, L.n_pixels - p0);
    for (uint32_t i = tid; i < TP * T + 2 * TP; i += nb) lds[i] = 0.0f;
    w.live[tid] = 0;
    if (tid < 4) ctr[tid] = 0u;
    __syncthreads();
    // paths without a vertex (max_depth too small) contribute nothing
    const uint32_t work = last_vertex(S, L) >= 1 ? npix * L.spp : 0u;

    while (true) {
        // GEN: dead slots take new samples
        if (!w.live[tid] && ctr[3] < work) {
            const uint32_t item = atomicAdd(&ctr[3], 1u);
            if (item < work) {
                const uint32_t pl = item / L.spp;
                const uint32_t s = L.sample_offset + (item - pl * L.spp);
                tally.add(kTallyDraws);
                PathState ps;
                begin_path(S, L, p0 + pl, s, ps);
                store_state(w, tid, ps);
                w.pl[tid] = (int)pl;
                w.sample[tid] = s;
                w.live[tid] = 1;
                w.ray_q[atomicAdd(&ctr[0], 1u)] = tid;
            }
        }
        __syncthreads();
        const int nr = (int)ctr[0];
        if (nr == 0) break;
        // INTERSECT
        for (int j = tid; j < nr; j += nb) {
            const int i = w.ray_q[j];
            const PathState ps = load_state(w, i);
            const Hit h = closest_hit(S, make_ray(ps.o, ps.d), ps.prev, stk, tally);
            float t_hit;
            bool med;
            if (resolve_event(S, ps, h, t_hit, med)) {
                w.ht[i] = t_hit;
                w.hprim[i] = h.prim;
                w.hsorted[i] = h.sorted;
                w.hmed[i] = med ? 1 : 0;
                w.hit_q[atomicAdd(&ctr[1], 1u)] = i;
            } else {
                w.live[i] = 0;
            }
        }
        __syncthreads();
        if (tid == 0) ctr[0] = 0u;
        const int nh = (int)ctr[1];
        __syncthreads();
        // SHADE
        for (int j = tid; j < nh; j += nb) {
            const int i = w.hit_q[j];
            PathState ps = load_state(w, i);
            const int v = ps.v;
            Hit h;
            h.t = w.ht[i];
            h.prim = w.hprim[i];
            h.sorted = w.hsorted[i];
            Nee nee;
            Cont cont;
            shade_vertex<false>(S, L, p0 + (uint32_t)w.pl[i], w.sample[i], ps, h, h.t, w.hmed[i] != 0, nee, cont,
                                tally);
            if (nee.valid) {
                w.sox[i] = nee.so.x; w.soy[i] = nee.so.y; w.soz[i] = nee.so.z;
                w.sdx[i] = nee.sd.x; w.sdy[i] = nee.sd.y; w.sdz[i] = nee.sd.z;
                w.stmax[i] = nee.tmax; w.sc[i] = nee.c; w.sexcl[i] = nee.excl; w.sbin[i] = nee.bin;
                w.stof[i] = nee.tof; w.sv[i] = v;
                w.sh_q[atomicAdd(&ctr[2], 1u)] = i;
            }
            if (cont.alive) {
                store_state(w, i, ps);
                w.ray_q[atomicAdd(&ctr[0], 1u)] = i;
            } else {
                w.live[i] = 0;
            }
        }
        __syncthreads();
        if (tid == 0) ctr[1] = 0u;
        const int ns = (int)ctr[2];
        __syncthreads();
        // SHADOW + accumulate into the tile film
        for (int j = tid; j < ns; j += nb) {
            const int i = w.sh_q[j];
            const Ray sh = make_ray(v3(w.sox[i], w.soy[i], w.soz[i]), v3(w.sdx[i], w.sdy[i], w.sdz[i]));
            if (!occluded(S, sh, w.sexcl[i], w.stmax[i], stk, tally)) {
                tally.add(kTallyContrib);
                const float c = w.sc[i];
                const int bin = w.sbin[i];
                const int pl = w.pl[i];
                tally.record(L, p0 + (uint32_t)pl, w.sample[i], w.sv[i], w.sexcl[i], c, bin, w.stof[i]);
                if (bin >= 0) atomicAdd(tfilm + (size_t)pl * T + bin, c);
                else atomicAdd(toow + pl, c);
                atomicAdd(tsteady + pl, c);
            }
        }
        __syncthreads();
        if (tid == 0) ctr[2] = 0u;
    }
    tally.flush(counts);
    __syncthreads();

    const bool acc = (L.flags & kFlagAccumulate) != 0;
    const size_t base = (size_t)p0 * T;
    const uint32_t nvals = npix * T;
    for (uint32_t i = tid; i < nvals; i += nb) {
        const float v = tfilm[i] * L.norm;
        L.film[base + i] = acc ? L.film[base + i] + v : v;
    }
    if ((uint32_t)tid < npix) {
        const uint32_t p = p0 + tid;
        if (L.steady) {
            const float v = tsteady[tid] * L.norm;
            L.steady[p] = acc ? L.steady[p] + v : v;
        }
        if (L.oow) {
            const float v = toow[tid] * L.norm;
            L.oow[p] = acc ? L.oow[p] + v : v;
        }
    }
}

// ---------------------------------------------------------------------------
// backward mode: path replay
// ---------------------------------------------------------------------------
// pass 1 sums a_j = delta[bin_j] c_j / N over the path; pass 2 replays the
// same path and, at each vertex v, adds a_v d log f_nee + (A - sum_{j<=v} a_j)
// d log f_cont to the vertex's triangle (contributions after v depend on the
// direction sampled at v).
struct AdjointSumSink {
    static constexpr bool kWantsGradients = false;
    const float* delta;  // LDS gradient row of the pixel
    float norm;
    double total;
    __device__ __forceinline__ void contribution(int, int, float c, int bin, float, float, float)
    {
        if (bin >= 0) total += (double)delta[bin] * (double)c * (double)norm;
    }
    __device__ __forceinline__ void continuation(int, int, float, float) {}
};

// Per-workgroup gradient cache in LDS.  The paths of a tile keep meeting
// the same triangles, so instead of one global atomic per vertex and
// parameter, a workgroup sums its gradients in an open-addressing table of
// kGradSlots slots keyed by triangle (LDS atomics), and adds each touched
// triangle's two sums to the global gradients once, at the end of the tile.
// A triangle that finds no slot within kGradProbes probes goes straight to
// the global gradients.  GradF64 sums in FP64 (layout from an 8-byte aligned
// base: albedo sums, roughness sums, int keys, -1 = empty); GradFixed, the
// deterministic form, in 128-bit fixed point (albedo [slot][2] words,
// roughness [slot][2] words, int keys), with global sums [2][n_tris][2].
constexpr uint32_t kGradSlots = 512;
constexpr int kGradProbes = 8;

__device__ __forceinline__ int grad_slot(int* key, int k)
{
    const uint32_t h = ((uint32_t)k * 2654435761u) >> 23;
    for (int p = 0; p < kGradProbes; ++p) {
        const uint32_t slot = (h + (uint32_t)p) & (kGradSlots - 1);
        int cur = key[slot];
        if (cur == -1) cur = atomicCAS(key + slot, -1, k);
        if (cur == -1 || cur == k) return (int)slot;
    }
    return -1;
}

struct GradF64 {
    static constexpr uint32_t kFloats = kGradSlots * 5;  // 2 doubles + 1 int per slot, in 4-byte words
    double* cache;
    double* g_alb;
    double* g_rough;
    __device__ __forceinline__ GradF64(float* lds, const SceneView&, const LaunchArgs& L)
        : cache(reinterpret_cast<double*>(lds)), g_alb(L.g_alb), g_rough(L.g_rough)
    {
    }
    __device__ __forceinline__ int* key() const { return reinterpret_cast<int*>(cache + 2 * kGradSlots); }
    __device__ __forceinline__ void add(int k, double a, double r)
    {
        if (a == 0.0 && r == 0.0) return;
        const int slot = grad_slot(key(), k);
        double* ga = slot >= 0 ? cache + slot : g_alb + k;
        double* gr = slot >= 0 ? cache + kGradSlots + slot : g_rough + k;
        if (a != 0.0) unsafeAtomicAdd(ga, a);
        if (r != 0.0) unsafeAtomicAdd(gr, r);
    }
    __device__ __forceinline__ void clear()
    {
        for (uint32_t i = threadIdx.x; i < kGradSlots; i += blockDim.x) {
            cache[i] = 0.0;
            cache[kGradSlots + i] = 0.0;
            key()[i] = -1;
        }
    }
    // after a barrier: the table's sums to the global gradients
    __device__ __forceinline__ void flush() const
    {
        for (uint32_t i = threadIdx.x; i < kGradSlots; i += blockDim.x) {
            const int k = key()[i];
            if (k < 0) continue;
            if (cache[i] != 0.0) unsafeAtomicAdd(g_alb + k, cache[i]);
            if (cache[kGradSlots + i] != 0.0) unsafeAtomicAdd(g_rough + k, cache[kGradSlots + i]);
        }
    }
};

struct GradFixed {
    static constexpr uint32_t kFloats = kGradSlots * 9;  // 4 words of 8 bytes + 1 int per slot
    unsigned long long* cache;
    unsigned long long* g;  // [2][n_tris][2]
    uint32_t n_tris;
    __device__ __forceinline__ GradFixed(float* lds, const SceneView& S, const LaunchArgs& L)
        : cache(reinterpret_cast<unsigned long long*>(lds)), g(L.g_fixed), n_tris(S.n_tris)
    {
    }
    __device__ __forceinline__ int* key() const { return reinterpret_cast<int*>(cache + 4 * kGradSlots); }
    __device__ __forceinline__ void add(int k, double a, double r)
    {
        if (a == 0.0 && r == 0.0) return;
        const int slot = grad_slot(key(), k);
        unsigned long long* ga = slot >= 0 ? cache + 2 * slot : g + 2ull * k;
        unsigned long long* gr = slot >= 0 ? cache + 2 * (kGradSlots + slot) : g + 2ull * (n_tris + k);
        fixed_add(ga, to_fixed(a));
        fixed_add(gr, to_fixed(r));
    }
    __device__ __forceinline__ void clear()
    {
        for (uint32_t i = threadIdx.x; i < 4 * kGradSlots; i += blockDim.x) cache[i] = 0ull;
        for (uint32_t i = threadIdx.x; i < kGradSlots; i += blockDim.x) key()[i] = -1;
    }
    __device__ __forceinline__ void flush() const
    {
        for (uint32_t i = threadIdx.x; i < kGradSlots; i += blockDim.x) {
            const int k = key()[i];
            if (k < 0) continue;
            fixed_add(g + 2ull * k, Fixed128{cache[2 * i], cache[2 * i + 1]});
            fixed_add(g + 2ull * (n_tris + k), Fixed128{cache[2 * (kGradSlots + i)], cache[2 * (kGradSlots + i) + 1]});
        }
    }
};

template <class Acc>
struct AdjointScatterSink {
    static constexpr bool kWantsGradients = true;
    const float* delta;
    float* primal_row;  // optional LDS primal film row
    float norm;
    double total;       // A from pass 1
    double prefix;      // sum of a_j so far
    Acc* acc;           // the workgroup's gradient table
    __device__ __forceinline__ void contribution(int, int k, float c, int bin, float, float g_alb_nee,
                                                 float g_rough_nee)
    {
        if (bin < 0) return;
        if (primal_row) atomicAdd(primal_row + bin, c);
        const double a = (double)delta[bin] * (double)c * (double)norm;
        prefix += a;
        if (k >= 0 && a != 0.0) acc->add(k, a * (double)g_alb_nee, a * (double)g_rough_nee);
    }
    __device__ __forceinline__ void continuation(int, int k, float g_alb_c, float g_rough_c)
    {
        const double rest = total - prefix;
        if (rest != 0.0) acc->add(k, rest * (double)g_alb_c, rest * (double)g_rough_c);
    }
};

// Forward mode (Sec. 4.4): the derivative of the film along a direction
// (v_albedo, v_roughness) of the per-triangle parameters, at a fixed seed
// with detached sampling.  Contribution j of a path is
// c_j = prod_{v<j} w_v * (NEE factor at j), so its derivative is
// c_j * (sum_{v<j} d log w_v + d log f_nee(j)) along the direction: the sink
// carries the running sum over the continuations of the path.
struct TangentSink {
    static constexpr bool kWantsGradients = true;
    float* row;          // LDS primal row of the pixel
    float* drow;         // LDS tangent row
    const float* v_alb;  // direction (caller order), may be NULL
    const float* v_rough;
    float tang;          // sum of d log w of the path's continuations so far
    float steady;
    __device__ __forceinline__ float along(int k, float g_alb, float g_rough) const
    {
        if (k < 0) return 0.0f;
        float d = 0.0f;
        if (v_alb) d = v_alb[k] * g_alb;
        if (v_rough) d = fmaf(v_rough[k], g_rough, d);
        return d;
    }
    __device__ __forceinline__ void contribution(int, int k, float c, int bin, float, float g_alb_nee,
                                                 float g_rough_nee)
    {
        steady += c;
        if (bin < 0) return;
        atomicAdd(row + bin, c);
        atomicAdd(drow + bin, c * (tang + along(k, g_alb_nee, g_rough_nee)));
    }
    __device__ __forceinline__ void continuation(int, int k, float g_alb_c, float g_rough_c)
    {
        tang += along(k, g_alb_c, g_rough_c);
    }
};

template <class W>
__global__ void __launch_bounds__(256) k_render_tangent(SceneView S, LaunchArgs L)
{
    Tally<kPlain> tally;
    extern __shared__ float lds[];
    const uint32_t T = S.n_bins;
    const uint32_t TP = L.tile_pixels;
    float* tfilm = lds;
    float* tdfilm = lds + (size_t)TP * T;
    float* tsteady = tdfilm + (size_t)TP * T;
    LdsStack<W> stk{reinterpret_cast<W*>(tsteady + TP) + threadIdx.x, (int)blockDim.x};
    const uint32_t p0 = tile_first_pixel(S, L, TP);
    const uint32_t npix = min(TP, L.n_pixels - p0);
    for (uint32_t i = threadIdx.x; i < 2 * TP * T + TP; i += blockDim.x) lds[i] = 0.0f;
    __syncthreads();

    const uint32_t work = npix * L.spp;
    for (uint32_t w = threadIdx.x; w < work; w += blockDim.x) {
        const uint32_t pl = w / L.spp;
        const uint32_t s = w - pl * L.spp;
        TangentSink sink{tfilm + (size_t)pl * T, tdfilm + (size_t)pl * T, L.tan_albedo, L.tan_rough, 0.0f, 0.0f};
        trace_path(S, L, p0 + pl, L.sample_offset + s, stk, sink, tally);
        atomicAdd(tsteady + pl, sink.steady);
    }
    __syncthreads();

    const bool acc = (L.flags & kFlagAccumulate) != 0;
    const size_t base = (size_t)p0 * T;
    for (uint32_t i = threadIdx.x; i < npix * T; i += blockDim.x) {
        const float v = tfilm[i] * L.norm, dv = tdfilm[i] * L.norm;
        L.film[base + i] = acc ? L.film[base + i] + v : v;
        L.dfilm[base + i] = acc ? L.dfilm[base + i] + dv : dv;
    }
    if (L.steady && threadIdx.x < npix) {
        const uint32_t p = p0 + threadIdx.x;
        const float v = tsteady[threadIdx.x] * L.norm;
        L.steady[p] = acc ? L.steady[p] + v : v;
    }
}

template <class W, class Acc>
__global__ void __launch_bounds__(256) k_backward(SceneView S, LaunchArgs L)
{
    Tally<kPlain> tally;
    extern __shared__ float lds[];
    const uint32_t T = S.n_bins;
    const uint32_t TP = L.tile_pixels;
    const bool want_primal = L.primal != nullptr;
    Acc acc(lds, S, L);
    float* tdelta = lds + Acc::kFloats;
    float* tprimal = tdelta + (size_t)TP * T;
    LdsStack<W> stk{reinterpret_cast<W*>(tprimal + (want_primal ? (size_t)TP * T : 0)) + threadIdx.x,
                    (int)blockDim.x};
    const uint32_t p0 = tile_first_pixel(S, L, TP);
    const uint32_t npix = min(TP, L.n_pixels - p0);
    const size_t base = (size_t)p0 * T;
    for (uint32_t i = threadIdx.x; i < TP * T; i += blockDim.x) {
        tdelta[i] = (i < npix * T) ? L.grad_film[base + i] : 0.0f;
        if (want_primal) tprimal[i] = 0.0f;
    }
    acc.clear();
    __syncthreads();

    const uint32_t work = npix * L.spp;
    for (uint32_t w = threadIdx.x; w < work; w += blockDim.x) {
        const uint32_t pl = w / L.spp;
        const uint32_t s = w - pl * L.spp;
        const float* drow = tdelta + (size_t)pl * T;
        AdjointSumSink first{drow, L.norm, 0.0};
        trace_path(S, L, p0 + pl, L.sample_offset + s, stk, first, tally);
        AdjointScatterSink<Acc> second{drow, want_primal ? tprimal + (size_t)pl * T : nullptr, L.norm, first.total,
                                       0.0, &acc};
        trace_path(S, L, p0 + pl, L.sample_offset + s, stk, second, tally);
    }
    __syncthreads();
    acc.flush();
    if (want_primal)
        for (uint32_t i = threadIdx.x; i < npix * T; i += blockDim.x) L.primal[base + i] = tprimal[i] * L.norm;
}

// Single-trace adjoint for paths of at most kMaxCont continuations.  The
// sink keeps, per continuation vertex v, its triangle, d log f of the
// sampled direction, a_v times d log f of its connection, and R_v, the sum
// of a_j over the contributions after v (each contribution adds its a_j to
// every stashed vertex).  At the end of the path every stashed vertex adds
// a_v dlogf_nee + R_v dlogf_cont to its triangle: the same gradient as path
// replay, from one trace.  The stash lives in registers (static indices).
template <int kMaxCont, class Acc>
struct AdjointStashSink {
    static constexpr bool kWantsGradients = true;
    const float* delta;
    float* primal_row;
    float norm;
    Acc* acc;  // the workgroup's gradient table
    int nv = 0;
    int k[kMaxCont];
    float ca[kMaxCont], cr[kMaxCont], na[kMaxCont], nr[kMaxCont], R[kMaxCont];
    bool pending = false;  // connection term of the current vertex
    int pk = -1;
    float pa = 0.0f, pr = 0.0f;

    __device__ __forceinline__ void contribution(int, int kv, float c, int bin, float, float g_alb_nee,
                                                 float g_rough_nee)
    {
        if (bin < 0) return;
        if (primal_row) atomicAdd(primal_row + bin, c);
        const float a = (delta[bin] * c) * norm;
#pragma unroll
        for (int i = 0; i < kMaxCont; ++i)
            if (i < nv) R[i] += a;
        if (kv >= 0) {
            pending = true;
            pk = kv;
            pa = a * g_alb_nee;
            pr = a * g_rough_nee;
        }
    }
    __device__ __forceinline__ void continuation(int, int kv, float g_alb_c, float g_rough_c)
    {
        const bool mine = pending && pk == kv;
#pragma unroll
        for (int i = 0; i < kMaxCont; ++i)
            if (i == nv) {
                k[i] = kv;
                ca[i] = g_alb_c;
                cr[i] = g_rough_c;
                na[i] = mine ? pa : 0.0f;
                nr[i] = mine ? pr : 0.0f;
                R[i] = 0.0f;
            }
        ++nv;
        pending = false;
    }
    __device__ __forceinline__ void finish()
    {
        if (pending) acc->add(pk, (double)pa, (double)pr);
#pragma unroll
        for (int i = 0; i < kMaxCont; ++i)
            if (i < nv) {
                const double ga = (double)na[i] + (double)R[i] * (double)ca[i];
                const double gr = (double)nr[i] + (double)R[i] * (double)cr[i];
                acc->add(k[i], ga, gr);
            }
    }
};

// Four waves per SIMD (at most 128 VGPRs) instead of three.
template <int kMaxCont, class W, class Acc>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_backward_stash(SceneView S, LaunchArgs L)
{
    Tally<kPlain> tally;
    extern __shared__ float lds[];
    const uint32_t T = S.n_bins;
    const uint32_t TP = L.tile_pixels;
    const bool want_primal = L.primal != nullptr;
    Acc acc(lds, S, L);
    float* tdelta = lds + Acc::kFloats;
    float* tprimal = tdelta + (size_t)TP * T;
    LdsStack<W> stk{reinterpret_cast<W*>(tprimal + (want_primal ? (size_t)TP * T : 0)) + threadIdx.x,
                    (int)blockDim.x};
    const uint32_t p0 = tile_first_pixel(S, L, TP);
    const uint32_t npix = min(TP, L.n_pixels - p0);
    const size_t base = (size_t)p0 * T;
    for (uint32_t i = threadIdx.x; i < TP * T; i += blockDim.x) {
        tdelta[i] = (i < npix * T) ? L.grad_film[base + i] : 0.0f;
        if (want_primal) tprimal[i] = 0.0f;
    }
    acc.clear();
    __syncthreads();
    const uint32_t work = npix * L.spp;
    for (uint32_t w = threadIdx.x; w < work; w += blockDim.x) {
        const uint32_t pl = w / L.spp;
        const uint32_t s = w - pl * L.spp;
        AdjointStashSink<kMaxCont, Acc> sink;
        sink.delta = tdelta + (size_t)pl * T;
        sink.primal_row = want_primal ? tprimal + (size_t)pl * T : nullptr;
        sink.norm = L.norm;
        sink.acc = &acc;
        trace_path(S, L, p0 + pl, L.sample_offset + s, stk, sink, tally);
        sink.finish();
    }
    __syncthreads();
    acc.flush();
    if (want_primal)
        for (uint32_t i = threadIdx.x; i < npix * T; i += blockDim.x) L.primal[base + i] = tprimal[i] * L.norm;
}


__global__ void k_zero_f32(float* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_zero_f64(double* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_f64_to_f32(const double* __restrict__ s, float* __restrict__ d, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}

}  // namespace

size_t render_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes)
{
    return ((size_t)tile_pixels * n_bins + 2ull * tile_pixels) * sizeof(float) + (size_t)block * stack_bytes;
}

size_t wavefront_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes)
{
    return ((size_t)tile_pixels * n_bins + 2ull * tile_pixels) * sizeof(float) +
           (size_t)kWfWords * block * sizeof(float) + (size_t)block * stack_bytes;
}

size_t tangent_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes)
{
    return (2ull * tile_pixels * n_bins + tile_pixels) * sizeof(float) + (size_t)block * stack_bytes;
}

hipError_t launch_render_tangent(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream)
{
    const size_t lds = tangent_lds_bytes(L.tile_pixels, S.n_bins, block, stack_lane_bytes(S.n_tris, S.stack_depth));
    const dim3 grid((L.n_pixels + L.tile_pixels - 1) / L.tile_pixels);
    if (short_stack(S.n_tris))
        hipLaunchKernelGGL((k_render_tangent<uint16_t>), grid, dim3(block), lds, stream, S, L);
    else
        hipLaunchKernelGGL((k_render_tangent<uint32_t>), grid, dim3(block), lds, stream, S, L);
    return hipGetLastError();
}

size_t backward_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes, bool primal,
                          bool fixed)
{
    return (size_t)(fixed ? GradFixed::kFloats : GradF64::kFloats) * sizeof(float) +
           (size_t)tile_pixels * n_bins * sizeof(float) * (primal ? 2 : 1) + (size_t)block * stack_bytes;
}

size_t fixed_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes)
{
    return ((size_t)tile_pixels * n_bins + 2ull * tile_pixels) * 2 * sizeof(unsigned long long) +
           (size_t)block * stack_bytes;
}

size_t deferred_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes)
{
    return ((size_t)tile_pixels * n_bins + 2ull * tile_pixels + deferred_words(block)) *
               sizeof(float) +
           (size_t)block * stack_bytes;
}

size_t batch_lds_bytes(uint32_t film_words, uint32_t block, uint32_t stack_bytes, bool deferred)
{
    return ((size_t)film_words + (deferred ? deferred_words(block) : 0)) * sizeof(float) +
           (size_t)block * stack_bytes;
}

namespace {

uint32_t tiles_of(const LaunchArgs& L) { return (L.n_pixels + L.tile_pixels - 1) / L.tile_pixels; }

// the build a forward launch runs: recording when the launch carries a
// record buffer, counting when it carries counters, plain otherwise
int mode_of(const LaunchArgs& L, const unsigned long long* counts)
{
    return L.record_count ? kRecording : (counts ? kCounting : kPlain);
}

template <class W>
void launch_render_w(const SceneView& S, const LaunchArgs& L, uint32_t block, size_t lds, hipStream_t stream,
                     unsigned long long* counts)
{
    const dim3 grid(tiles_of(L));
    switch (mode_of(L, counts)) {
    case kRecording: hipLaunchKernelGGL((k_render<kRecording, W>), grid, dim3(block), lds, stream, S, L, counts); break;
    case kCounting: hipLaunchKernelGGL((k_render<kCounting, W>), grid, dim3(block), lds, stream, S, L, counts); break;
    default: hipLaunchKernelGGL((k_render<kPlain, W>), grid, dim3(block), lds, stream, S, L, counts);
    }
}

template <class W>
void launch_hbm_w(const SceneView& S, const LaunchArgs& L, uint32_t block, size_t lds, hipStream_t stream,
                  unsigned long long* counts)
{
    const dim3 grid(tiles_of(L));
    switch (mode_of(L, counts)) {
    case kRecording: hipLaunchKernelGGL((k_render_hbm<kRecording, W>), grid, dim3(block), lds, stream, S, L, counts); break;
    case kCounting: hipLaunchKernelGGL((k_render_hbm<kCounting, W>), grid, dim3(block), lds, stream, S, L, counts); break;
    default: hipLaunchKernelGGL((k_render_hbm<kPlain, W>), grid, dim3(block), lds, stream, S, L, counts);
    }
}

void launch_fill_zero(float* p, size_t n, hipStream_t stream)
{
    const unsigned g = (unsigned)std::min<size_t>(4096, (n + 255) / 256 + 1);
    hipLaunchKernelGGL(k_zero_f32, dim3(g), dim3(256), 0, stream, p, n);
}

template <class W>
void launch_wavefront_w(const SceneView& S, const LaunchArgs& L, uint32_t block, size_t lds, hipStream_t stream,
                        unsigned long long* counts)
{
    const dim3 grid(tiles_of(L));
    switch (mode_of(L, counts)) {
    case kRecording:
        hipLaunchKernelGGL((k_render_wf<kRecording, W>), grid, dim3(block), lds, stream, S, L, counts);
        break;
    case kCounting: hipLaunchKernelGGL((k_render_wf<kCounting, W>), grid, dim3(block), lds, stream, S, L, counts); break;
    default: hipLaunchKernelGGL((k_render_wf<kPlain, W>), grid, dim3(block), lds, stream, S, L, counts);
    }
}

template <class W, bool kArea>
void launch_deferred_wa(const SceneView& S, const LaunchArgs& L, uint32_t block, size_t lds, hipStream_t stream,
                        unsigned long long* counts)
{
    const dim3 grid(tiles_of(L) * L.chunks);
    switch (mode_of(L, counts)) {
    case kRecording:
        hipLaunchKernelGGL((k_render_deferred<kRecording, W, kArea>), grid, dim3(block), lds, stream, S, L, counts);
        break;
    case kCounting:
        hipLaunchKernelGGL((k_render_deferred<kCounting, W, kArea>), grid, dim3(block), lds, stream, S, L, counts);
        break;
    default: hipLaunchKernelGGL((k_render_deferred<kPlain, W, kArea>), grid, dim3(block), lds, stream, S, L, counts);
    }
}

template <class W>
void launch_deferred_w(const SceneView& S, const LaunchArgs& L, uint32_t block, size_t lds, hipStream_t stream,
                       unsigned long long* counts)
{
    if (L.flags & kFlagNlosArea)
        launch_deferred_wa<W, true>(S, L, block, lds, stream, counts);
    else
        launch_deferred_wa<W, false>(S, L, block, lds, stream, counts);
}



template <class W, class Acc>
void launch_backward_w(const SceneView& S, const LaunchArgs& L, uint32_t block, int max_cont, size_t lds,
                       hipStream_t stream)
{
    if (max_cont == 2)
        hipLaunchKernelGGL((k_backward_stash<2, W, Acc>), dim3(tiles_of(L)), dim3(block), lds, stream, S, L);
    else if (max_cont == 7)
        hipLaunchKernelGGL((k_backward_stash<7, W, Acc>), dim3(tiles_of(L)), dim3(block), lds, stream, S, L);
    else
        hipLaunchKernelGGL((k_backward<W, Acc>), dim3(tiles_of(L)), dim3(block), lds, stream, S, L);
}


}  // namespace

hipError_t launch_render(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                         unsigned long long* counts)
{
    const uint32_t words = L.n_freq ? 2 * L.n_freq : S.n_bins;
    const size_t lds = render_lds_bytes(L.tile_pixels, words, block, stack_lane_bytes(S.n_tris, S.stack_depth));
    if (short_stack(S.n_tris))
        launch_render_w<uint16_t>(S, L, block, lds, stream, counts);
    else
        launch_render_w<uint32_t>(S, L, block, lds, stream, counts);
    return hipGetLastError();
}

size_t hbm_lds_bytes(uint32_t block, uint32_t stack_bytes) { return (size_t)block * stack_bytes; }

bool split_stack_enabled()
{
    const char* v = std::getenv("TRHIP_SPLIT_STACK");
    return !(v && v[0] == '0' && v[1] == '\0');
}

hipError_t launch_render_hbm(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                             unsigned long long* counts)
{
    if ((L.flags & kFlagAccumulate) == 0) {
        launch_fill_zero(L.film, (size_t)L.n_pixels * S.n_bins, stream);
        if (L.steady) launch_fill_zero(L.steady, L.n_pixels, stream);
        if (L.oow) launch_fill_zero(L.oow, L.n_pixels, stream);
    }
    const size_t lds = hbm_lds_bytes(block, hbm_stack_lane_bytes(S.n_tris, S.stack_depth));
    if (short_stack(S.n_tris)) {
        launch_hbm_w<uint16_t>(S, L, block, lds, stream, counts);
    } else if (split_stack(S.n_tris, S.stack_depth)) {
        const dim3 grid(tiles_of(L));
        switch (mode_of(L, counts)) {
        case kRecording:
            hipLaunchKernelGGL((k_render_hbm_split<kRecording>), grid, dim3(block), lds, stream, S, L, counts);
            break;
        case kCounting:
            hipLaunchKernelGGL((k_render_hbm_split<kCounting>), grid, dim3(block), lds, stream, S, L, counts);
            break;
        default: hipLaunchKernelGGL((k_render_hbm_split<kPlain>), grid, dim3(block), lds, stream, S, L, counts);
        }
    } else {
        launch_hbm_w<uint32_t>(S, L, block, lds, stream, counts);
    }
    return hipGetLastError();
}

hipError_t launch_render_wavefront(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                                   unsigned long long* counts)
{
    const size_t lds =
        wavefront_lds_bytes(L.tile_pixels, S.n_bins, block, stack_lane_bytes(S.n_tris, S.stack_depth));
    if (short_stack(S.n_tris))
        launch_wavefront_w<uint16_t>(S, L, block, lds, stream, counts);
    else
        launch_wavefront_w<uint32_t>(S, L, block, lds, stream, counts);
    return hipGetLastError();
}

// The deferred form may split a tile's samples into chunks of whole sort
// batches (the caller sets L.chunks, L.chunk_spp and the scratch, see
// deferred_chunks): shorter workgroups shrink the tail of the launch.
hipError_t launch_render_deferred(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                                  unsigned long long* counts)
{
    const uint32_t words = L.n_freq ? 2 * L.n_freq : S.n_bins;
    const size_t lds = deferred_lds_bytes(L.tile_pixels, words, block, stack_lane_bytes(S.n_tris, S.stack_depth));
    if (short_stack(S.n_tris))
        launch_deferred_w<uint16_t>(S, L, block, lds, stream, counts);
    else
        launch_deferred_w<uint32_t>(S, L, block, lds, stream, counts);
    return hipGetLastError();
}

namespace {
// film += sum over planes c of plane[c] (the partial tiles of chunks 1..),
// in chunk order; steady and oow likewise when present
__global__ void k_add_planes(float* __restrict__ film, float* __restrict__ steady, float* __restrict__ oow,
                             const float* __restrict__ planes, size_t film_n, uint32_t n_pixels, uint32_t n_planes)
{
    const size_t per = film_n + 2ull * n_pixels;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x) {
        float* dst = i < film_n ? film + i : (i < film_n + n_pixels ? steady : oow);
        if (i >= film_n) {
            if (!dst) continue;
            dst += (i - film_n) % n_pixels;
        }
        float v = *dst;
        for (uint32_t c = 0; c < n_planes; ++c) v = v + planes[c * per + i];
        *dst = v;
    }
}
}  // namespace

hipError_t launch_add_planes(const LaunchArgs& L, uint32_t words, hipStream_t stream)
{
    const size_t n = (size_t)L.n_pixels * words + 2ull * L.n_pixels;
    const unsigned g = (unsigned)std::min<size_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_add_planes, dim3(g), dim3(256), 0, stream, L.film, L.steady, L.oow, L.chunk_scratch,
                       (size_t)L.n_pixels * words, L.n_pixels, L.chunks - 1);
    return hipGetLastError();
}

// Sample chunks of the deferred form: a tile with more samples than one sort
// batch (kSortPerLane * block) is split into at most kMaxChunks chunks of
// whole batches, one workgroup each (measured on the confocal workload, 4096
// samples per pixel in two chunks: +4.5%; one workgroup per half batch loses
// more to per-workgroup work than it gains).
uint32_t deferred_chunks(uint32_t spp, uint32_t block, uint32_t* chunk_spp)
{
    const uint32_t c = kSortPerLane * block;
    uint32_t chunks = (spp + c - 1) / c;
    if (chunks > kMaxChunks) chunks = kMaxChunks;
    if (chunks < 1) chunks = 1;
    const uint32_t batches = (spp + c - 1) / c;
    *chunk_spp = ((batches + chunks - 1) / chunks) * c;
    return (spp + *chunk_spp - 1) / *chunk_spp;
}

hipError_t launch_backward(const SceneView& S, const LaunchArgs& L, uint32_t block, int max_cont, hipStream_t stream)
{
    const bool fixed = L.g_fixed != nullptr;
    const size_t lds = backward_lds_bytes(L.tile_pixels, S.n_bins, block, stack_lane_bytes(S.n_tris, S.stack_depth),
                                          L.primal != nullptr, fixed);
    if (short_stack(S.n_tris)) {
        if (fixed) launch_backward_w<uint16_t, GradFixed>(S, L, block, max_cont, lds, stream);
        else launch_backward_w<uint16_t, GradF64>(S, L, block, max_cont, lds, stream);
    } else {
        if (fixed) launch_backward_w<uint32_t, GradFixed>(S, L, block, max_cont, lds, stream);
        else launch_backward_w<uint32_t, GradF64>(S, L, block, max_cont, lds, stream);
    }
    return hipGetLastError();
}

hipError_t launch_render_fixed(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream)
{
    const size_t lds = fixed_lds_bytes(L.tile_pixels, S.n_bins, block, stack_lane_bytes(S.n_tris, S.stack_depth));
    const dim3 grid(tiles_of(L));
    if (short_stack(S.n_tris))
        hipLaunchKernelGGL((k_render_fixed<uint16_t>), grid, dim3(block), lds, stream, S, L);
    else
        hipLaunchKernelGGL((k_render_fixed<uint32_t>), grid, dim3(block), lds, stream, S, L);
    return hipGetLastError();
}

size_t fixed_film_words(uint32_t n_pixels, uint32_t n_bins)
{
    return (size_t)kLimbWords * ((size_t)n_pixels * n_bins + 2ull * n_pixels);
}

hipError_t launch_render_fixed_hbm(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream)
{
    launch_fill_zero(reinterpret_cast<float*>(L.fixed_film), 2 * fixed_film_words(L.n_pixels, S.n_bins), stream);
    const dim3 grid(tiles_of(L));
    const size_t lds = hbm_lds_bytes(block, hbm_stack_lane_bytes(S.n_tris, S.stack_depth));
    if (short_stack(S.n_tris))
        hipLaunchKernelGGL((k_render_fixed_hbm<uint16_t>), grid, dim3(block), lds, stream, S, L);
    else if (split_stack(S.n_tris, S.stack_depth))
        hipLaunchKernelGGL(k_render_fixed_hbm_split, grid, dim3(block), lds, stream, S, L);
    else
        hipLaunchKernelGGL((k_render_fixed_hbm<uint32_t>), grid, dim3(block), lds, stream, S, L);
    const size_t n = (size_t)L.n_pixels * S.n_bins + 2ull * L.n_pixels;
    const unsigned g = (unsigned)std::min<size_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_fixed_film_out, dim3(g), dim3(256), 0, stream, L, S.n_bins);
    return hipGetLastError();
}

namespace {
__global__ void k_fixed_to_f32(const unsigned long long* __restrict__ s, float* __restrict__ d, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = (float)from_fixed(s[2 * i], s[2 * i + 1]);
}
}  // namespace

hipError_t launch_fixed_to_f32(const unsigned long long* src, float* dst, size_t n, hipStream_t stream)
{
    const unsigned g = (unsigned)std::min<size_t>(1024, (n + 255) / 256 + 1);
    hipLaunchKernelGGL(k_fixed_to_f32, dim3(g), dim3(256), 0, stream, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchTables& B, uint32_t groups, uint32_t block, uint32_t stack_depth, bool short_links,
                        bool deferred, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset_cursor, dim3(1), dim3(64), 0, stream, B.cursor);
    const size_t lds = batch_lds_bytes(B.film_words, block, stack_depth * (short_links ? 2u : 4u), deferred);
    if (short_links) {
        if (deferred) hipLaunchKernelGGL((k_batch<true, uint16_t>), dim3(groups), dim3(block), lds, stream, B);
        else hipLaunchKernelGGL((k_batch<false, uint16_t>), dim3(groups), dim3(block), lds, stream, B);
    } else {
        if (deferred) hipLaunchKernelGGL((k_batch<true, uint32_t>), dim3(groups), dim3(block), lds, stream, B);
        else hipLaunchKernelGGL((k_batch<false, uint32_t>), dim3(groups), dim3(block), lds, stream, B);
    }
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, size_t n, hipStream_t stream)
{
    const unsigned g = (unsigned)std::min<size_t>(1024, (n + 255) / 256 + 1);
    hipLaunchKernelGGL(k_zero_f64, dim3(g), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double* src, float* dst, size_t n, hipStream_t stream)
{
    const unsigned g = (unsigned)std::min<size_t>(1024, (n + 255) / 256 + 1);
    hipLaunchKernelGGL(k_f64_to_f32, dim3(g), dim3(256), 0, stream, src, dst, n);
    return hipGetLastError();
}

}  // namespace trhip
