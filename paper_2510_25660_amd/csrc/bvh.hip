// bvh.hip -- linear BVH built on the device.
//
// Triangle boxes are padded by pad = (largest |coordinate|) * 2^-16 (exact
// scaling), Morton codes of the box centres (10 bits per axis) are radix
// sorted, the hierarchy over the sorted codes is emitted in parallel (one
// thread per internal node, Karras, "Maximizing Parallelism in the
// Construction of BVHs, Octrees, and k-d Trees", HPG 2012), boxes are
// refitted bottom-up with one atomic arrival counter per node, and the
// result is laid out as 64-byte two-child nodes plus 48-byte triangles in
// Morton order (scenes with more than 32,768 triangles: 32-byte nodes with
// FP16 child boxes rounded outward, plus 64-byte triangles that carry their
// padded boxes).  Every box is a union of padded triangle boxes, so a box
// always contains the padded boxes of all triangles below it.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <utility>

#include "internal.h"
#include "scene_view.h"

namespace trhip {

namespace {

__device__ __forceinline__ uint32_t ordered_bits(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// stats[0] = max |coordinate| bits, stats[1..3] centre min (ordered),
// stats[4..6] centre max (ordered)
__global__ void k_scene_stats(const float* __restrict__ tri9, uint32_t nt, uint32_t* __restrict__ stats)
{
    __shared__ uint32_t red[7];
    if (threadIdx.x < 7) red[threadIdx.x] = (threadIdx.x == 0) ? 0u : (threadIdx.x < 4 ? 0xffffffffu : 0u);
    __syncthreads();
    uint32_t mabs = 0u;
    uint32_t cmin[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, cmax[3] = {0u, 0u, 0u};
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
        const float* t = tri9 + 9ull * k;
        for (int a = 0; a < 3; ++a) {
            const float x0 = t[a], x1 = t[3 + a], x2 = t[6 + a];
            mabs = max(mabs, __float_as_uint(fmaxf(fmaxf(fabsf(x0), fabsf(x1)), fabsf(x2))));
            const float lo = fminf(fminf(x0, x1), x2), hi = fmaxf(fmaxf(x0, x1), x2);
            const uint32_t c = ordered_bits(0.5f * (lo + hi));
            cmin[a] = min(cmin[a], c);
            cmax[a] = max(cmax[a], c);
        }
    }
    atomicMax(&red[0], mabs);
    for (int a = 0; a < 3; ++a) {
        atomicMin(&red[1 + a], cmin[a]);
        atomicMax(&red[4 + a], cmax[a]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(&stats[0], red[0]);
        for (int a = 0; a < 3; ++a) {
            atomicMin(&stats[1 + a], red[1 + a]);
            atomicMax(&stats[4 + a], red[4 + a]);
        }
    }
}

__global__ void k_init_stats(uint32_t* stats)
{
    if (threadIdx.x < 7) stats[threadIdx.x] = (threadIdx.x == 0) ? 0u : (threadIdx.x < 4 ? 0xffffffffu : 0u);
}

__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v = (v * 0x00010001u) & 0xFF0000FFu;
    v = (v * 0x00000101u) & 0x0F00F00Fu;
    v = (v * 0x00000011u) & 0xC30C30C3u;
    v = (v * 0x00000005u) & 0x49249249u;
    return v;
}

// padded boxes (caller order) and Morton codes of the unpadded box centres
__global__ void k_boxes_codes(const float* __restrict__ tri9, uint32_t nt, const uint32_t* __restrict__ stats,
                              float* __restrict__ box, uint32_t* __restrict__ codes, uint32_t* __restrict__ ids)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const float pad = __uint_as_float(stats[0]) * 0x1p-16f;
    const float* t = tri9 + 9ull * k;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        const float x0 = t[a], x1 = t[3 + a], x2 = t[6 + a];
        const float lo = fminf(fminf(x0, x1), x2), hi = fmaxf(fmaxf(x0, x1), x2);
        box[6ull * k + a] = lo - pad;
        box[6ull * k + 3 + a] = hi + pad;
        const float cmin = from_ordered(stats[1 + a]), cmax = from_ordered(stats[4 + a]);
        const float ext = cmax - cmin;
        const float rel = (ext > 0.0f) ? (0.5f * (lo + hi) - cmin) / ext : 0.5f;
        q[a] = (uint32_t)fminf(fmaxf(rel * 1024.0f, 0.0f), 1023.0f);
    }
    codes[k] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    ids[k] = k;
}

// common-prefix length of sorted codes i and j (index tie-break for equal codes)
__device__ __forceinline__ int prefix_len(const uint32_t* __restrict__ codes, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint32_t a = codes[i], b = codes[j];
    if (a == b) return 32 + __clz((uint32_t)i ^ (uint32_t)j);
    return __clz(a ^ b);
}

// internal node i spans a contiguous key range; children are internal
// nodes (>= 0) or leaves (~sorted index)
__global__ void k_hierarchy(const uint32_t* __restrict__ codes, int n, int32_t* __restrict__ child,
                            int32_t* __restrict__ parent_int, int32_t* __restrict__ parent_leaf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (prefix_len(codes, n, i, i + 1) - prefix_len(codes, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = prefix_len(codes, n, i, i - d);
    long long lmax = 2;
    while (prefix_len(codes, n, i, (int)(i + lmax * d)) > dmin) lmax *= 2;
    long long l = 0;
    for (long long t = lmax / 2; t >= 1; t /= 2)
        if (prefix_len(codes, n, i, (int)(i + (l + t) * d)) > dmin) l += t;
    const int j = (int)(i + l * d);
    const int dnode = prefix_len(codes, n, i, j);
    int s = 0;
    long long step = l;
    do {
        step = (step + 1) / 2;
        if (prefix_len(codes, n, i, (int)(i + (s + step) * d)) > dnode) s += (int)step;
    } while (step > 1);
    const int split = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    const int c0 = (lo == split) ? ~split : split;
    const int c1 = (hi == split + 1) ? ~(split + 1) : (split + 1);
    child[2 * i] = c0;
    child[2 * i + 1] = c1;
    if (c0 < 0) parent_leaf[~c0] = i; else parent_int[c0] = i;
    if (c1 < 0) parent_leaf[~c1] = i; else parent_int[c1] = i;
}

// internal-node boxes are read through volatile: during the refit they were
// written by another wave, possibly on another compute unit
__device__ __forceinline__ void child_box(const int32_t c, const float* __restrict__ tri_box,
                                          const uint32_t* __restrict__ ids, const volatile float* node_box,
                                          float lo[3], float hi[3])
{
    if (c < 0) {
        const float* b = tri_box + 6ull * ids[~c];
        for (int a = 0; a < 3; ++a) {
            lo[a] = b[a];
            hi[a] = b[3 + a];
        }
    } else {
        const volatile float* b = node_box + 6ull * c;
        for (int a = 0; a < 3; ++a) {
            lo[a] = b[a];
            hi[a] = b[3 + a];
        }
    }
}

// bottom-up refit: the second arrival at a node merges both children
__global__ void k_refit(int n, const int32_t* __restrict__ child, const int32_t* __restrict__ parent_int,
                        const int32_t* __restrict__ parent_leaf, const float* __restrict__ tri_box,
                        const uint32_t* __restrict__ ids, float* node_box, uint32_t* arrivals)
{
    const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
    if (leaf >= n) return;
    int node = parent_leaf[leaf];
    for (int guard = 0; node >= 0 && guard < n; ++guard) {
        __threadfence();
        if (atomicAdd(&arrivals[node], 1u) == 0u) return;
        __threadfence();
        float l0[3], h0[3], l1[3], h1[3];
        child_box(child[2 * node], tri_box, ids, node_box, l0, h0);
        child_box(child[2 * node + 1], tri_box, ids, node_box, l1, h1);
        volatile float* nb = node_box + 6ull * node;
        for (int a = 0; a < 3; ++a) {
            nb[a] = fminf(l0[a], l1[a]);
            nb[3 + a] = fmaxf(h0[a], h1[a]);
        }
        node = parent_int[node];
    }
}

__global__ void k_layout(int n, const int32_t* __restrict__ child, const float* __restrict__ tri_box,
                         const uint32_t* __restrict__ ids, const float* __restrict__ node_box,
                         BvhNode* __restrict__ nodes)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    float l0[3], h0[3], l1[3], h1[3];
    const int32_t c0 = child[2 * i], c1 = child[2 * i + 1];
    child_box(c0, tri_box, ids, node_box, l0, h0);
    child_box(c1, tri_box, ids, node_box, l1, h1);
    BvhNode nd;
    nd.lo0x = l0[0]; nd.lo0y = l0[1]; nd.lo0z = l0[2]; nd.hi0x = h0[0];
    nd.hi0y = h0[1]; nd.hi0z = h0[2]; nd.lo1x = l1[0]; nd.lo1y = l1[1];
    nd.lo1z = l1[2]; nd.hi1x = h1[0]; nd.hi1y = h1[1]; nd.hi1z = h1[2];
    nd.child0 = c0; nd.child1 = c1; nd.unused0 = 0; nd.unused1 = 0;
    nodes[i] = nd;
}

// FP16 bit patterns of the largest half <= x and the smallest half >= x
// (round to nearest, then one step toward the bound when it overshot; the
// conversion back to FP32 is exact)
__device__ __forceinline__ uint16_t half_bits(_Float16 h) { return __builtin_bit_cast(uint16_t, h); }
__device__ __forceinline__ float half_value(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
__device__ __forceinline__ uint16_t half_down(float x)
{
    uint16_t b = half_bits((_Float16)x);
    if (half_value(b) > x) b = (b == 0x0000u) ? (uint16_t)0x8001u : (b & 0x8000u) ? (uint16_t)(b + 1u) : (uint16_t)(b - 1u);
    return b;
}
__device__ __forceinline__ uint16_t half_up(float x)
{
    uint16_t b = half_bits((_Float16)x);
    if (half_value(b) < x) b = (b == 0x8000u) ? (uint16_t)0x0001u : (b & 0x8000u) ? (uint16_t)(b - 1u) : (uint16_t)(b + 1u);
    return b;
}

__global__ void k_layout_compact(int n, const int32_t* __restrict__ child, const float* __restrict__ tri_box,
                                 const uint32_t* __restrict__ ids, const float* __restrict__ node_box,
                                 CompactNode* __restrict__ nodes)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    float l0[3], h0[3], l1[3], h1[3];
    const int32_t c0 = child[2 * i], c1 = child[2 * i + 1];
    child_box(c0, tri_box, ids, node_box, l0, h0);
    child_box(c1, tri_box, ids, node_box, l1, h1);
    CompactNode nd;
    for (int a = 0; a < 3; ++a) {
        nd.box[2 * a] = half_down(l0[a]);
        nd.box[2 * a + 1] = half_up(h0[a]);
        nd.box[6 + 2 * a] = half_down(l1[a]);
        nd.box[6 + 2 * a + 1] = half_up(h1[a]);
    }
    nd.child0 = c0;
    nd.child1 = c1;
    nodes[i] = nd;
}

// compact layout: the record with the triangle's padded box
__global__ void k_tris_box(int n, const float* __restrict__ tri9, const uint32_t* __restrict__ ids,
                           const float* __restrict__ tri_box, TriRecBox* __restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t k = ids[j];
    const float* t = tri9 + 9ull * k;
    const float* b = tri_box + 6ull * k;
    TriRecBox r;
    r.v0x = t[0]; r.v0y = t[1]; r.v0z = t[2];
    r.prim = k;
    r.e1x = t[3] - t[0]; r.e1y = t[4] - t[1]; r.e1z = t[5] - t[2];
    r.e2x = t[6] - t[0]; r.e2y = t[7] - t[1]; r.e2z = t[8] - t[2];
    r.lox = b[0]; r.loy = b[1]; r.loz = b[2];
    r.hix = b[3]; r.hiy = b[4]; r.hiz = b[5];
    out[j] = r;
}

__global__ void k_tris(int n, const float* __restrict__ tri9, const uint32_t* __restrict__ ids,
                       TriRec* __restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t k = ids[j];
    const float* t = tri9 + 9ull * k;
    TriRec r;
    r.v0x = t[0]; r.v0y = t[1]; r.v0z = t[2];
    r.prim = k;
    r.e1x = t[3] - t[0]; r.e1y = t[4] - t[1]; r.e1z = t[5] - t[2];
    r.e2x = t[6] - t[0]; r.e2y = t[7] - t[1]; r.e2z = t[8] - t[2];
    r.unused0 = 0.0f; r.unused1 = 0.0f;
    out[j] = r;
}

// depth (edges) of every leaf; max into *depth
__global__ void k_depth(int n, const int32_t* __restrict__ parent_int, const int32_t* __restrict__ parent_leaf,
                        uint32_t* depth)
{
    const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
    if (leaf >= n) return;
    uint32_t d = 0;
    int node = parent_leaf[leaf];
    for (int guard = 0; node >= 0 && guard < n; ++guard) {
        ++d;
        node = parent_int[node];
    }
    atomicMax(depth, d);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Locally-ordered clustering over the Morton order (Meister and Bittner,
// "Parallel Locally-Ordered Clustering for Bounding Volume Hierarchy
// Construction", IEEE TVCG 2018): every cluster picks, among its kPlocRadius
// neighbours on each side in the current order, the one whose union box has
// the smallest surface area; mutual nearest neighbours merge into a new
// internal node; survivors are compacted in order; repeat until one cluster.
// A radius of 6 against 16: 6.6 % fewer node visits on a confocal scan
// (+3.5 %), 1.3 % fewer on a 1M-triangle scene (+0.8 %).
// ---------------------------------------------------------------------------
constexpr int kPlocRadius = 6;

__device__ __forceinline__ float half_area(float lx, float ly, float lz, float hx, float hy, float hz)
{
    const float dx = hx - lx, dy = hy - ly, dz = hz - lz;
    return dx * dy + dy * dz + dz * dx;
}

__global__ void k_ploc_init(int n, const float* __restrict__ tri_box, const uint32_t* __restrict__ ids,
                            int32_t* __restrict__ c_node, float* __restrict__ c_box)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    c_node[j] = ~j;
    const float* b = tri_box + 6ull * ids[j];
    for (int a = 0; a < 6; ++a) c_box[6ull * j + a] = b[a];
}

// nearest neighbour in the window; boxes of the block and its halo in LDS
__global__ void __launch_bounds__(256) k_ploc_nn(int nc, const float* __restrict__ c_box, int32_t* __restrict__ nn)
{
    __shared__ float sb[(256 + 2 * kPlocRadius) * 6];
    const int first = blockIdx.x * 256 - kPlocRadius;
    for (int k = threadIdx.x; k < (256 + 2 * kPlocRadius) * 6; k += 256) {
        const int c = first + k / 6;
        sb[k] = (c >= 0 && c < nc) ? c_box[6ll * c + k % 6] : 0.0f;
    }
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nc) return;
    const float* bi = sb + 6 * (threadIdx.x + kPlocRadius);
    float best = __builtin_huge_valf();
    int arg = -1;
    const int lo = max(0, i - kPlocRadius), hi = min(nc - 1, i + kPlocRadius);
    for (int j = lo; j <= hi; ++j) {
        if (j == i) continue;
        const float* bj = sb + 6 * (j - first);
        const float a = half_area(fminf(bi[0], bj[0]), fminf(bi[1], bj[1]), fminf(bi[2], bj[2]), fmaxf(bi[3], bj[3]),
                                  fmaxf(bi[4], bj[4]), fmaxf(bi[5], bj[5]));
        if (a < best) {  // ties keep the smaller index (scanned first)
            best = a;
            arg = j;
        }
    }
    nn[i] = arg;
}

// merge flags: 1 where cluster i starts a new node (mutual pair, i < partner);
// keep flags: 1 where cluster i survives (merged-into or unpaired)
__global__ void k_ploc_flags(int nc, const int32_t* __restrict__ nn, int force_pairs, uint32_t* __restrict__ mflag,
                             uint32_t* __restrict__ keep)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    int j = nn[i];
    bool mutual = j >= 0 && nn[j] == i;
    if (force_pairs) {  // progress guarantee: pair neighbours (2k, 2k+1)
        j = (i & 1) ? i - 1 : (i + 1 < nc ? i + 1 : -1);
        mutual = j >= 0;
    }
    mflag[i] = (mutual && i < j) ? 1u : 0u;
    keep[i] = (mutual && i > j) ? 0u : 1u;
}

__global__ void k_ploc_merge(int nc, const int32_t* __restrict__ nn, int force_pairs, const uint32_t* __restrict__ mflag,
                             const uint32_t* __restrict__ moff, const uint32_t* __restrict__ koff,
                             const int32_t* __restrict__ c_node, const float* __restrict__ c_box, int node_base,
                             int32_t* __restrict__ child, float* __restrict__ node_box, int32_t* __restrict__ c_node2,
                             float* __restrict__ c_box2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    int j = nn[i];
    bool mutual = j >= 0 && nn[j] == i;
    if (force_pairs) {
        j = (i & 1) ? i - 1 : (i + 1 < nc ? i + 1 : -1);
        mutual = j >= 0;
    }
    if (mutual && i > j) return;  // absorbed by its partner
    const int out = (int)koff[i];
    if (mflag[i]) {
        const int idx = node_base + (int)moff[i];
        child[2 * idx] = c_node[i];
        child[2 * idx + 1] = c_node[j];
        float b[6];
        for (int a = 0; a < 3; ++a) {
            b[a] = fminf(c_box[6ll * i + a], c_box[6ll * j + a]);
            b[3 + a] = fmaxf(c_box[6ll * i + 3 + a], c_box[6ll * j + 3 + a]);
        }
        for (int a = 0; a < 6; ++a) {
            node_box[6ll * idx + a] = b[a];
            c_box2[6ll * out + a] = b[a];
        }
        c_node2[out] = idx;
    } else {
        c_node2[out] = c_node[i];
        for (int a = 0; a < 6; ++a) c_box2[6ll * out + a] = c_box[6ll * i + a];
    }
}

__global__ void k_parents(int ni, const int32_t* __restrict__ child, int32_t* __restrict__ parent_int,
                          int32_t* __restrict__ parent_leaf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    for (int s = 0; s < 2; ++s) {
        const int c = child[2 * i + s];
        if (c < 0) parent_leaf[~c] = i;
        else parent_int[c] = i;
    }
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

#define TR_CHECK(expr)                   \
    do {                                 \
        hipError_t e_ = (expr);          \
        if (e_ != hipSuccess) {          \
            err = e_;                    \
            goto done;                   \
        }                                \
    } while (0)

hipError_t build_bvh(const float* d_tri9, uint32_t nt, int builder, hipStream_t stream, BvhBuild* out)
{
    hipError_t err = hipSuccess;
    const int n = (int)nt;
    uint32_t *stats = nullptr, *codes = nullptr, *codes_sorted = nullptr, *ids = nullptr, *ids_sorted = nullptr;
    uint32_t *arrivals = nullptr, *depth = nullptr;
    int32_t *c_node = nullptr, *c_node2 = nullptr, *nn = nullptr;
    float *c_box = nullptr, *c_box2 = nullptr;
    uint32_t *mflag = nullptr, *keep = nullptr, *moff = nullptr, *koff = nullptr;
    void* scan_temp = nullptr;
    size_t scan_bytes = 0;
    float *tri_box = nullptr, *node_box = nullptr;
    int32_t *child = nullptr, *parent_int = nullptr, *parent_leaf = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    uint32_t host_stats[7] = {0};
    uint32_t host_depth = 0;
    const int ni = n > 1 ? n - 1 : 1;
    out->nodes = nullptr;
    out->tris = nullptr;

    TR_CHECK(hipMalloc(&stats, 7 * sizeof(uint32_t)));
    TR_CHECK(hipMalloc(&codes, nt * sizeof(uint32_t)));
    TR_CHECK(hipMalloc(&codes_sorted, nt * sizeof(uint32_t)));
    TR_CHECK(hipMalloc(&ids, nt * sizeof(uint32_t)));
    TR_CHECK(hipMalloc(&ids_sorted, nt * sizeof(uint32_t)));
    TR_CHECK(hipMalloc(&tri_box, 6ull * nt * sizeof(float)));
    TR_CHECK(hipMalloc(&node_box, 6ull * ni * sizeof(float)));
    TR_CHECK(hipMalloc(&child, 2ull * ni * sizeof(int32_t)));
    TR_CHECK(hipMalloc(&parent_int, (size_t)ni * sizeof(int32_t)));
    TR_CHECK(hipMalloc(&parent_leaf, (size_t)nt * sizeof(int32_t)));
    TR_CHECK(hipMalloc(&arrivals, (size_t)ni * sizeof(uint32_t)));
    TR_CHECK(hipMalloc(&depth, sizeof(uint32_t)));
    out->compact = !short_stack(nt);
    TR_CHECK(hipMalloc(&out->nodes, (size_t)ni * (out->compact ? sizeof(CompactNode) : sizeof(BvhNode))));
    TR_CHECK(hipMalloc(&out->tris, (size_t)nt * (out->compact ? sizeof(TriRecBox) : sizeof(TriRec))));

    k_init_stats<<<1, 64, 0, stream>>>(stats);
    {
        const unsigned g = min(1024u, blocks_for(nt, 256));
        k_scene_stats<<<g, 256, 0, stream>>>(d_tri9, nt, stats);
    }
    k_boxes_codes<<<blocks_for(nt, 256), 256, 0, stream>>>(d_tri9, nt, stats, tri_box, codes, ids);
    TR_CHECK(hipGetLastError());
    TR_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, codes, codes_sorted, ids, ids_sorted, n, 0,
                                                30, stream));
    TR_CHECK(hipMalloc(&temp, temp_bytes));
    TR_CHECK(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, codes, codes_sorted, ids, ids_sorted, n, 0, 30,
                                                stream));
    k_fill_i32<<<blocks_for(ni, 256), 256, 0, stream>>>(parent_int, -1, (size_t)ni);
    k_fill_i32<<<blocks_for(nt, 256), 256, 0, stream>>>(parent_leaf, -1, (size_t)nt);
    k_fill_u32<<<blocks_for(ni, 256), 256, 0, stream>>>(arrivals, 0u, (size_t)ni);
    k_fill_u32<<<1, 64, 0, stream>>>(depth, 0u, 1);
    out->root = (n > 1) ? 0 : ~0;
    if (n > 1 && builder == kBuilderLbvh) {
        k_hierarchy<<<blocks_for(n - 1, 256), 256, 0, stream>>>(codes_sorted, n, child, parent_int, parent_leaf);
        k_refit<<<blocks_for(n, 256), 256, 0, stream>>>(n, child, parent_int, parent_leaf, tri_box, ids_sorted,
                                                        node_box, arrivals);
    } else if (n > 1) {
        TR_CHECK(hipMalloc(&c_node, (size_t)n * sizeof(int32_t)));
        TR_CHECK(hipMalloc(&c_node2, (size_t)n * sizeof(int32_t)));
        TR_CHECK(hipMalloc(&nn, (size_t)n * sizeof(int32_t)));
        TR_CHECK(hipMalloc(&c_box, 6ull * n * sizeof(float)));
        TR_CHECK(hipMalloc(&c_box2, 6ull * n * sizeof(float)));
        TR_CHECK(hipMalloc(&mflag, ((size_t)n + 1) * sizeof(uint32_t)));
        TR_CHECK(hipMalloc(&keep, ((size_t)n + 1) * sizeof(uint32_t)));
        TR_CHECK(hipMalloc(&moff, ((size_t)n + 1) * sizeof(uint32_t)));
        TR_CHECK(hipMalloc(&koff, ((size_t)n + 1) * sizeof(uint32_t)));
        TR_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, mflag, moff, n + 1, stream));
        TR_CHECK(hipMalloc(&scan_temp, scan_bytes));
        k_ploc_init<<<blocks_for(n, 256), 256, 0, stream>>>(n, tri_box, ids_sorted, c_node, c_box);
        int nc = n;
        int made = 0;  // internal nodes so far; node indices grow in creation order
        int stall = 0;
        while (nc > 1) {
            const int force = stall ? 1 : 0;
            k_ploc_nn<<<blocks_for(nc, 256), 256, 0, stream>>>(nc, c_box, nn);
            k_ploc_flags<<<blocks_for(nc, 256), 256, 0, stream>>>(nc, nn, force, mflag, keep);
            // exclusive scans over nc + 1 entries give the totals in the last slot
            k_fill_u32<<<1, 64, 0, stream>>>(mflag + nc, 0u, 1);
            k_fill_u32<<<1, 64, 0, stream>>>(keep + nc, 0u, 1);
            TR_CHECK(hipcub::DeviceScan::ExclusiveSum(scan_temp, scan_bytes, mflag, moff, nc + 1, stream));
            TR_CHECK(hipcub::DeviceScan::ExclusiveSum(scan_temp, scan_bytes, keep, koff, nc + 1, stream));
            k_ploc_merge<<<blocks_for(nc, 256), 256, 0, stream>>>(nc, nn, force, mflag, moff, koff, c_node, c_box,
                                                                  made, child, node_box, c_node2, c_box2);
            TR_CHECK(hipGetLastError());
            uint32_t counts[2];
            TR_CHECK(hipMemcpyAsync(&counts[0], moff + nc, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
            TR_CHECK(hipMemcpyAsync(&counts[1], koff + nc, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
            TR_CHECK(hipStreamSynchronize(stream));
            made += (int)counts[0];
            stall = (counts[0] == 0) ? 1 : 0;
            nc = (int)counts[1];
            std::swap(c_node, c_node2);
            std::swap(c_box, c_box2);
            if (made > n - 1) {
                err = hipErrorUnknown;
                goto done;
            }
        }
        out->root = made - 1;
        k_parents<<<blocks_for(n - 1, 256), 256, 0, stream>>>(n - 1, child, parent_int, parent_leaf);
    }
    if (n > 1) {
        if (out->compact)
            k_layout_compact<<<blocks_for(n - 1, 256), 256, 0, stream>>>(n, child, tri_box, ids_sorted, node_box,
                                                                         static_cast<CompactNode*>(out->nodes));
        else
            k_layout<<<blocks_for(n - 1, 256), 256, 0, stream>>>(n, child, tri_box, ids_sorted, node_box,
                                                                 static_cast<BvhNode*>(out->nodes));
        k_depth<<<blocks_for(n, 256), 256, 0, stream>>>(n, parent_int, parent_leaf, depth);
    }
    if (out->compact)
        k_tris_box<<<blocks_for(n, 256), 256, 0, stream>>>(n, d_tri9, ids_sorted, tri_box,
                                                            static_cast<TriRecBox*>(out->tris));
    else
        k_tris<<<blocks_for(n, 256), 256, 0, stream>>>(n, d_tri9, ids_sorted, static_cast<TriRec*>(out->tris));
    TR_CHECK(hipGetLastError());
    TR_CHECK(hipMemcpyAsync(host_stats, stats, sizeof(host_stats), hipMemcpyDeviceToHost, stream));
    TR_CHECK(hipMemcpyAsync(&host_depth, depth, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    if (n == 1) {
        float b[6];
        TR_CHECK(hipMemcpyAsync(b, tri_box, sizeof(b), hipMemcpyDeviceToHost, stream));
        TR_CHECK(hipStreamSynchronize(stream));
        for (int a = 0; a < 3; ++a) {
            out->root_lo[a] = b[a];
            out->root_hi[a] = b[3 + a];
        }
    }
    TR_CHECK(hipStreamSynchronize(stream));
    {
        float mabs;
        memcpy(&mabs, &host_stats[0], 4);
        out->pad = mabs * 0x1p-16f;
    }
    out->n_internal = (uint32_t)(n > 1 ? n - 1 : 0);
    out->depth = host_depth;

done:
    hipFree(stats); hipFree(codes); hipFree(codes_sorted); hipFree(ids); hipFree(ids_sorted);
    hipFree(tri_box); hipFree(node_box); hipFree(child); hipFree(parent_int); hipFree(parent_leaf);
    hipFree(arrivals); hipFree(depth); hipFree(temp);
    hipFree(c_node); hipFree(c_node2); hipFree(nn); hipFree(c_box); hipFree(c_box2);
    hipFree(mflag); hipFree(keep); hipFree(moff); hipFree(koff); hipFree(scan_temp);
    if (err != hipSuccess) {
        hipFree(out->nodes);
        hipFree(out->tris);
        out->nodes = nullptr;
        out->tris = nullptr;
    }
    return err;
}

namespace {

// inverse of the BVH order: out[caller index] = BVH-order index
__global__ void k_sorted_of(uint32_t n, const uint32_t* __restrict__ prim, uint32_t stride_words,
                            uint32_t* __restrict__ out)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[prim[(size_t)j * stride_words]] = j;
}

}  // namespace

hipError_t launch_sorted_of(const void* tris, bool compact, uint32_t nt, uint32_t* out, hipStream_t stream)
{
    if (nt == 0) return hipSuccess;
    // the caller index is word 3 of either record
    const uint32_t* prim = static_cast<const uint32_t*>(tris) + 3;
    const uint32_t stride = (uint32_t)((compact ? sizeof(TriRecBox) : sizeof(TriRec)) / 4);
    hipLaunchKernelGGL(k_sorted_of, dim3((nt + 255) / 256), dim3(256), 0, stream, nt, prim, stride, out);
    return hipGetLastError();
}

}  // namespace trhip
