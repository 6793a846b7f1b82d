// internal.h -- declarations shared by the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "scene_view.h"

namespace trhip {

struct BvhBuild {
    void* nodes;   // BvhNode[] or, when compact, CompactNode[]
    void* tris;    // TriRec[] or, when compact, TriRecBox[]
    bool compact;  // more than kShortStackMaxTris triangles
    int32_t root;
    float root_lo[3], root_hi[3];
    uint32_t n_internal;
    uint32_t depth;
    float pad;
};

constexpr int kBuilderPloc = 0;
constexpr int kBuilderLbvh = 1;

// Builds the BVH of nt triangles given as a device float[nt][9] array;
// synchronises `stream`.  On failure nothing stays allocated.
hipError_t build_bvh(const float* d_tri9, uint32_t nt, int builder, hipStream_t stream, BvhBuild* out);

// out[tris[j].prim] = j for the nt triangle records of a built BVH
hipError_t launch_sorted_of(const void* tris, bool compact, uint32_t nt, uint32_t* out, hipStream_t stream);

// Traversal stacks hold one BVH link per level.  With at most 32,768
// triangles every link (internal node index, or ~sorted triangle index)
// fits in 16 bits, which halves the stacks' LDS; larger scenes use 32 bits.
constexpr uint32_t kShortStackMaxTris = 32768;
inline bool short_stack(uint32_t n_tris) { return n_tris <= kShortStackMaxTris; }
// LDS bytes of one lane's stack
inline uint32_t stack_lane_bytes(uint32_t n_tris, uint32_t stack_depth)
{
    return stack_depth * (short_stack(n_tris) ? 2u : 4u);
}

// The HBM-film path form keeps the first kSplitStackLds words of a 32-bit
// stack in LDS and the deeper ones in per-lane scratch memory, for trees of
// at most kSplitStackLds + kSplitStackDeep levels (deeper trees keep the
// whole stack in LDS).  LDS bytes of one lane's stack in that form:
// The environment variable TRHIP_SPLIT_STACK=0 keeps whole stacks in LDS
// (read at every launch).
constexpr uint32_t kSplitStackLds = 16;
constexpr uint32_t kSplitStackDeep = 48;
bool split_stack_enabled();
inline bool split_stack(uint32_t n_tris, uint32_t stack_depth)
{
    return !short_stack(n_tris) && stack_depth <= kSplitStackLds + kSplitStackDeep && split_stack_enabled();
}
inline uint32_t hbm_stack_lane_bytes(uint32_t n_tris, uint32_t stack_depth)
{
    return split_stack(n_tris, stack_depth) ? 4u * (stack_depth < kSplitStackLds ? stack_depth : kSplitStackLds)
                                            : stack_lane_bytes(n_tris, stack_depth);
}

// entries of the counting build's output (TRHIP_COUNT_N)
constexpr int kWorkCounters = 10;

// LDS bytes of one render / backward workgroup (stack_bytes per lane)
size_t render_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes);
size_t wavefront_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes);
size_t backward_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes,
                          bool primal, bool fixed);
// path per lane with the film in HBM (float atomics, no LDS film; zero-fills
// the outputs first unless accumulating); LDS = the lanes' stacks
size_t hbm_lds_bytes(uint32_t block, uint32_t stack_bytes);
hipError_t launch_render_hbm(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                             unsigned long long* counts = nullptr);
// deterministic forward render (path per lane, fixed-point tile sums)
size_t fixed_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes);
hipError_t launch_render_fixed(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream);
// fixed-point sums (two 64-bit words each, as the deterministic kernels hold them) to FP32
// deterministic forward with the film in HBM: 64-bit words of L.fixed_film
size_t fixed_film_words(uint32_t n_pixels, uint32_t n_bins);
hipError_t launch_render_fixed_hbm(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream);
hipError_t launch_fixed_to_f32(const unsigned long long* src, float* dst, size_t n, hipStream_t stream);

// counts: optional device uint64[7] receiving the work counters (node
// visits, triangle tests, closest rays, shadow rays, vertices, Philox draws,
// contributions); selects the counting build of the kernel
hipError_t launch_render(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                         unsigned long long* counts = nullptr);
hipError_t launch_render_wavefront(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                                   unsigned long long* counts = nullptr);
// max_cont 2 or 7: single-trace adjoint with a per-path stash of that many
// continuation vertices; anything else: path replay (two traces per path).
// L.g_fixed set: deterministic fixed-point gradient sums ([2][n_tris][2]
// words) instead of FP64 atomics into L.g_alb, L.g_rough
hipError_t launch_backward(const SceneView& S, const LaunchArgs& L, uint32_t block, int max_cont, hipStream_t stream);
size_t tangent_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes);
// forward-mode render: film and its derivative along (tan_albedo, tan_rough)
hipError_t launch_render_tangent(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream);
size_t deferred_lds_bytes(uint32_t tile_pixels, uint32_t n_bins, uint32_t block, uint32_t stack_bytes);
size_t batch_lds_bytes(uint32_t film_words, uint32_t block, uint32_t stack_bytes, bool deferred);
// resets the cursor and launches the persistent kernel (groups workgroups)
// for scenes that all have 16-bit (short_links) or all 32-bit stack links,
// stack_depth the deepest of their BVHs
hipError_t launch_batch(const BatchTables& B, uint32_t groups, uint32_t block, uint32_t stack_depth, bool short_links,
                        bool deferred, hipStream_t stream);
hipError_t launch_render_deferred(const SceneView& S, const LaunchArgs& L, uint32_t block, hipStream_t stream,
                                  unsigned long long* counts = nullptr);
// sample chunks per tile of the deferred form (sets the samples per chunk);
// chunks > 1 need L.chunk_scratch ((chunks - 1) * (n_pixels * words +
// 2 * n_pixels) floats, words = floats of one pixel's film), and after the
// render launch_add_planes, which adds those partial films to the outputs
constexpr uint32_t kMaxChunks = 4;
uint32_t deferred_chunks(uint32_t spp, uint32_t block, uint32_t* chunk_spp);
hipError_t launch_add_planes(const LaunchArgs& L, uint32_t words, hipStream_t stream);
hipError_t launch_zero_f64(double* p, size_t n, hipStream_t stream);
// out[i] = Poisson(scale * film[i]) / scale (noise.hip)
hipError_t launch_poisson(const float* film, float* out, uint64_t n, float scale, uint64_t seed, hipStream_t stream);
hipError_t launch_f64_to_f32(const double* src, float* dst, size_t n, hipStream_t stream);
hipError_t launch_scene_fill(const float* tri9, uint32_t nt, hipStream_t stream);

// numerics probe (probe.hip): one primitive per element, TRHIP_PROBE_* order
enum { kProbeSinCos2Pi = 0, kProbeLog1m = 1, kProbePhilox = 2, kProbeDiv = 3, kProbeSqrt = 4 };
hipError_t launch_probe(int op, const void* in, void* out, uint64_t n, uint64_t first, hipStream_t stream);

}  // namespace trhip
