// scene_view.h -- device-side layout of an uploaded scene and of one launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trhip {

// One internal BVH node, 64 bytes = four 16-byte loads: the boxes of both
// children (so one fetch decides both) and the two child links.  A link
// >= 0 is an internal node; a link < 0 is ~(sorted triangle index) and the
// box stored for it is exactly that triangle's padded box.
struct alignas(16) BvhNode {
    float lo0x, lo0y, lo0z, hi0x;
    float hi0y, hi0z, lo1x, lo1y;
    float lo1z, hi1x, hi1y, hi1z;
    int32_t child0, child1, unused0, unused1;
};
static_assert(sizeof(BvhNode) == 64, "BvhNode must be 64 bytes");

// One triangle in BVH (Morton) order, 48 bytes: v0, e1 = v1 - v0,
// e2 = v2 - v0 and the caller's triangle index.
struct alignas(16) TriRec {
    float v0x, v0y, v0z;
    uint32_t prim;
    float e1x, e1y, e1z, unused0;
    float e2x, e2y, e2z, unused1;
};
static_assert(sizeof(TriRec) == 48, "TriRec must be 48 bytes");

// Scenes with more than 32,768 triangles (32-bit stack links) use a compact
// layout, so that a node visit issues two 16-byte loads instead of four.
// CompactNode, 32 bytes: both children's boxes as FP16 bit patterns rounded
// outward (lo down, hi up: each contains the FP32 box it stands for) in the
// order lo0x hi0x lo0y hi0y lo0z hi0z lo1x hi1x lo1y hi1y lo1z hi1z (one
// 32-bit word per child and axis, lo in its low half), then the two links.  Traversal only: a leaf's FP16 box contains its padded
// box, so every triangle the padded box admits is still reached.
struct alignas(16) CompactNode {
    uint16_t box[12];
    int32_t child0, child1;
};
static_assert(sizeof(CompactNode) == 32, "CompactNode must be 32 bytes");

// TriRecBox, 64 bytes: TriRec's v0, prim, e1, e2 with the triangle's padded
// box (lo, hi) in the remaining words, for the acceptance rule.
struct alignas(16) TriRecBox {
    float v0x, v0y, v0z;
    uint32_t prim;
    float e1x, e1y, e1z, lox;
    float e2x, e2y, e2z, loy;
    float loz, hix, hiy, hiz;
};
static_assert(sizeof(TriRecBox) == 64, "TriRecBox must be 64 bytes");

struct SceneView {
    const void* nodes;       // BvhNode[], or CompactNode[] when compact
    const void* tris;        // TriRec[], or TriRecBox[] when compact
    const uint8_t* mat;      // caller order
    const float* albedo;     // caller order
    const float* rough;      // caller order
    const float* scan;       // [n_pixels][3], confocal only
    int32_t root;            // >= 0 internal node, < 0 leaf
    float root_lo[3], root_hi[3];
    uint32_t n_tris;
    uint32_t stack_depth;    // longest root-to-leaf path (edges), >= 1
    uint32_t compact;        // 1: CompactNode / TriRecBox layout (more than 32,768 triangles)

    int32_t sensor;          // 0 pinhole, 1 confocal
    uint32_t width, height;
    float cam_o[3], cam_r[3], cam_u[3], cam_f[3];
    float tan_x, tan_y;
    float wall_n[3];
    float wall_albedo, laser_power;
    float light[3];
    float intensity;
    float sigma_t, medium_albedo;
    uint32_t n_bins;
    float bin_width, bin_start;
    int32_t unwarp;

    // NLOS area sampling (confocal), one set of tables per scan region
    // (area_region[scan point]): inclusive FP64 prefix sums of the triangles'
    // sampling weights in caller order ([region][n_tris], 0 on the relay
    // wall's plane), their totals ([region]), the inverse area densities
    // W_r A_k / w_k of a point drawn on triangle k ([region][n_tris]), and
    // guide tables of the inversion ([region][guide_cells + 1]: entry m is
    // the first triangle whose prefix sum exceeds (m / guide_cells) * W_r,
    // clamped to n_tris - 1; guide_cells a power of two <= 2^20); plus the
    // BVH-order index of each caller triangle
    const double* area_cdf;
    const float* area_invp;
    const uint32_t* area_guide;
    const double* area_wtotal;
    const uint8_t* area_region;
    const uint32_t* sorted_of;
    float guide_cells;

    // refractive indices and scattering delays (caller order; nullptr when
    // the scene has no dielectric / no delay) and the index of the space
    // around the meshes
    const float* ior;
    const float* delay;
    float eta0;
};

constexpr uint32_t kMatDielectric = 2;

constexpr uint32_t kMaxFreq = 32;  // frequencies of one phasor film

constexpr uint32_t kFlagPixelCentre = 1u << 0;
constexpr uint32_t kFlagAccumulate = 1u << 1;
constexpr uint32_t kFlagFrozen = 1u << 2;
constexpr uint32_t kFlagNlosArea = 1u << 3;
constexpr uint32_t kFlagDeterministic = 1u << 4;

// One next-event contribution of the recording build (32 bytes; the layout
// of trhip_record): the path's pixel or scan point and sample index, the
// 1-based vertex of the connection, its bin (-1 outside the window), the
// value c before the 1/N normalisation, the connected path's optical
// length and the vertex's triangle (caller index, -1 for a medium vertex).
struct alignas(16) ContribRecord {
    uint32_t pixel, sample;
    int32_t vertex, bin;
    float value, tof;
    int32_t tri;
    uint32_t reserved;
};
static_assert(sizeof(ContribRecord) == 32, "ContribRecord must be 32 bytes");

struct LaunchArgs {
    uint32_t spp, sample_offset, max_depth, stream_id;
    uint32_t key0, key1, flags;
    uint32_t tile_pixels, n_pixels;
    uint32_t chunks;            // sample chunks per tile (deferred form), one workgroup each
    uint32_t chunk_spp;         // samples per chunk
    float* chunk_scratch;       // chunks > 1: partial films of chunks 1.., [chunk - 1][n_pixels * words + 2 * n_pixels]
    float norm;                 // 1 / norm_spp
    uint32_t norm_spp;          // the film's divisor N
    const float* albedo;        // evaluation albedo (caller order)
    const float* rough_eval;    // evaluation roughness
    const float* rough_sample;  // sampling roughness (== rough_eval unless frozen)
    float* film;
    float* steady;
    float* oow;
    const float* grad_film;     // backward
    double* g_alb;
    double* g_rough;
    unsigned long long* g_fixed;  // deterministic backward: fixed-point sums [2][n_tris][2] (else NULL)
    // deterministic forward with the film in HBM: fixed-point film, steady
    // and oow of the launch, [n_pixels][n_bins][2], [n_pixels][2], [n_pixels][2]
    unsigned long long* fixed_film;
    float* primal;
    const float* tan_albedo;    // forward mode: direction of the albedo (caller order), may be NULL
    const float* tan_rough;     // forward mode: direction of the roughness, may be NULL
    float* dfilm;               // forward mode: derivative film
    // phasor film (n_freq > 0): film is [n_pixels][n_freq][2] (re, im) of
    // sum c exp(-2 pi i f tof) over all contributions, f = freq[j] in cycles
    // per metre of optical path; n_freq = 0: the time histogram
    uint32_t n_freq;
    float freq[kMaxFreq];
    // recording build: contributions of the pixels with record_mask[p] != 0
    // are appended to records (the first record_cap of them; record_count
    // counts all)
    const uint8_t* record_mask;
    ContribRecord* records;
    unsigned long long record_cap;
    unsigned long long* record_count;
};

// Tables of the batched persistent kernel (device memory).
struct BatchTables {
    const SceneView* views;      // [n_scenes]
    const LaunchArgs* args;      // [n_scenes]
    const uint32_t* item_start;  // [n_scenes + 1]: first work item of the k-th scene in processing order
    const uint32_t* order;       // [n_scenes]: scene index of the k-th scene in processing order
    uint32_t n_scenes;
    uint32_t n_items;
    uint32_t film_words;         // LDS floats reserved for the largest tile film
    uint32_t* cursor;            // next work item
};

}  // namespace trhip
