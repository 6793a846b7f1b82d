/*
 * trhip.h -- C ABI of the MI355X (gfx950) transient path tracer.
 *
 * The library renders time-resolved (transient) images by Monte Carlo path
 * tracing, after arXiv 2510.25660 ("mitransient"), Sec. 3: light paths
 * x0 -> ... -> xk (Eq. 1) are sampled with BSDF sampling and next-event
 * estimation; the Monte Carlo estimator of Eq. 9 is histogrammed per pixel
 * into time bins floor((tof - b_start) / b_width) (Sec. 3, "Path reuse and
 * histogramming"), where tof is the summed segment length of the path
 * (Eqs. 3-4, eta = 1, c = 1, so time is optical path length in metres) and
 * emitters pulse at t = 0 (Eq. 5).  The steady image of the same paths is
 * produced alongside (the (steady, transient) pair of the paper's Sec. 2
 * example).  Backward mode (Sec. 4.4, Eqs. 15-17) propagates dL/dfilm to
 * per-triangle albedo and roughness.
 *
 * Conventions for every entry point:
 *  - every function returns trhip_status (0 = TRHIP_OK); no exception or
 *    abort crosses the ABI; trhip_last_error() gives a thread-local message;
 *  - arguments are validated on the host before any HIP call, so invalid
 *    input is reported without touching the GPU;
 *  - "host pointer" arguments are read during the call only; "device
 *    pointer" arguments are HBM buffers owned by the caller, which must stay
 *    valid until the work enqueued on `stream` has completed;
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream);
 *    all device work is enqueued on it, asynchronously;
 *  - the library never keeps a caller pointer after a call returns;
 *  - a scene may be used by one stream at a time: it owns the scratch
 *    memory of its launches (the backward pass's gradient sums, the
 *    deferred form's partial films), so calls on one scene that overlap in
 *    time on different streams race; serialise them (one stream, or events).
 */
#ifndef TRHIP_H
#define TRHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int trhip_status;

enum {
    TRHIP_OK = 0,
    TRHIP_ERR_INVALID_ARG = 1, /* a bad pointer, size, enum or value */
    TRHIP_ERR_OOM = 2,         /* a device or host allocation failed */
    TRHIP_ERR_HIP = 3,         /* a HIP runtime call failed (message has the hipError_t) */
    TRHIP_ERR_UNSUPPORTED = 4, /* a valid request the library cannot serve (e.g. LDS budget) */
    TRHIP_ERR_BAD_HANDLE = 5   /* NULL, destroyed or foreign handle */
};

enum { TRHIP_SENSOR_PINHOLE = 0, TRHIP_SENSOR_CONFOCAL = 1 };
enum { TRHIP_MAT_LAMBERT = 0, TRHIP_MAT_GGX = 1, TRHIP_MAT_DIELECTRIC = 2 };

/* render flags */
enum {
    TRHIP_FLAG_PIXEL_CENTRE = 1u << 0,    /* no sub-pixel jitter (pinhole) */
    TRHIP_FLAG_ACCUMULATE = 1u << 1,      /* add into the output buffers instead of overwriting */
    TRHIP_FLAG_FROZEN_PROPOSAL = 1u << 2, /* GGX: sample with the scene's roughness, evaluate
                                             with roughness_override (finite-difference mode) */
    TRHIP_FLAG_NLOS_AREA_SAMPLING = 1u << 3, /* confocal: area-sample the hidden vertex (below) */
    TRHIP_FLAG_DETERMINISTIC = 1u << 4       /* order-independent sums, bit-reproducible (below) */
};

/*
 * TRHIP_FLAG_DETERMINISTIC -- bit-reproducible films and gradients, for the
 * finite-difference checks of the gradients of Sec. 4.4 (Eqs. 15-16) and for
 * race detection: two renders with the same inputs then agree bit for bit,
 * whatever the launch shape (tile_pixels, block_size), the scheduling or
 * the GPU load.  Every contribution to the film, steady and oow sums, and
 * every gradient term, is accumulated as a 128-bit two's-complement fixed
 * point number with 64 fraction bits with integer atomics, which are
 * associative; the sums are rounded to FP32 once, after division by
 * norm_spp.  A film bin is then the exact sum of its FP32 contributions of
 * magnitude >= 2^-41 (smaller ones are truncated to multiples of 2^-64),
 * divided by N and rounded: it differs from an FP64 sum in path order only
 * by that sum's own rounding.  Values and sums must stay below 2^63 in
 * magnitude.  Accepted by trhip_render_transient and
 * trhip_render_transient_noalloc (the path form runs; a render->kernel
 * other than AUTO or PATH is UNSUPPORTED) and
 * trhip_render_transient_backward (gradients; primal_film is not covered);
 * the other entry points return UNSUPPORTED.  The fixed-point tile film
 * takes about 2x the LDS of the default film per pixel, so the automatic
 * shape takes fewer pixels per workgroup; where the path form keeps the
 * film in HBM (more than 32,768 triangles and 512 bins or more),
 * trhip_render_transient instead keeps the fixed-point sums of the whole
 * launch in a buffer of 24 bytes per bin that the scene allocates on first
 * use and keeps (not while the stream is being captured, not for spp *
 * max_depth >= 2^21, not when the device cannot hold it, and never in
 * trhip_render_transient_noalloc: those render the LDS form, with the same
 * result bit for bit).
 */

/*
 * TRHIP_FLAG_NLOS_AREA_SAMPLING -- sampling specific to non-line-of-sight
 * scenes (Sec. 4.5 adds NLOS-tailored samplers from the work it cites; this
 * is the area-sampling one, which aims every path at the hidden geometry
 * instead of the hemisphere above the relay wall).  The first path vertex
 * after the scan point is drawn on the scene's triangles that do not lie in
 * the relay wall's plane (the plane through the first scan point with
 * normal wall_normal, within 1e-6 * (1 + largest |vertex coordinate|)).
 * The scan points are split into 4 x 4 regions of their bounding box (over
 * its two axes of largest extent); for a scan point of region r, triangle k
 * is drawn with probability w_k / W_r, w_k = A_k (g_k + g_max / 20) in FP64
 * (A_k its area, g_k = (cos_s cos_h / r^2)^2 the squared geometry term
 * between the mean of the region's scan points and the triangle's
 * centroid, g_max the region's largest), the point uniformly within it
 * (square-root warp of two uniforms).  The vertex carries the weight
 * wall_albedo / pi * cos_wall * cos_hidden / r^2 * W_r A_k / w_k; its
 * visibility is the
 * next-event shadow test back to the scan point, which runs along the same
 * segment.  The estimate has the expectation of the default
 * (cosine-sampled) render.  A longer path continues from the drawn vertex
 * only if that shadow test finds its first segment unoccluded.
 * Valid for the confocal sensor with max_depth >= 4 (at least one hidden
 * vertex) and no medium
 * (sigma_t == 0); any kernel form but TRHIP_KERNEL_WAVEFRONT (the deferred
 * form, the automatic choice, orders each batch of samples by the BVH
 * position of the sampled triangle, so that a wave's shadow rays leave one
 * region of the hidden surface).  Anything else returns
 * TRHIP_ERR_UNSUPPORTED, as does a scene whose sampling set is empty.  Accepted by trhip_render_transient,
 * _counted, _phasor, _tangent and _backward, and by the batch API (where
 * such scenes run in the path form).
 */

/*
 * Scene description (all pointers are HOST pointers, read during
 * trhip_scene_create only).
 *
 * Geometry: vertices float[n_vertices][3], indices uint32[n_triangles][3]
 * (every index < n_vertices).  Triangles are two-sided.  Zero-area or
 * non-finite triangles are rejected (TRHIP_ERR_INVALID_ARG).
 * Materials per triangle: mat_type (TRHIP_MAT_*), albedo (Lambertian albedo,
 * or the constant reflectance F of the GGX conductor), roughness (GGX alpha,
 * unused for Lambertian).  Albedo must lie in (0, 1], roughness in (0, 1]
 * (both ignored, and not checked, for dielectric triangles).
 *
 * Refractive indices and scattering delays (Eqs. 3 and 10):
 *  - medium_ior: index of the space around the meshes, where the camera,
 *    the light and the relay wall are (0 means 1); every segment's time of
 *    flight is its length times the index of the medium it runs in.
 *  - TRHIP_MAT_DIELECTRIC triangles form closed meshes of a smooth
 *    dielectric whose inside, of index ior[k], lies on the side opposite to
 *    the winding normal (v1 - v0) x (v2 - v0): wind them outward.  At such
 *    a triangle a path reflects with the unpolarised Fresnel reflectance
 *    (1 beyond the critical angle) or refracts by Snell's law, with weight
 *    1 or (eta_i / eta_t)^2; there is no next-event connection (a delta
 *    interface) and no gradient parameter.  Dielectric meshes must not
 *    overlap or nest (leaving one always returns to medium_ior); a
 *    participating medium (sigma_t) fills only the space around them, and
 *    they block shadow rays like any triangle.  ior may be NULL if no
 *    triangle is dielectric; entries must be finite and in (0, 100].
 *  - delay (NULL = none): per triangle the mean tau >= 0 (metres of optical
 *    path) of an exponentially distributed scattering delay: at every
 *    surface vertex on a triangle with tau > 0 the path's time of flight
 *    grows by tau * E, E ~ Exp(1) drawn from the vertex's random numbers;
 *    the delay applies to that vertex's contribution and all later ones.
 *
 * Emitter: an isotropic point light of intensity light_intensity (W/sr) at
 * light_pos (pinhole sensor).  For the confocal sensor the emitter is the
 * laser spot on the relay wall, a Lambertian point emitter of power
 * laser_power * wall_albedo at each scan point.
 *
 * Sensor:
 *  - TRHIP_SENSOR_PINHOLE: camera at cam_origin with unit right/up/forward
 *    vectors and the tangents of the half fields of view; the film has
 *    width x height pixels, row-major, row 0 at the top.
 *  - TRHIP_SENSOR_CONFOCAL: laser and detector co-located at each of the
 *    width*height scan points (scan_points float[width*height][3], on the
 *    relay wall whose unit normal wall_normal faces the hidden scene);
 *    the film row p belongs to scan point p.  The segments between the
 *    devices and the wall are excluded from the time of flight.
 *
 * Medium: homogeneous, filling space, extinction sigma_t (1/m) and
 * single-scattering albedo medium_albedo; sigma_t == 0 disables it
 * (Sec. 4.1, "Volumetric scattering").
 *
 * Film: n_bins bins of bin_width metres of optical path length starting at
 * bin_start (the sensor window of Eq. 6, half-open at its end).
 * camera_unwarp != 0 omits the camera segment (Sec. 3, "Camera warp and
 * unwarping"); pinhole only.
 *
 * bvh_builder: TRHIP_BVH_PLOC (0, default: locally-ordered clustering over
 * the Morton order) or TRHIP_BVH_LBVH (Karras hierarchy over the Morton
 * order).  Any builder yields the same renders (see trhip_render_transient);
 * they differ in traversal cost.
 */
typedef struct {
    const float* vertices;
    uint32_t n_vertices;
    const uint32_t* indices;
    uint32_t n_triangles;
    const uint8_t* mat_type;
    const float* albedo;
    const float* roughness;

    float light_pos[3];
    float light_intensity;

    int32_t sensor;
    uint32_t width, height;
    float cam_origin[3], cam_right[3], cam_up[3], cam_fwd[3];
    float tan_x, tan_y;
    const float* scan_points;
    float wall_normal[3];
    float wall_albedo;
    float laser_power;

    float sigma_t;
    float medium_albedo;

    uint32_t n_bins;
    float bin_width;
    float bin_start;
    int32_t camera_unwarp;
    int32_t bvh_builder;

    const float* ior;       /* [n_triangles] or NULL (see above) */
    const float* delay;     /* [n_triangles] or NULL */
    float medium_ior;       /* 0 = 1 */
} trhip_scene_desc;

enum { TRHIP_BVH_PLOC = 0, TRHIP_BVH_LBVH = 1 };

/*
 * Render description.
 * spp: samples per pixel N of the estimator (Eq. 9), >= 1.
 * sample_offset: first sample index; samples [sample_offset, +spp) are drawn,
 *   so disjoint ranges rendered with TRHIP_FLAG_ACCUMULATE reproduce one
 *   render over the union.
 * norm_spp: divisor of the film (0 = spp); set it to the total sample count
 *   when accumulating several ranges.
 * max_depth: number of path segments including the device segments
 *   (a pinhole path has at most max_depth - 1 scattering vertices, a
 *   confocal path at most max_depth - 3 hidden-scene vertices), >= 1.
 * seed: 64-bit Philox key; stream_id: fourth Philox counter word
 *   (e.g. 0 for renders, 1 for targets).
 * albedo_override / roughness_override: optional DEVICE pointers to
 *   float[n_triangles] replacing the scene's values for this call.
 * tile_pixels / block_size: launch shape (0 = automatic choice).
 * kernel: form of the forward render kernel, TRHIP_KERNEL_* (0 = automatic):
 *   PATH traces one whole path per lane; DEFERRED traces the first ray of
 *   one sample per lane, buffers the first vertices in LDS and follows the
 *   rest of those paths on densely packed lanes; WAVEFRONT runs the stages
 *   of a workgroup's paths (generate, intersect, shade, shadow) over
 *   compacted queues held in LDS.  All produce the same film.  For the
 *   backward pass, TRHIP_KERNEL_PATH selects path replay (every path traced
 *   twice) and any other value the automatic choice (one trace per path with
 *   a per-path register stash when a path has at most 8 vertices, else
 *   replay); both give the same gradients up to rounding.
 */
typedef struct {
    uint32_t spp;
    uint32_t sample_offset;
    uint32_t norm_spp;
    uint32_t max_depth;
    uint64_t seed;
    uint32_t stream_id;
    uint32_t flags;
    const float* albedo_override;
    const float* roughness_override;
    uint32_t tile_pixels;
    uint32_t block_size;
    uint32_t kernel;
} trhip_render_desc;

enum { TRHIP_KERNEL_AUTO = 0, TRHIP_KERNEL_PATH = 1, TRHIP_KERNEL_WAVEFRONT = 2, TRHIP_KERNEL_DEFERRED = 3 };

typedef struct trhip_scene trhip_scene;

/* Read-only facts about an uploaded scene. */
typedef struct {
    uint32_t n_triangles;
    uint32_t n_pixels;
    uint32_t n_bins;
    uint32_t bvh_internal_nodes;
    uint32_t bvh_depth;         /* longest root-to-leaf path, in edges */
    float box_pad;              /* inflation of every triangle box (metres) */
    size_t device_bytes;        /* scene + BVH bytes held on the device */
} trhip_scene_info;

/*
 * Upload a scene and build its BVH on the device (30-bit Morton codes, radix
 * sort, then the hierarchy of desc->bvh_builder) on `stream`; blocks until
 * the build has finished.
 * On success *out owns all scene memory until trhip_scene_destroy.
 * Errors: INVALID_ARG (NULL desc/out, bad sizes or values, degenerate or
 * non-finite triangles, index out of range), OOM, HIP.
 */
trhip_status trhip_scene_create(const trhip_scene_desc* desc, void* stream, trhip_scene** out);

/* Free a scene (waits for the device).  NULL is accepted.  Errors: BAD_HANDLE. */
trhip_status trhip_scene_destroy(trhip_scene* scene);

/* Fill *info.  Errors: BAD_HANDLE, INVALID_ARG (NULL info). */
trhip_status trhip_scene_get_info(const trhip_scene* scene, trhip_scene_info* info);

/*
 * Forward transient render (Sec. 3, Eqs. 1-9 and the histogram rule).
 * film: DEVICE float[n_pixels][n_bins] (time fastest).  steady, oow:
 * optional DEVICE float[n_pixels]: the steady image (every contribution)
 * and the mass that fell outside the film window.  All three are
 * normalised by 1/norm_spp and overwritten unless TRHIP_FLAG_ACCUMULATE.
 * The path form of a scene with more than 32,768 triangles and a film of
 * 512 bins or more adds into the film in HBM, with each lane's traversal
 * stack split between LDS and scratch memory for trees of at most 64
 * levels; the environment variable TRHIP_SPLIT_STACK=0 (read at every call)
 * keeps whole stacks in LDS there.  The results do not depend on it.
 * Errors: BAD_HANDLE, INVALID_ARG, UNSUPPORTED (launch shape beyond LDS), HIP.
 */
trhip_status trhip_render_transient(trhip_scene* scene, const trhip_render_desc* render, float* film,
                                    float* steady, float* oow, void* stream);

/*
 * trhip_render_transient for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, same render (same paths, same film up to the
 * rounding of the sums), and no allocation of any kind: where the kernel
 * needs scratch memory (the deferred form's sample chunks keep the partial
 * films of all but the first sample chunk of a pixel), it uses a 32 MiB
 * device array that the library holds on every GPU it runs on until the
 * process ends, instead of the buffer trhip_render_transient allocates on
 * first use.  Renders whose scratch would exceed 32 MiB return
 * TRHIP_ERR_UNSUPPORTED (the confocal 64 x 64 scan with 512 bins at 4096 spp
 * needs about 8.4 MB).
 * All calls on one GPU share that array: calls that overlap in time on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  The scene's device must be the current one (else INVALID_ARG).
 * Errors: as trhip_render_transient.
 */
trhip_status trhip_render_transient_noalloc(trhip_scene* scene, const trhip_render_desc* render, float* film,
                                            float* steady, float* oow, void* stream);

/*
 * Backward mode (Sec. 4.4, Eqs. 15-17): given grad_film = dL/dfilm (DEVICE,
 * same layout as the film), writes dL/d(albedo) and dL/d(roughness) per
 * triangle (DEVICE float[n_triangles], overwritten; roughness gradients of
 * Lambertian triangles are 0).  The gradient is that of the estimator at
 * the given seed with the sampling pdf held fixed, from the same paths as
 * the forward render (see render->kernel for the two evaluation orders).
 * primal_film (optional,
 * DEVICE, film layout) receives the film of the replayed paths.
 * Errors: BAD_HANDLE, INVALID_ARG, UNSUPPORTED, OOM, HIP.
 */
trhip_status trhip_render_transient_backward(trhip_scene* scene, const trhip_render_desc* render,
                                             const float* grad_film, float* grad_albedo,
                                             float* grad_roughness, float* primal_film, void* stream);

/*
 * Diagnostic variant of trhip_render_transient: the same render (same
 * output, same paths) by a build of the kernel that also counts its work.
 * counts: HOST uint64[TRHIP_COUNT_N], overwritten, indexed by TRHIP_COUNT_*.
 * The first seven count work per path (lane); the WAVE_* entries count how
 * many times a wave executed the block with at least one lane, so that
 * TRHIP_COUNT_NODES / TRHIP_COUNT_WAVE_NODES is the mean number of active
 * lanes (of 64) in a node visit, and likewise for triangle tests and
 * vertices.  Synchronous (returns after the render has finished); allocates
 * a small device buffer.  Errors: as trhip_render_transient, plus
 * INVALID_ARG for a NULL counts.
 */
enum {
    TRHIP_COUNT_NODES = 0,       /* BVH internal-node visits (both child boxes tested) */
    TRHIP_COUNT_TRIS = 1,        /* ray-triangle tests */
    TRHIP_COUNT_RAYS = 2,        /* closest-hit rays */
    TRHIP_COUNT_SHADOW = 3,      /* shadow (any-hit) rays */
    TRHIP_COUNT_VERTS = 4,       /* scattering vertices (surface or medium) */
    TRHIP_COUNT_DRAWS = 5,       /* Philox4x32-10 evaluations */
    TRHIP_COUNT_CONTRIB = 6,     /* contributions scattered into the film */
    TRHIP_COUNT_WAVE_NODES = 7,  /* wave executions of a node visit */
    TRHIP_COUNT_WAVE_TRIS = 8,   /* wave executions of a triangle test */
    TRHIP_COUNT_WAVE_VERTS = 9,  /* wave executions of a vertex */
    TRHIP_COUNT_N = 10
};
trhip_status trhip_render_transient_counted(trhip_scene* scene, const trhip_render_desc* render, float* film,
                                            float* steady, float* oow, uint64_t* counts, void* stream);

/*
 * Diagnostic variant of trhip_render_transient that also lists its
 * contributions one by one, so that the bin index and the value of every
 * next-event contribution (Sec. 3, "Path reuse and histogramming": a
 * contribution c of a path of time of flight tof lands in bin
 * floor((tof - b_start) / b_width)) can be compared with an independent
 * implementation, not only their sums in the film.  The same render (same
 * film, steady and oow, same paths, the kernel form render->kernel
 * selects) by a build of that kernel that appends one trhip_record per
 * contribution of every pixel p with pixel_mask[p] != 0.
 *
 * pixel_mask: DEVICE uint8[n_pixels].  records: DEVICE
 * trhip_record[capacity] (NULL allowed when capacity is 0).  n_records:
 * HOST uint64, receives the number of contributions of the marked pixels;
 * when it exceeds capacity only `capacity` of them (in no particular order)
 * were written.  Records come in no particular order.  film, steady, oow:
 * as for trhip_render_transient.  Synchronous (returns after the render
 * has finished); allocates a small device buffer.
 * Errors: as trhip_render_transient, plus INVALID_ARG for a NULL
 * pixel_mask, n_records, or records with capacity > 0; UNSUPPORTED for a
 * phasor-style or batched render (only this entry records).
 */
typedef struct {
    uint32_t pixel;   /* pixel or scan point (row-major index) */
    uint32_t sample;  /* sample index, sample_offset included */
    int32_t vertex;   /* scattering vertex of the connection, 1-based */
    int32_t bin;      /* time bin, -1 outside the film window */
    float value;      /* contribution c, before the 1/norm_spp normalisation */
    float tof;        /* optical path length of the connected path (metres) */
    int32_t tri;      /* caller index of the vertex's triangle, -1 for a medium vertex */
    uint32_t reserved;
} trhip_record;
trhip_status trhip_render_transient_records(trhip_scene* scene, const trhip_render_desc* render,
                                            const uint8_t* pixel_mask, trhip_record* records, uint64_t capacity,
                                            uint64_t* n_records, float* film, float* steady, float* oow,
                                            void* stream);

/*
 * Numerics probe.  Every hit, sampled direction, free-flight distance and
 * bin index of the renderer is computed from a few FP32 and integer
 * primitives that an independent implementation must reproduce bit for bit
 * for bin indices to agree (the counter-based random numbers of the Monte
 * Carlo estimator, Eq. 9; the sine and cosine of the direction samplers;
 * ln(1 - u) of the free flight, Sec. 4.1; correctly rounded division and
 * square root).  This entry evaluates one of them per element, on the
 * device, with the same device functions and compiler flags as the render
 * kernels:
 *   TRHIP_PROBE_SINCOS2PI: out float[n][2] = (sin, cos)(2 pi u_i) with
 *     u_i = (first + i) * 2^-24 (the uniforms the renderer draws);
 *   TRHIP_PROBE_LOG1M: out float[n] = ln(1 - u_i), u_i as above;
 *   TRHIP_PROBE_PHILOX: in uint32[n][6] = (counter words 0..3, key low,
 *     key high), out uint32[n][4]: Philox4x32-10 (Salmon et al., SC 2011);
 *   TRHIP_PROBE_DIV: in float[n][2], out float[n] = in[i][0] / in[i][1];
 *   TRHIP_PROBE_SQRT: in float[n], out float[n] = sqrt(in[i]).
 * in, out: DEVICE pointers (in is ignored, and may be NULL, for the first
 * two).  first + n <= 2^24 for SINCOS2PI and LOG1M.  Asynchronous on
 * `stream`.  Errors: INVALID_ARG (unknown op, NULL pointer, range), HIP.
 */
enum {
    TRHIP_PROBE_SINCOS2PI = 0,
    TRHIP_PROBE_LOG1M = 1,
    TRHIP_PROBE_PHILOX = 2,
    TRHIP_PROBE_DIV = 3,
    TRHIP_PROBE_SQRT = 4
};
trhip_status trhip_numerics_probe(int32_t op, const void* in, void* out, uint64_t n, uint64_t first, void* stream);

/*
 * Batched persistent rendering of many scenes (e.g. NLOS datasets, Sec. 4.5)
 * by one graph launch.  The scenes are split into classes by stack-link
 * width (at most 32,768 triangles, or more) and film length (at most 640
 * bins, or more); each class runs one persistent launch of its own shape,
 * whose workgroups pop work items, (scene, pixel tile) pairs ordered by
 * estimated cost (largest first), from a global cursor.  The classes'
 * cursor resets and persistent kernels are captured once into a hipGraph,
 * so trhip_batch_render is one graph launch.  tile_pixels, when the caller
 * sets it, is every scene's pixels per item; when chosen, each class takes
 * either one pixel count for all its scenes or, for a scale s, max(1,
 * floor(s * 1026 / (T + 2))) pixels per item for a scene with T bins (so
 * longer films take fewer pixels).
 *
 * scenes: HOST array of n_scenes live scene handles; renders: HOST array of
 * n_scenes render descriptions (overrides must be NULL; flags may only hold
 * TRHIP_FLAG_PIXEL_CENTRE and TRHIP_FLAG_NLOS_AREA_SAMPLING; kernel/tile/block
 * fields are ignored); films:
 * HOST array of n_scenes DEVICE pointers, films[i] of scene i's film layout.
 * Unlike every other entry point, the batch keeps the scene handles and
 * the film pointers: the caller keeps them valid until trhip_batch_destroy.
 * Each film receives exactly what trhip_render_transient would write for
 * the same scene and render description.
 */
typedef struct trhip_batch trhip_batch;

typedef struct {
    uint32_t block_size;    /* workgroup size (multiple of 64, <= 256); 0 = choose */
    uint32_t tile_pixels;   /* pixels per work item; 0 = choose */
    uint32_t groups_per_cu; /* persistent workgroups per compute unit; 0 = choose */
    uint32_t kernel;        /* TRHIP_KERNEL_PATH or TRHIP_KERNEL_DEFERRED per work item; 0 = choose */
    int32_t autotune;       /* nonzero: time the candidate shapes for every field left 0 during
                               trhip_batch_create (renders into the films), per class, and keep the
                               fastest; the choice is cached for the same class shape in the process
                               and in the file TRHIP_TUNE_CACHE (default ~/.cache/trhip/batch_tune.txt),
                               which later processes load instead of tuning again */
} trhip_batch_opts;

typedef struct {
    uint32_t n_scenes;
    uint32_t n_items;       /* work items per render, all classes */
    uint32_t block_size, tile_pixels, groups; /* shape of the costliest class (tile_pixels: of its
                                                 costliest scene) */
    uint32_t kernel;        /* TRHIP_KERNEL_PATH or TRHIP_KERNEL_DEFERRED, costliest class */
    uint32_t stack_depth;   /* deepest BVH of the batch */
    size_t lds_bytes;       /* dynamic LDS per workgroup, the largest class */
    uint32_t candidates;    /* shapes timed by the autotuner, all classes (0: none, or cached) */
    float tune_ms;          /* wall time spent autotuning */
    float best_ms;          /* measured render time of the chosen shapes, summed (0 if not timed) */
    uint32_t n_classes;     /* persistent launches per render (scene classes) */
} trhip_batch_info;

/* Errors: INVALID_ARG, BAD_HANDLE (a scene), UNSUPPORTED (LDS), OOM, HIP.
 * Synchronises `stream`. */
trhip_status trhip_batch_create(trhip_scene* const* scenes, const trhip_render_desc* renders, uint32_t n_scenes,
                                float* const* films, const trhip_batch_opts* opts, void* stream,
                                trhip_batch** out);
/* One graph launch on `stream`.  Errors: BAD_HANDLE, HIP. */
trhip_status trhip_batch_render(trhip_batch* batch, void* stream);
trhip_status trhip_batch_get_info(const trhip_batch* batch, trhip_batch_info* info);
/* Waits for the device, frees the batch (not the scenes or films).  NULL is accepted. */
trhip_status trhip_batch_destroy(trhip_batch* batch);

/*
 * Forward-mode derivative (Sec. 4.4, "forward mode differentiation"): the
 * film of trhip_render_transient and, in the same pass, its derivative
 * along a direction of the per-triangle parameters,
 *   dfilm = sum_k (dfilm/dalbedo_k) tangent_albedo[k]
 *         + (dfilm/droughness_k) tangent_roughness[k],
 * for the estimator at the render's seed with the sampling held fixed (the
 * gradient that trhip_render_transient_backward transposes: for any dL/dfilm
 * the two satisfy <dL/dfilm, dfilm> = <grad_albedo, tangent_albedo> +
 * <grad_roughness, tangent_roughness>).  One parameter pi_i is the
 * indicator direction of the triangles it controls.
 *
 * render: as for trhip_render_transient (kernel, tile and block fields:
 * path per lane; TRHIP_FLAG_FROZEN_PROPOSAL for roughness directions that
 * finite differences at a fixed seed can check).  tangent_albedo,
 * tangent_roughness: DEVICE float[n_triangles] (caller order) or NULL for a
 * zero component.  film, dfilm: DEVICE float[n_pixels][n_bins]; steady:
 * DEVICE float[n_pixels] or NULL.
 * Errors: INVALID_ARG, BAD_HANDLE, UNSUPPORTED (LDS), HIP.
 */
trhip_status trhip_render_transient_tangent(trhip_scene* scene, const trhip_render_desc* render,
                                            const float* tangent_albedo, const float* tangent_roughness, float* film,
                                            float* dfilm, float* steady, void* stream);

/*
 * Frequency-space (phasor) film, Sec. 4.3: per pixel and frequency f_j
 * (cycles per metre of optical path, i.e. Omega_j = 2 pi f_j in the
 * exp(-i Omega t) of Eq. 13 with t in metres), the Monte Carlo estimate of
 * Eq. 14: (1/N) sum over the contributions c of the pixel's N paths of
 * c exp(-2 pi i f_j tof), accumulated per sample during rendering with no
 * time histogram and no window (every contribution counts, so the
 * transform covers all t).  tof is the optical path length that the time
 * histogram bins (camera unwarping and the confocal convention apply).
 * The phase is reduced exactly to one cycle of FP32 f_j * tof, so it is
 * accurate while f_j * tof stays far below 2^23 cycles.
 *
 * render: as for trhip_render_transient (kernel WAVEFRONT is UNSUPPORTED;
 * ACCUMULATE adds into phasor and steady).  freqs: HOST float[n_freq],
 * 1 <= n_freq <= TRHIP_MAX_FREQS, finite (0 gives the steady image as a
 * real number).  phasor: DEVICE float[n_pixels][n_freq][2] (re, im), the
 * layout of a complex64 array [H][W][n_freq]; steady: DEVICE float[n_pixels]
 * or NULL.  The same paths as trhip_render_transient with the same render
 * description.
 * Errors: INVALID_ARG, BAD_HANDLE, UNSUPPORTED, HIP.
 */
#define TRHIP_MAX_FREQS 32
trhip_status trhip_render_phasor(trhip_scene* scene, const trhip_render_desc* render, const float* freqs,
                                 uint32_t n_freq, float* phasor, float* steady, void* stream);

/*
 * Photon-count (shot) noise for synthetic captures, a measurement-free
 * stand-in for the device noise that Sec. 4.5 ("Realistic hardware noise")
 * adds to simulated NLOS captures.  Reads film[i] as the expected count
 * scale * film[i] and writes one draw of it: out[i] = N_i / scale with
 * N_i ~ Poisson(scale * film[i]) (exact inversion in FP64 up to a mean of
 * 2^16, the normal approximation above; non-positive values give 0).
 * film, out: DEVICE float[n] (out may equal film); scale > 0 and finite;
 * the draws depend only on (seed, i, film[i], scale).
 * Errors: INVALID_ARG (NULL pointer with n > 0, bad scale), HIP.
 */
trhip_status trhip_poisson_noise(const float* film, float* out, uint64_t n, float scale, uint64_t seed,
                                 void* stream);

/* Static strings; never NULL. */
const char* trhip_status_string(trhip_status status);
const char* trhip_last_error(void);
const char* trhip_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TRHIP_H */
