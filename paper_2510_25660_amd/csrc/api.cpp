// api.cpp -- C ABI of the transient path tracer (see include/trhip.h).
//
// Host-side responsibilities: validate every argument before any HIP call,
// own the scene's device memory, choose the launch shape (pixels per tile,
// workgroup size) within the LDS budget, and enqueue the kernels on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/trhip.h"
#include "internal.h"
#include "scene_view.h"

namespace {

constexpr uint32_t kSceneMagic = 0x54524850u;  // "TRHP"
constexpr size_t kLdsBudget = 64 * 1024;       // bytes per workgroup
constexpr uint32_t kMaxBlock = 256;

thread_local std::string g_last_error;

trhip_status fail(trhip_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
trhip_status fail(trhip_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

trhip_status hip_fail(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(TRHIP_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return fail(TRHIP_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

}  // namespace

struct trhip_scene {
    uint32_t magic;
    int device;
    trhip::SceneView view;
    trhip::BvhBuild bvh;
    uint8_t* d_mat;
    float* d_albedo;
    float* d_rough;
    float* d_scan;
    double* d_grad;  // 2 * n_tris doubles of backward workspace
    uint32_t n_pixels;
    size_t device_bytes;
};

namespace {

// live handles, so that a destroyed or foreign handle is reported instead of
// dereferenced
std::mutex g_live_mutex;
std::unordered_set<const trhip_scene*> g_live;

bool is_live(const trhip_scene* s)
{
    std::lock_guard<std::mutex> lock(g_live_mutex);
    return s && g_live.count(s) != 0;
}

trhip_status check_scene(const trhip_scene* s)
{
    if (!is_live(s) || s->magic != kSceneMagic) return fail(TRHIP_ERR_BAD_HANDLE, "invalid scene handle");
    return TRHIP_OK;
}

void free_scene(trhip_scene* s)
{
    (void)hipFree(s->bvh.nodes);
    (void)hipFree(s->bvh.tris);
    (void)hipFree(s->d_mat);
    (void)hipFree(s->d_albedo);
    (void)hipFree(s->d_rough);
    (void)hipFree(s->d_scan);
    (void)hipFree(s->d_grad);
    s->magic = 0;
    delete s;
}

trhip_status validate_desc(const trhip_scene_desc* d, std::vector<float>& tri9)
{
    if (!d) return fail(TRHIP_ERR_INVALID_ARG, "scene desc is NULL");
    if (!d->vertices || !d->indices || !d->mat_type || !d->albedo || !d->roughness)
        return fail(TRHIP_ERR_INVALID_ARG, "scene arrays must be non-NULL");
    if (d->n_triangles == 0 || d->n_vertices == 0) return fail(TRHIP_ERR_INVALID_ARG, "empty scene");
    if (d->n_triangles > (1u << 30)) return fail(TRHIP_ERR_INVALID_ARG, "too many triangles");
    if (d->sensor != TRHIP_SENSOR_PINHOLE && d->sensor != TRHIP_SENSOR_CONFOCAL)
        return fail(TRHIP_ERR_INVALID_ARG, "unknown sensor %d", d->sensor);
    if (d->width == 0 || d->height == 0) return fail(TRHIP_ERR_INVALID_ARG, "film has no pixels");
    if ((uint64_t)d->width * d->height > (1ull << 31)) return fail(TRHIP_ERR_INVALID_ARG, "film too large");
    if (d->n_bins == 0 || d->n_bins > (1u << 24)) return fail(TRHIP_ERR_INVALID_ARG, "n_bins out of range");
    if (!(d->bin_width > 0.0f) || !std::isfinite(d->bin_width) || !std::isfinite(d->bin_start))
        return fail(TRHIP_ERR_INVALID_ARG, "bin_width must be > 0 and finite");
    if (!(d->sigma_t >= 0.0f) || !std::isfinite(d->sigma_t))
        return fail(TRHIP_ERR_INVALID_ARG, "sigma_t must be >= 0");
    if (d->sigma_t > 0.0f && !(d->medium_albedo >= 0.0f && d->medium_albedo <= 1.0f))
        return fail(TRHIP_ERR_INVALID_ARG, "medium_albedo must lie in [0, 1]");
    if (d->sensor == TRHIP_SENSOR_PINHOLE) {
        if (!finite3(d->cam_origin) || !finite3(d->cam_right) || !finite3(d->cam_up) || !finite3(d->cam_fwd) ||
            !std::isfinite(d->tan_x) || !std::isfinite(d->tan_y))
            return fail(TRHIP_ERR_INVALID_ARG, "camera parameters must be finite");
        if (!finite3(d->light_pos) || !(d->light_intensity >= 0.0f))
            return fail(TRHIP_ERR_INVALID_ARG, "light must be finite with intensity >= 0");
    } else {
        if (!d->scan_points) return fail(TRHIP_ERR_INVALID_ARG, "confocal sensor needs scan_points");
        if (!finite3(d->wall_normal) || !(d->wall_albedo >= 0.0f) || !(d->laser_power >= 0.0f))
            return fail(TRHIP_ERR_INVALID_ARG, "wall parameters invalid");
        if (d->camera_unwarp) return fail(TRHIP_ERR_INVALID_ARG, "camera_unwarp applies to the pinhole sensor");
        const size_t np = (size_t)d->width * d->height;
        for (size_t i = 0; i < np; ++i)
            if (!finite3(d->scan_points + 3 * i)) return fail(TRHIP_ERR_INVALID_ARG, "scan point %zu not finite", i);
    }
    for (uint64_t i = 0; i < 3ull * d->n_vertices; ++i)
        if (!std::isfinite(d->vertices[i])) return fail(TRHIP_ERR_INVALID_ARG, "vertex coordinate not finite");
    tri9.resize(9ull * d->n_triangles);
    for (uint32_t k = 0; k < d->n_triangles; ++k) {
        const uint32_t* id = d->indices + 3ull * k;
        for (int j = 0; j < 3; ++j) {
            if (id[j] >= d->n_vertices) return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: index out of range", k);
            std::memcpy(&tri9[9ull * k + 3 * j], d->vertices + 3ull * id[j], 3 * sizeof(float));
        }
        const float* t = &tri9[9ull * k];
        const float e1[3] = {t[3] - t[0], t[4] - t[1], t[5] - t[2]};
        const float e2[3] = {t[6] - t[0], t[7] - t[1], t[8] - t[2]};
        const float cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                    cz = e1[0] * e2[1] - e1[1] * e2[0];
        if (cx == 0.0f && cy == 0.0f && cz == 0.0f)
            return fail(TRHIP_ERR_INVALID_ARG, "triangle %u has zero area", k);
        if (d->mat_type[k] != TRHIP_MAT_LAMBERT && d->mat_type[k] != TRHIP_MAT_GGX)
            return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: unknown material %u", k, d->mat_type[k]);
        if (!(d->albedo[k] > 0.0f && d->albedo[k] <= 1.0f))
            return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: albedo must lie in (0, 1]", k);
        if (!(d->roughness[k] > 0.0f && d->roughness[k] <= 1.0f))
            return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: roughness must lie in (0, 1]", k);
    }
    return TRHIP_OK;
}

template <class T>
hipError_t upload(T** dst, const T* src, size_t n, hipStream_t s)
{
    hipError_t e = hipMalloc(dst, n * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, s);
}

void fill_view(trhip_scene* s, const trhip_scene_desc* d)
{
    trhip::SceneView& v = s->view;
    std::memset(&v, 0, sizeof(v));
    v.nodes = s->bvh.nodes;
    v.tris = s->bvh.tris;
    v.mat = s->d_mat;
    v.albedo = s->d_albedo;
    v.rough = s->d_rough;
    v.scan = s->d_scan;
    v.root = s->bvh.root;
    for (int a = 0; a < 3; ++a) {
        v.root_lo[a] = s->bvh.root_lo[a];
        v.root_hi[a] = s->bvh.root_hi[a];
    }
    v.n_tris = d->n_triangles;
    v.stack_depth = std::max<uint32_t>(1u, s->bvh.depth);
    v.sensor = d->sensor;
    v.width = d->width;
    v.height = d->height;
    std::memcpy(v.cam_o, d->cam_origin, sizeof(v.cam_o));
    std::memcpy(v.cam_r, d->cam_right, sizeof(v.cam_r));
    std::memcpy(v.cam_u, d->cam_up, sizeof(v.cam_u));
    std::memcpy(v.cam_f, d->cam_fwd, sizeof(v.cam_f));
    v.tan_x = d->tan_x;
    v.tan_y = d->tan_y;
    std::memcpy(v.wall_n, d->wall_normal, sizeof(v.wall_n));
    v.wall_albedo = d->wall_albedo;
    v.laser_power = d->laser_power;
    std::memcpy(v.light, d->light_pos, sizeof(v.light));
    v.intensity = d->light_intensity;
    v.sigma_t = d->sigma_t;
    v.medium_albedo = d->medium_albedo;
    v.n_bins = d->n_bins;
    v.bin_width = d->bin_width;
    v.bin_start = d->bin_start;
    v.unwarp = d->camera_unwarp ? 1 : 0;
}

trhip_status validate_render(const trhip_scene* s, const trhip_render_desc* r)
{
    if (!r) return fail(TRHIP_ERR_INVALID_ARG, "render desc is NULL");
    if (r->spp == 0) return fail(TRHIP_ERR_INVALID_ARG, "spp must be >= 1");
    if (r->max_depth == 0 || r->max_depth > 1024) return fail(TRHIP_ERR_INVALID_ARG, "max_depth out of range");
    if ((uint64_t)r->sample_offset + r->spp > (1ull << 32))
        return fail(TRHIP_ERR_INVALID_ARG, "sample index range exceeds 32 bits");
    if (r->block_size != 0 && (r->block_size % 64 != 0 || r->block_size > kMaxBlock))
        return fail(TRHIP_ERR_INVALID_ARG, "block_size must be a multiple of 64 and <= %u", kMaxBlock);
    if (r->flags & ~(uint32_t)(TRHIP_FLAG_PIXEL_CENTRE | TRHIP_FLAG_ACCUMULATE | TRHIP_FLAG_FROZEN_PROPOSAL))
        return fail(TRHIP_ERR_INVALID_ARG, "unknown flag bits");
    return TRHIP_OK;
}

// Launch shape: enough pixels per tile that a workgroup has ~block samples
// of work, capped by the LDS budget (tile film + traversal stacks).
trhip_status choose_shape(const trhip_scene* s, const trhip_render_desc* r, bool backward, bool primal,
                          uint32_t* tile, uint32_t* block)
{
    const uint32_t T = s->view.n_bins, depth = s->view.stack_depth;
    uint32_t bs = r->block_size ? r->block_size : kMaxBlock;
    if (!r->block_size) {
        // small per-tile work: narrower groups keep more of them in flight
        if ((uint64_t)s->n_pixels * r->spp < 256ull * 1024) bs = 64;
    }
    uint32_t tp = r->tile_pixels;
    if (!tp) {
        tp = std::max<uint32_t>(1u, (bs + r->spp - 1) / r->spp);
        tp = std::min<uint32_t>(tp, s->n_pixels);
        while (tp > 1) {
            const size_t b = backward ? trhip::backward_lds_bytes(tp, T, bs, depth, primal)
                                      : trhip::render_lds_bytes(tp, T, bs, depth);
            if (b <= kLdsBudget) break;
            tp /= 2;
        }
    }
    if ((uint64_t)tp * r->spp >= (1ull << 32))
        return fail(TRHIP_ERR_INVALID_ARG, "tile_pixels * spp must stay below 2^32");
    const size_t need = backward ? trhip::backward_lds_bytes(tp, T, bs, depth, primal)
                                 : trhip::render_lds_bytes(tp, T, bs, depth);
    if (need > kLdsBudget)
        return fail(TRHIP_ERR_UNSUPPORTED, "launch needs %zu bytes of LDS (tile %u x %u bins, block %u, stack %u)",
                    need, tp, T, bs, depth);
    *tile = tp;
    *block = bs;
    return TRHIP_OK;
}

void fill_launch(const trhip_scene* s, const trhip_render_desc* r, uint32_t tile, trhip::LaunchArgs* L)
{
    std::memset(L, 0, sizeof(*L));
    L->spp = r->spp;
    L->sample_offset = r->sample_offset;
    L->max_depth = r->max_depth;
    L->stream_id = r->stream_id;
    L->key0 = (uint32_t)(r->seed & 0xffffffffu);
    L->key1 = (uint32_t)(r->seed >> 32);
    L->flags = r->flags;
    L->tile_pixels = tile;
    L->n_pixels = s->n_pixels;
    L->norm = 1.0f / (float)(r->norm_spp ? r->norm_spp : r->spp);
    L->albedo = r->albedo_override ? r->albedo_override : s->d_albedo;
    L->rough_eval = r->roughness_override ? r->roughness_override : s->d_rough;
    L->rough_sample = (r->flags & TRHIP_FLAG_FROZEN_PROPOSAL) ? s->d_rough : L->rough_eval;
}

}  // namespace

extern "C" {

trhip_status trhip_scene_create(const trhip_scene_desc* desc, void* stream, trhip_scene** out)
{
    if (!out) return fail(TRHIP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::vector<float> tri9;
    trhip_status st = validate_desc(desc, tri9);
    if (st != TRHIP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    trhip_scene* sc = new (std::nothrow) trhip_scene();
    if (!sc) return fail(TRHIP_ERR_OOM, "host allocation failed");
    std::memset(sc, 0, sizeof(*sc));
    hipError_t e = hipGetDevice(&sc->device);
    float* d_tri9 = nullptr;
    const uint32_t nt = desc->n_triangles;
    sc->n_pixels = desc->width * desc->height;
    if (e == hipSuccess) e = upload(&d_tri9, tri9.data(), tri9.size(), s);
    if (e == hipSuccess) e = upload(&sc->d_mat, desc->mat_type, nt, s);
    if (e == hipSuccess) e = upload(&sc->d_albedo, desc->albedo, nt, s);
    if (e == hipSuccess) e = upload(&sc->d_rough, desc->roughness, nt, s);
    if (e == hipSuccess && desc->sensor == TRHIP_SENSOR_CONFOCAL)
        e = upload(&sc->d_scan, desc->scan_points, 3ull * sc->n_pixels, s);
    if (e == hipSuccess) e = hipMalloc(&sc->d_grad, 2ull * nt * sizeof(double));
    if (e == hipSuccess) e = trhip::build_bvh(d_tri9, nt, s, &sc->bvh);
    (void)hipFree(d_tri9);
    if (e != hipSuccess) {
        free_scene(sc);
        return hip_fail(e, "scene upload / BVH build");
    }
    sc->magic = kSceneMagic;
    fill_view(sc, desc);
    {
        std::lock_guard<std::mutex> lock(g_live_mutex);
        g_live.insert(sc);
    }
    sc->device_bytes = (size_t)sc->bvh.n_internal * sizeof(trhip::BvhNode) + (size_t)nt * sizeof(trhip::TriRec) +
                       (size_t)nt * (1 + 4 + 4 + 16) + (sc->d_scan ? 12ull * sc->n_pixels : 0);
    *out = sc;
    return TRHIP_OK;
}

trhip_status trhip_scene_destroy(trhip_scene* scene)
{
    if (!scene) return TRHIP_OK;
    {
        std::lock_guard<std::mutex> lock(g_live_mutex);
        if (!g_live.erase(scene)) return fail(TRHIP_ERR_BAD_HANDLE, "invalid scene handle");
    }
    (void)hipDeviceSynchronize();
    free_scene(scene);
    return TRHIP_OK;
}

trhip_status trhip_scene_get_info(const trhip_scene* scene, trhip_scene_info* info)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if (!info) return fail(TRHIP_ERR_INVALID_ARG, "info is NULL");
    info->n_triangles = scene->view.n_tris;
    info->n_pixels = scene->n_pixels;
    info->n_bins = scene->view.n_bins;
    info->bvh_internal_nodes = scene->bvh.n_internal;
    info->bvh_depth = scene->bvh.depth;
    info->box_pad = scene->bvh.pad;
    info->device_bytes = scene->device_bytes;
    return TRHIP_OK;
}

trhip_status trhip_render_transient(trhip_scene* scene, const trhip_render_desc* render, float* film, float* steady,
                                    float* oow, void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (!film) return fail(TRHIP_ERR_INVALID_ARG, "film is NULL");
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, false, false, &tile, &block)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = film;
    L.steady = steady;
    L.oow = oow;
    hipError_t e = trhip::launch_render(scene->view, L, block, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return TRHIP_OK;
}

trhip_status trhip_render_transient_counted(trhip_scene* scene, const trhip_render_desc* render, float* film,
                                            float* steady, float* oow, uint64_t* counts, void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (!film || !counts) return fail(TRHIP_ERR_INVALID_ARG, "film and counts must be non-NULL");
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, false, false, &tile, &block)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = film;
    L.steady = steady;
    L.oow = oow;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d_counts = nullptr;
    hipError_t e = hipMalloc(&d_counts, TRHIP_COUNT_N * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemsetAsync(d_counts, 0, TRHIP_COUNT_N * sizeof(unsigned long long), s);
    if (e == hipSuccess) e = trhip::launch_render(scene->view, L, block, s, d_counts);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts, d_counts, TRHIP_COUNT_N * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_counts);
    if (e != hipSuccess) return hip_fail(e, "counted render");
    return TRHIP_OK;
}

trhip_status trhip_render_transient_backward(trhip_scene* scene, const trhip_render_desc* render,
                                             const float* grad_film, float* grad_albedo, float* grad_roughness,
                                             float* primal_film, void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (!grad_film || !grad_albedo || !grad_roughness)
        return fail(TRHIP_ERR_INVALID_ARG, "grad_film, grad_albedo and grad_roughness must be non-NULL");
    if (render->flags & TRHIP_FLAG_ACCUMULATE)
        return fail(TRHIP_ERR_INVALID_ARG, "ACCUMULATE does not apply to the backward pass");
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, true, primal_film != nullptr, &tile, &block)) != TRHIP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t nt = scene->view.n_tris;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.grad_film = grad_film;
    L.g_alb = scene->d_grad;
    L.g_rough = scene->d_grad + nt;
    L.primal = primal_film;
    hipError_t e = trhip::launch_zero_f64(scene->d_grad, 2 * nt, s);
    if (e == hipSuccess) e = trhip::launch_backward(scene->view, L, block, s);
    if (e == hipSuccess) e = trhip::launch_f64_to_f32(scene->d_grad, grad_albedo, nt, s);
    if (e == hipSuccess) e = trhip::launch_f64_to_f32(scene->d_grad + nt, grad_roughness, nt, s);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return TRHIP_OK;
}

const char* trhip_status_string(trhip_status status)
{
    switch (status) {
    case TRHIP_OK: return "ok";
    case TRHIP_ERR_INVALID_ARG: return "invalid argument";
    case TRHIP_ERR_OOM: return "out of memory";
    case TRHIP_ERR_HIP: return "HIP runtime error";
    case TRHIP_ERR_UNSUPPORTED: return "unsupported";
    case TRHIP_ERR_BAD_HANDLE: return "bad handle";
    default: return "unknown status";
    }
}

const char* trhip_last_error(void) { return g_last_error.c_str(); }

const char* trhip_version(void) { return "trhip 0.1.0 (gfx950)"; }

}  // extern "C"
