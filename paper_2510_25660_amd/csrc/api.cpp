// api.cpp -- C ABI of the transient path tracer (see include/trhip.h).
//
// Host-side responsibilities: validate every argument before any HIP call,
// own the scene's device memory, choose the launch shape (pixels per tile,
// workgroup size) within the LDS budget, and enqueue the kernels on the
// caller's stream.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/trhip.h"
#include "internal.h"
#include "scene_view.h"

static_assert(trhip::kWorkCounters == TRHIP_COUNT_N, "counting build and ABI agree");

namespace {

constexpr uint32_t kSceneMagic = 0x54524850u;  // "TRHP"
constexpr size_t kLdsBudget = 63 * 1024;       // dynamic LDS bytes per workgroup
constexpr uint32_t kMaxBlock = 256;
constexpr size_t kCuLds = 160 * 1024;            // LDS bytes per CU
constexpr uint32_t kPathWavesPerSimd = 4;        // k_render's register budget allows 4 waves per SIMD

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
    float* d_ior;    // nullptr: no dielectric triangle
    float* d_delay;  // nullptr: no scattering delay
    double* d_grad;  // backward workspace: 2 * n_tris doubles, or [2][n_tris][2] fixed-point words (4 * n_tris)
    // deferred form with sample chunks: partial films of chunks 1..
    float* d_chunk_scratch;
    unsigned long long* d_fixed_film;  // deterministic HBM-film form (allocated on first use)
    size_t fixed_film_words;
    size_t chunk_scratch_floats;
    // confocal: NLOS area-sampling tables, one set per scan region
    double* d_area_cdf;      // [region][n_tris] prefix sums of the weights (caller order)
    float* d_area_invp;      // [region][n_tris] inverse area densities
    uint32_t* d_area_guide;  // [region][guide_cells + 1] guide tables
    double* d_area_wtotal;   // [region] weight totals
    uint8_t* d_area_region;  // [scan point] region
    uint32_t* d_sorted_of;   // BVH-order index of each caller triangle
    uint32_t guide_cells;
    double area_total;       // area of the sampling set
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
    (void)hipFree(s->d_ior);
    (void)hipFree(s->d_delay);
    (void)hipFree(s->d_grad);
    (void)hipFree(s->d_chunk_scratch);
    (void)hipFree(s->d_fixed_film);
    (void)hipFree(s->d_area_cdf);
    (void)hipFree(s->d_area_invp);
    (void)hipFree(s->d_sorted_of);
    (void)hipFree(s->d_area_guide);
    (void)hipFree(s->d_area_wtotal);
    (void)hipFree(s->d_area_region);
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
    if (d->bvh_builder != TRHIP_BVH_PLOC && d->bvh_builder != TRHIP_BVH_LBVH)
        return fail(TRHIP_ERR_INVALID_ARG, "unknown bvh_builder %d", d->bvh_builder);
    if (!(d->sigma_t >= 0.0f) || !std::isfinite(d->sigma_t))
        return fail(TRHIP_ERR_INVALID_ARG, "sigma_t must be >= 0");
    if (d->sigma_t > 0.0f && !(d->medium_albedo >= 0.0f && d->medium_albedo <= 1.0f))
        return fail(TRHIP_ERR_INVALID_ARG, "medium_albedo must lie in [0, 1]");
    if (!(d->medium_ior == 0.0f || (d->medium_ior > 0.0f && d->medium_ior <= 100.0f)))
        return fail(TRHIP_ERR_INVALID_ARG, "medium_ior must be 0 (= 1) or in (0, 100]");
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
        if (d->mat_type[k] != TRHIP_MAT_LAMBERT && d->mat_type[k] != TRHIP_MAT_GGX &&
            d->mat_type[k] != TRHIP_MAT_DIELECTRIC)
            return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: unknown material %u", k, d->mat_type[k]);
        if (d->mat_type[k] == TRHIP_MAT_DIELECTRIC) {
            if (!d->ior) return fail(TRHIP_ERR_INVALID_ARG, "triangle %u is dielectric but ior is NULL", k);
            if (!(d->ior[k] > 0.0f && d->ior[k] <= 100.0f))
                return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: ior must lie in (0, 100]", k);
        } else {
            if (!(d->albedo[k] > 0.0f && d->albedo[k] <= 1.0f))
                return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: albedo must lie in (0, 1]", k);
            if (!(d->roughness[k] > 0.0f && d->roughness[k] <= 1.0f))
                return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: roughness must lie in (0, 1]", k);
        }
        if (d->delay && !(d->delay[k] >= 0.0f && std::isfinite(d->delay[k])))
            return fail(TRHIP_ERR_INVALID_ARG, "triangle %u: delay must be finite and >= 0", k);
    }
    return TRHIP_OK;
}

constexpr int kAreaG = 4;                  // scan-point regions per axis
constexpr int kAreaRegions = kAreaG * kAreaG;

// Tables of NLOS area sampling.  The sampling set is every triangle not
// lying in the relay wall's plane (the plane through the first scan point
// with normal wn, within 1e-6 * (1 + largest |coordinate|)): seen from a scan
// point those subtend no solid angle.  The np scan points are split into
// kAreaG x kAreaG regions of their bounding box over its two axes of
// largest extent (the larger first, ties to the lower axis); region r has
// its own triangle pdf: triangle k of the set with weight
// w_k = A_k (g_k + g_max / 20), A_k its area and g_k = (cos_s cos_h / r^2)^2 the
// squared geometry term between the region's representative c (the mean of
// its scan points; of all scan points if it has none) and the triangle's
// centroid (d = centroid - c, r = |d|, cos_s = wn . d / r clamped at 0,
// cos_h = |n_k . d| / r), g_max the region's largest g_k; the floor keeps
// every triangle of the set drawable (all weights A_k if every g_k is 0).
// Fills, region after region, the inclusive prefix sums in caller order
// (cdf, [region][nt]), invp = W_r A_k / w_k (the inverse area density of a
// point drawn uniformly on triangle k; 0 outside the set), the totals W_r,
// each scan point's region, and returns the set's area.  FP64 throughout:
// differences of FP32 coordinates are exact there.
double area_tables(const std::vector<float>& tri9, uint32_t nt, const float* scan, size_t np, const float* wn,
                   std::vector<double>& cdf, std::vector<float>& invp, std::vector<double>& wtotal,
                   std::vector<uint8_t>& region)
{
#pragma clang fp contract(off)
    float maxabs = 0.0f;
    for (const float c : tri9) maxabs = std::max(maxabs, std::fabs(c));
    const double tol = 1e-6 * (1.0 + (double)maxabs);
    const double n[3] = {(double)wn[0], (double)wn[1], (double)wn[2]};
    double lo[3], hi[3], ext[3], all[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = (double)scan[a];
    for (size_t i = 0; i < np; ++i)
        for (int a = 0; a < 3; ++a) {
            const double v = (double)scan[3 * i + a];
            all[a] += v;
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    for (int a = 0; a < 3; ++a) {
        all[a] = all[a] / (double)np;
        ext[a] = hi[a] - lo[a];
    }
    int ax0 = 0;
    for (int a = 1; a < 3; ++a)
        if (ext[a] > ext[ax0]) ax0 = a;
    int ax1 = ax0 == 0 ? 1 : 0;
    for (int a = 0; a < 3; ++a)
        if (a != ax0 && ext[a] > ext[ax1]) ax1 = a;
    double repr[kAreaRegions][3] = {}, cnt[kAreaRegions] = {};
    region.resize(np);
    for (size_t i = 0; i < np; ++i) {
        const int axes[2] = {ax0, ax1};
        int cell[2];
        for (int q = 0; q < 2; ++q) {
            const int b = axes[q];
            const double f = ext[b] > 0.0 ? ((double)scan[3 * i + b] - lo[b]) / ext[b] : 0.0;
            int c = (int)std::floor(f * (double)kAreaG);
            cell[q] = std::min(kAreaG - 1, std::max(0, c));
        }
        const int r = cell[0] * kAreaG + cell[1];
        region[i] = (uint8_t)r;
        cnt[r] += 1.0;
        for (int a = 0; a < 3; ++a) repr[r][a] += (double)scan[3 * i + a];
    }
    for (int r = 0; r < kAreaRegions; ++r)
        for (int a = 0; a < 3; ++a) repr[r][a] = cnt[r] > 0.0 ? repr[r][a] / cnt[r] : all[a];
    std::vector<double> area(nt, 0.0), nrm(3ull * nt, 0.0), cen(3ull * nt, 0.0), geo(nt, 0.0);
    double set_area = 0.0;
    for (uint32_t k = 0; k < nt; ++k) {
        const float* t = &tri9[9ull * k];
        bool on_wall = true;
        for (int j = 0; j < 3; ++j) {
            const double h = ((double)t[3 * j] - (double)scan[0]) * n[0] +
                             ((double)t[3 * j + 1] - (double)scan[1]) * n[1] +
                             ((double)t[3 * j + 2] - (double)scan[2]) * n[2];
            if (std::fabs(h) > tol) on_wall = false;
        }
        if (on_wall) continue;
        double e1[3], e2[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = (double)t[3 + a] - (double)t[a];
            e2[a] = (double)t[6 + a] - (double)t[a];
            cen[3 * k + a] = (((double)t[a] + (double)t[3 + a]) + (double)t[6 + a]) / 3.0;
        }
        const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        area[k] = 0.5 * len;
        for (int a = 0; a < 3; ++a) nrm[3 * k + a] = c[a] / len;
        set_area += area[k];
    }
    cdf.resize((size_t)kAreaRegions * nt);
    invp.resize((size_t)kAreaRegions * nt);
    wtotal.resize(kAreaRegions);
    for (int r = 0; r < kAreaRegions; ++r) {
        double gmax = 0.0;
        for (uint32_t k = 0; k < nt; ++k) {
            geo[k] = 0.0;
            if (!(area[k] > 0.0)) continue;
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = cen[3 * k + a] - repr[r][a];
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 > 0.0) {
                const double rr = std::sqrt(r2);
                double cos_s = (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]) / rr;
                if (cos_s < 0.0) cos_s = 0.0;
                const double cos_h = std::fabs(nrm[3 * k] * d[0] + nrm[3 * k + 1] * d[1] + nrm[3 * k + 2] * d[2]) / rr;
                const double q = (cos_s * cos_h) / r2;
                geo[k] = q * q;
            }
            if (geo[k] > gmax) gmax = geo[k];
        }
        const double floor_w = gmax > 0.0 ? gmax / 20.0 : 1.0;
        double acc = 0.0;
        for (uint32_t k = 0; k < nt; ++k) {
            acc += area[k] * (geo[k] + floor_w);
            cdf[(size_t)r * nt + k] = acc;
        }
        for (uint32_t k = 0; k < nt; ++k) {
            const double w = area[k] * (geo[k] + floor_w);
            invp[(size_t)r * nt + k] = w > 0.0 ? (float)((acc * area[k]) / w) : 0.0f;
        }
        wtotal[r] = acc;
    }
    return set_area;
}

// Guide table of one region's prefix sums (cutpoint method): cells = the
// smallest power of two >= nt / 4 (at least 1, at most 2^20); guide[m] = first
// k with cdf[k] > (m / cells) * total, or nt - 1 if none, for m = 0 .. cells.
uint32_t guide_cells_for(uint32_t nt)
{
    uint32_t cells = 1;
    while (cells < (nt + 3) / 4 && cells < (1u << 20)) cells <<= 1;
    return cells;
}

void area_guide(const double* cdf, uint32_t nt, double total, uint32_t cells, uint32_t* guide)
{
    uint32_t k = 0;
    for (uint32_t m = 0; m <= cells; ++m) {
        const double t = ((double)m / (double)cells) * total;
        while (k < nt - 1 && !(cdf[k] > t)) ++k;
        guide[m] = k;
    }
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
    v.compact = s->bvh.compact ? 1u : 0u;
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
    v.area_cdf = s->d_area_cdf;
    v.sorted_of = s->d_sorted_of;
    v.area_invp = s->d_area_invp;
    v.area_guide = s->d_area_guide;
    v.area_wtotal = s->d_area_wtotal;
    v.area_region = s->d_area_region;
    v.guide_cells = (float)s->guide_cells;
    v.ior = s->d_ior;
    v.delay = s->d_delay;
    v.eta0 = d->medium_ior > 0.0f ? d->medium_ior : 1.0f;
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
    if (r->flags & ~(uint32_t)(TRHIP_FLAG_PIXEL_CENTRE | TRHIP_FLAG_ACCUMULATE | TRHIP_FLAG_FROZEN_PROPOSAL |
                               TRHIP_FLAG_NLOS_AREA_SAMPLING | TRHIP_FLAG_DETERMINISTIC))
        return fail(TRHIP_ERR_INVALID_ARG, "unknown flag bits");
    if ((r->flags & TRHIP_FLAG_DETERMINISTIC) && r->kernel != TRHIP_KERNEL_AUTO && r->kernel != TRHIP_KERNEL_PATH)
        return fail(TRHIP_ERR_UNSUPPORTED, "DETERMINISTIC renders run the path form only");
    if (r->kernel > TRHIP_KERNEL_DEFERRED) return fail(TRHIP_ERR_INVALID_ARG, "unknown kernel %u", r->kernel);
    if (r->flags & TRHIP_FLAG_NLOS_AREA_SAMPLING) {
        if (s->view.sensor != TRHIP_SENSOR_CONFOCAL)
            return fail(TRHIP_ERR_UNSUPPORTED, "NLOS area sampling needs the confocal sensor");
        if (r->max_depth < 4)
            return fail(TRHIP_ERR_UNSUPPORTED, "NLOS area sampling needs a hidden vertex (max_depth >= 4)");
        if (s->view.sigma_t > 0.0f) return fail(TRHIP_ERR_UNSUPPORTED, "NLOS area sampling excludes media");
        if (!(s->area_total > 0.0))
            return fail(TRHIP_ERR_UNSUPPORTED, "NLOS area sampling: no triangle off the relay wall's plane");
        if (r->kernel == TRHIP_KERNEL_WAVEFRONT)
            return fail(TRHIP_ERR_UNSUPPORTED, "the wavefront form has no NLOS area sampling");
    }
    return TRHIP_OK;
}

enum class Kind { Path, Wavefront, Deferred, Backward, BackwardPrimal, Tangent, PathFixed, BackwardFixed,
                  BackwardPrimalFixed, PathHbm, PathFixedHbm };

// stack: LDS bytes of one lane's traversal stack
size_t lds_bytes(Kind kind, uint32_t tp, uint32_t T, uint32_t bs, uint32_t stack)
{
    switch (kind) {
    case Kind::Path: return trhip::render_lds_bytes(tp, T, bs, stack);
    case Kind::Wavefront: return trhip::wavefront_lds_bytes(tp, T, bs, stack);
    case Kind::Deferred: return trhip::deferred_lds_bytes(tp, T, bs, stack);
    case Kind::Backward: return trhip::backward_lds_bytes(tp, T, bs, stack, false, false);
    case Kind::Tangent: return trhip::tangent_lds_bytes(tp, T, bs, stack);
    case Kind::PathFixed: return trhip::fixed_lds_bytes(tp, T, bs, stack);
    // the HBM form needs only its stacks; the shape must also fit the LDS
    // form, which renders instead when the scratch film cannot be allocated
    case Kind::PathFixedHbm: return trhip::fixed_lds_bytes(tp, T, bs, stack);
    case Kind::PathHbm: return trhip::hbm_lds_bytes(bs, stack);
    case Kind::BackwardFixed: return trhip::backward_lds_bytes(tp, T, bs, stack, false, true);
    case Kind::BackwardPrimalFixed: return trhip::backward_lds_bytes(tp, T, bs, stack, true, true);
    default: return trhip::backward_lds_bytes(tp, T, bs, stack, true, false);
    }
}

uint32_t lane_stack_bytes(const trhip_scene* s) { return trhip::stack_lane_bytes(s->view.n_tris, s->view.stack_depth); }

// Launch shape: enough pixels per tile that a workgroup has ~block samples
// of work, capped by the LDS budget (tile film + traversal stacks, plus the
// path slots and queues of the wavefront form).
// words: floats of one pixel's film (0: the time bins)
trhip_status choose_shape(const trhip_scene* s, const trhip_render_desc* r, Kind kind, uint32_t* tile,
                          uint32_t* block, uint32_t words = 0)
{
    const uint32_t T = words ? words : s->view.n_bins;
    const uint32_t depth = kind == Kind::PathHbm ? trhip::hbm_stack_lane_bytes(s->view.n_tris, s->view.stack_depth)
                                                 : lane_stack_bytes(s);
    uint32_t bs = r->block_size ? r->block_size : kMaxBlock;
    if (!r->block_size) {
        // small per-tile work: narrower groups keep more of them in flight
        if ((uint64_t)s->n_pixels * r->spp < 256ull * 1024) bs = 64;
        while (bs > 64 && lds_bytes(kind, 1, T, bs, depth) > kLdsBudget) bs /= 2;
    }
    auto tile_for = [&](uint32_t b) {
        uint32_t t = std::max<uint32_t>(1u, (b + r->spp - 1) / r->spp);
        t = std::min<uint32_t>(t, s->n_pixels);
        while (t > 1 && lds_bytes(kind, t, T, b, depth) > kLdsBudget) t /= 2;
        return t;
    };
    uint32_t tp = r->tile_pixels;
    // Film in HBM on a scene too large for an XCD's L2: 64-lane workgroups
    // of one pixel (for >= 64 spp), whose tiles the 8 x 8 pixel-block order
    // keeps together (1M-triangle scene: +8.5 % over 256 lanes).
    if ((kind == Kind::PathHbm || kind == Kind::PathFixedHbm) && !r->block_size && !r->tile_pixels &&
        !trhip::short_stack(s->view.n_tris))
        bs = 64;
    if (!tp) {
        tp = tile_for(bs);
        // The path-per-lane kernel holds kPathWavesPerSimd waves per SIMD by
        // its registers.  When the LDS of a full-width workgroup (deep 32-bit
        // stacks, a wide tile film) would hold fewer, 64-lane workgroups keep
        // the CU as full and balance better (1M-triangle scene: +6 %).
        if (kind == Kind::Path && !r->block_size && bs > 64 &&
            (kCuLds / lds_bytes(kind, tp, T, bs, depth)) * (bs / 64) < 4u * kPathWavesPerSimd) {
            bs = 64;
            tp = tile_for(bs);
        }
    }
    if ((uint64_t)tp * r->spp >= (1ull << 32))
        return fail(TRHIP_ERR_INVALID_ARG, "tile_pixels * spp must stay below 2^32");
    const size_t need = lds_bytes(kind, tp, T, bs, depth);
    if (need > kLdsBudget)
        return fail(TRHIP_ERR_UNSUPPORTED,
                    "launch needs %zu bytes of LDS (tile %u x %u bins, block %u, stack %u bytes per lane)",
                    need, tp, T, bs, depth);
    *tile = tp;
    *block = bs;
    return TRHIP_OK;
}

// Forward kernel form.  Measured on MI355X: deferring first hits pays when
// most first rays leave the scene (confocal NLOS: +25%) and costs when
// nearly all of them hit (closed pinhole scenes: -28%), so the automatic
// choice follows the sensor; the wavefront form is never faster here.
// Film length from which the path form keeps the film in HBM (no LDS film)
// on scenes too large for 16-bit stack links: there a pixel's LDS row of
// 2 KB or more next to the deep 32-bit stacks is what limits the workgroups
// per CU (1M-triangle scene: 1,024 bins 256 -> 366 Mpath-samples/s with
// whole stacks in LDS, 442 with split stacks; 512 bins 297 -> 367); on small
// scenes the LDS film is as fast or faster (box room, 512 bins: 965 against
// 881).
constexpr uint32_t kHbmFilmBins = 512;

bool hbm_film(const trhip_scene* s) { return s->view.n_bins >= kHbmFilmBins && !trhip::short_stack(s->view.n_tris); }

// histogram: a time histogram (the phasor film keeps its tile film in LDS)
Kind forward_kind(const trhip_scene* s, const trhip_render_desc* r, bool histogram = true)
{
    if (r->flags & TRHIP_FLAG_DETERMINISTIC) return histogram && hbm_film(s) ? Kind::PathFixedHbm : Kind::PathFixed;
    if (r->kernel == TRHIP_KERNEL_PATH || (r->kernel == TRHIP_KERNEL_AUTO && s->view.sensor != TRHIP_SENSOR_CONFOCAL))
        return histogram && hbm_film(s) ? Kind::PathHbm : Kind::Path;
    if (r->kernel == TRHIP_KERNEL_WAVEFRONT) return Kind::Wavefront;
    if (r->kernel == TRHIP_KERNEL_DEFERRED) return Kind::Deferred;
    if (s->view.sensor != TRHIP_SENSOR_CONFOCAL) return Kind::Path;
    const uint32_t bs = r->block_size ? r->block_size : 64;
    return lds_bytes(Kind::Deferred, 1, s->view.n_bins, bs, lane_stack_bytes(s)) <= kLdsBudget ? Kind::Deferred
                                                                                                 : Kind::Path;
}

// Scratch of the deferred form's sample chunks (the partial films of chunks
// 1..), grown on demand and kept by the scene (which one stream uses at a
// time).  Nothing is allocated while the stream is being captured into a
// graph: *ready stays false and the launch keeps one chunk per tile, which
// renders the same film.
hipError_t ensure_chunk_scratch(trhip_scene* sc, size_t floats, hipStream_t s, bool* ready)
{
    *ready = false;
    if (sc->chunk_scratch_floats >= floats) {
        *ready = true;
        return hipSuccess;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess || cs != hipStreamCaptureStatusNone) return e;
    e = hipStreamSynchronize(s);  // earlier launches may still use the old buffer
    if (e != hipSuccess) return e;
    (void)hipFree(sc->d_chunk_scratch);
    sc->d_chunk_scratch = nullptr;
    sc->chunk_scratch_floats = 0;
    e = hipMalloc(&sc->d_chunk_scratch, floats * sizeof(float));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {  // one chunk per tile renders the same film
        (void)hipGetLastError();
        sc->d_chunk_scratch = nullptr;
        return hipSuccess;
    }
    if (e != hipSuccess) return e;
    sc->chunk_scratch_floats = floats;
    *ready = true;
    return hipSuccess;
}

// Fixed-point film of the deterministic HBM-film form, grown on demand and
// kept by the scene like the chunk scratch (nothing allocated under graph
// capture: the LDS form then renders the same sums).
hipError_t ensure_fixed_film(trhip_scene* sc, size_t words, hipStream_t s, bool* ready)
{
    *ready = false;
    if (sc->fixed_film_words >= words) {
        *ready = true;
        return hipSuccess;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess || cs != hipStreamCaptureStatusNone) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    (void)hipFree(sc->d_fixed_film);
    sc->d_fixed_film = nullptr;
    sc->fixed_film_words = 0;
    e = hipMalloc(&sc->d_fixed_film, words * sizeof(unsigned long long));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {  // the LDS form renders the same sums
        (void)hipGetLastError();
        sc->d_fixed_film = nullptr;
        return hipSuccess;
    }
    if (e != hipSuccess) return e;
    sc->fixed_film_words = words;
    *ready = true;
    return hipSuccess;
}

// floats of the chunk scratch: (chunks - 1) partial films, steady and oow
size_t chunk_scratch_floats(const trhip::LaunchArgs& L, uint32_t chunks, uint32_t words)
{
    return (size_t)(chunks - 1) * ((size_t)L.n_pixels * words + 2ull * L.n_pixels);
}

hipError_t launch_forward(trhip_scene* sc, Kind kind, trhip::LaunchArgs L, uint32_t block, hipStream_t stream,
                          unsigned long long* counts)
{
    switch (kind) {
    case Kind::PathFixed: return trhip::launch_render_fixed(sc->view, L, block, stream);
    case Kind::PathFixedHbm: {
        // the HBM form's limb words stay exact for fewer than 2^21 adds per sum
        if ((uint64_t)L.spp * L.max_depth >= (1ull << 21)) return trhip::launch_render_fixed(sc->view, L, block, stream);
        bool ready = false;
        const hipError_t e = ensure_fixed_film(sc, trhip::fixed_film_words(L.n_pixels, sc->view.n_bins), stream,
                                               &ready);
        if (e != hipSuccess) return e;
        if (!ready) return trhip::launch_render_fixed(sc->view, L, block, stream);  // same sums, LDS form
        L.fixed_film = sc->d_fixed_film;
        return trhip::launch_render_fixed_hbm(sc->view, L, block, stream);
    }
    case Kind::PathHbm: return trhip::launch_render_hbm(sc->view, L, block, stream, counts);
    case Kind::Wavefront: return trhip::launch_render_wavefront(sc->view, L, block, stream, counts);
    case Kind::Deferred: {
        uint32_t chunk_spp = L.spp;
        const uint32_t chunks = trhip::deferred_chunks(L.spp, block, &chunk_spp);
        const uint32_t words = L.n_freq ? 2 * L.n_freq : sc->view.n_bins;
        if (chunks > 1) {
            bool ready = false;
            const hipError_t e = ensure_chunk_scratch(sc, chunk_scratch_floats(L, chunks, words), stream, &ready);
            if (e != hipSuccess) return e;
            if (ready) {
                L.chunks = chunks;
                L.chunk_spp = chunk_spp;
                L.chunk_scratch = sc->d_chunk_scratch;
            }
        }
        hipError_t e = trhip::launch_render_deferred(sc->view, L, block, stream, counts);
        if (e == hipSuccess && L.chunks > 1) e = trhip::launch_add_planes(L, words, stream);
        return e;
    }
    default: return trhip::launch_render(sc->view, L, block, stream, counts);
    }
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
    L->chunks = 1;
    L->chunk_spp = r->spp;
    L->norm = 1.0f / (float)(r->norm_spp ? r->norm_spp : r->spp);
    L->norm_spp = r->norm_spp ? r->norm_spp : r->spp;
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
    std::vector<double> cdf, wtotal;
    std::vector<uint32_t> guide;
    std::vector<float> invp;
    std::vector<uint8_t> region;
    if (e == hipSuccess && desc->sensor == TRHIP_SENSOR_CONFOCAL) {
        e = upload(&sc->d_scan, desc->scan_points, 3ull * sc->n_pixels, s);
        sc->area_total = area_tables(tri9, nt, desc->scan_points, (size_t)sc->n_pixels, desc->wall_normal, cdf, invp,
                                     wtotal, region);
        sc->guide_cells = guide_cells_for(nt);
        guide.resize((size_t)kAreaRegions * (sc->guide_cells + 1));
        for (int r = 0; r < kAreaRegions; ++r)
            area_guide(cdf.data() + (size_t)r * nt, nt, wtotal[r], sc->guide_cells,
                       guide.data() + (size_t)r * (sc->guide_cells + 1));
        if (e == hipSuccess) e = upload(&sc->d_area_cdf, cdf.data(), cdf.size(), s);
        if (e == hipSuccess) e = upload(&sc->d_area_invp, invp.data(), invp.size(), s);
        if (e == hipSuccess) e = upload(&sc->d_area_guide, guide.data(), guide.size(), s);
        if (e == hipSuccess) e = upload(&sc->d_area_wtotal, wtotal.data(), wtotal.size(), s);
        if (e == hipSuccess) e = upload(&sc->d_area_region, region.data(), region.size(), s);
        if (e == hipSuccess) e = hipMalloc(&sc->d_sorted_of, (size_t)nt * sizeof(uint32_t));
    }
    bool any_dielectric = false, any_delay = false;
    for (uint32_t k = 0; k < nt; ++k) {
        any_dielectric = any_dielectric || desc->mat_type[k] == TRHIP_MAT_DIELECTRIC;
        any_delay = any_delay || (desc->delay && desc->delay[k] > 0.0f);
    }
    if (e == hipSuccess && any_dielectric) e = upload(&sc->d_ior, desc->ior, nt, s);
    if (e == hipSuccess && any_delay) e = upload(&sc->d_delay, desc->delay, nt, s);
    if (e == hipSuccess) e = hipMalloc(&sc->d_grad, 4ull * nt * sizeof(double));
    if (e == hipSuccess)
        e = trhip::build_bvh(d_tri9, nt, desc->bvh_builder == TRHIP_BVH_LBVH ? trhip::kBuilderLbvh : trhip::kBuilderPloc,
                             s, &sc->bvh);
    if (e == hipSuccess && sc->d_sorted_of) e = trhip::launch_sorted_of(sc->bvh.tris, sc->bvh.compact, nt, sc->d_sorted_of, s);
    if (e == hipSuccess && sc->d_sorted_of) e = hipStreamSynchronize(s);
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
    sc->device_bytes = (size_t)sc->bvh.n_internal * (sc->bvh.compact ? sizeof(trhip::CompactNode)
                                                                      : sizeof(trhip::BvhNode)) +
                       (size_t)nt * (sc->bvh.compact ? sizeof(trhip::TriRecBox) : sizeof(trhip::TriRec)) +
                       (size_t)nt * (1 + 4 + 4 + 32) + (sc->d_scan ? 13ull * sc->n_pixels + 4ull * nt + (size_t)kAreaRegions * (12ull * nt + 4ull * (sc->guide_cells + 1) + 8) : 0) +
                       (sc->d_ior ? 4ull * nt : 0) + (sc->d_delay ? 4ull * nt : 0);
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
    const Kind kind = forward_kind(scene, render);
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, kind, &tile, &block)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = film;
    L.steady = steady;
    L.oow = oow;
    hipError_t e = launch_forward(scene, kind, L, block, (hipStream_t)stream, nullptr);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return TRHIP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free forward render
// ---------------------------------------------------------------------------
// Scratch of trhip_render_transient_noalloc: the deferred form's partial
// tiles and per-tile counters, in a device array that every GPU the library
// runs on holds from the library's load until the process ends.  Host code
// never uses the array's name as an address: each device's copy is looked up
// once with hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t kStaticScratchBytes = 32ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mutex;
std::unordered_map<int, unsigned char*> g_scratch_ptr;  // device -> its copy of `scratch`

// with `device` current
hipError_t static_scratch(int device, unsigned char** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    const auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
    *out = static_cast<unsigned char*>(p);
    return hipSuccess;
}

}  // namespace

extern "C" {

trhip_status trhip_render_transient_noalloc(trhip_scene* scene, const trhip_render_desc* render, float* film,
                                            float* steady, float* oow, void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (!film) return fail(TRHIP_ERR_INVALID_ARG, "film is NULL");
    const Kind kind = forward_kind(scene, render);
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, kind, &tile, &block)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = film;
    L.steady = steady;
    L.oow = oow;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    switch (kind) {
    case Kind::PathFixed:
    case Kind::PathFixedHbm: e = trhip::launch_render_fixed(scene->view, L, block, s); break;  // no scratch film
    case Kind::PathHbm: e = trhip::launch_render_hbm(scene->view, L, block, s, nullptr); break;
    case Kind::Wavefront: e = trhip::launch_render_wavefront(scene->view, L, block, s, nullptr); break;
    case Kind::Deferred: {
        uint32_t chunk_spp = L.spp;
        const uint32_t chunks = trhip::deferred_chunks(L.spp, block, &chunk_spp);
        const uint32_t words = scene->view.n_bins;
        if (chunks > 1) {
            const size_t need = chunk_scratch_floats(L, chunks, words) * sizeof(float);
            if (need > kStaticScratchBytes)
                return fail(TRHIP_ERR_UNSUPPORTED,
                            "this render needs %zu bytes of scratch; the allocation-free render holds %zu "
                            "(use trhip_render_transient, or fewer samples per pixel per call)",
                            need, kStaticScratchBytes);
            int dev = -1;
            e = hipGetDevice(&dev);
            if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
            if (dev != scene->device)
                return fail(TRHIP_ERR_INVALID_ARG, "the scene lives on device %d, device %d is current", scene->device,
                            dev);
            unsigned char* base = nullptr;
            e = static_scratch(dev, &base);
            if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
            L.chunks = chunks;
            L.chunk_spp = chunk_spp;
            L.chunk_scratch = reinterpret_cast<float*>(base);
        }
        // every plane of the scratch is written in full before it is read
        e = trhip::launch_render_deferred(scene->view, L, block, s, nullptr);
        if (e == hipSuccess && L.chunks > 1) e = trhip::launch_add_planes(L, words, s);
        break;
    }
    default: e = trhip::launch_render(scene->view, L, block, s, nullptr);
    }
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return TRHIP_OK;
}

static_assert(TRHIP_MAX_FREQS == trhip::kMaxFreq, "phasor frequency limit");

trhip_status trhip_render_phasor(trhip_scene* scene, const trhip_render_desc* render, const float* freqs,
                                 uint32_t n_freq, float* phasor, float* steady, void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (render->flags & TRHIP_FLAG_DETERMINISTIC)
        return fail(TRHIP_ERR_UNSUPPORTED, "DETERMINISTIC applies to the forward render and the backward pass, not the phasor film");
    if (!phasor) return fail(TRHIP_ERR_INVALID_ARG, "phasor is NULL");
    if (!freqs || n_freq == 0 || n_freq > trhip::kMaxFreq)
        return fail(TRHIP_ERR_INVALID_ARG, "freqs must hold 1..%u frequencies", trhip::kMaxFreq);
    for (uint32_t j = 0; j < n_freq; ++j)
        if (!std::isfinite(freqs[j])) return fail(TRHIP_ERR_INVALID_ARG, "freqs[%u] is not finite", j);
    if (render->kernel == TRHIP_KERNEL_WAVEFRONT)
        return fail(TRHIP_ERR_UNSUPPORTED, "the wavefront form has no phasor film");
    const Kind kind = forward_kind(scene, render, false);
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, kind, &tile, &block, 2 * n_freq)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = phasor;
    L.steady = steady;
    L.oow = nullptr;
    L.n_freq = n_freq;
    for (uint32_t j = 0; j < n_freq; ++j) L.freq[j] = freqs[j];
    hipError_t e = launch_forward(scene, kind, L, block, (hipStream_t)stream, nullptr);
    if (e != hipSuccess) return hip_fail(e, "phasor launch");
    return TRHIP_OK;
}

trhip_status trhip_render_transient_tangent(trhip_scene* scene, const trhip_render_desc* render,
                                            const float* tangent_albedo, const float* tangent_roughness, float* film,
                                            float* dfilm, float* steady, void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (render->flags & TRHIP_FLAG_DETERMINISTIC)
        return fail(TRHIP_ERR_UNSUPPORTED, "DETERMINISTIC applies to the forward render and the backward pass, not the forward-mode render");
    if (!film || !dfilm) return fail(TRHIP_ERR_INVALID_ARG, "film and dfilm must be non-NULL");
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, Kind::Tangent, &tile, &block)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = film;
    L.dfilm = dfilm;
    L.steady = steady;
    L.tan_albedo = tangent_albedo;
    L.tan_rough = tangent_roughness;
    hipError_t e = trhip::launch_render_tangent(scene->view, L, block, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "tangent launch");
    return TRHIP_OK;
}

trhip_status trhip_render_transient_counted(trhip_scene* scene, const trhip_render_desc* render, float* film,
                                            float* steady, float* oow, uint64_t* counts, void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (render->flags & TRHIP_FLAG_DETERMINISTIC)
        return fail(TRHIP_ERR_UNSUPPORTED, "DETERMINISTIC applies to the forward render and the backward pass, not the counting build");
    if (!film || !counts) return fail(TRHIP_ERR_INVALID_ARG, "film and counts must be non-NULL");
    const Kind kind = forward_kind(scene, render);
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, kind, &tile, &block)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = film;
    L.steady = steady;
    L.oow = oow;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d_counts = nullptr;
    hipError_t e = hipMalloc(&d_counts, TRHIP_COUNT_N * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemsetAsync(d_counts, 0, TRHIP_COUNT_N * sizeof(unsigned long long), s);
    if (e == hipSuccess) e = launch_forward(scene, kind, L, block, s, d_counts);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts, d_counts, TRHIP_COUNT_N * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_counts);
    if (e != hipSuccess) return hip_fail(e, "counted render");
    return TRHIP_OK;
}

static_assert(sizeof(trhip_record) == sizeof(trhip::ContribRecord), "record layout");
static_assert(offsetof(trhip_record, value) == offsetof(trhip::ContribRecord, value), "record layout");
static_assert(offsetof(trhip_record, tri) == offsetof(trhip::ContribRecord, tri), "record layout");

trhip_status trhip_render_transient_records(trhip_scene* scene, const trhip_render_desc* render,
                                            const uint8_t* pixel_mask, trhip_record* records, uint64_t capacity,
                                            uint64_t* n_records, float* film, float* steady, float* oow,
                                            void* stream)
{
    trhip_status st = check_scene(scene);
    if (st != TRHIP_OK) return st;
    if ((st = validate_render(scene, render)) != TRHIP_OK) return st;
    if (render->flags & TRHIP_FLAG_DETERMINISTIC)
        return fail(TRHIP_ERR_UNSUPPORTED, "DETERMINISTIC applies to the forward render and the backward pass, not the recording build");
    if (!film || !pixel_mask || !n_records)
        return fail(TRHIP_ERR_INVALID_ARG, "film, pixel_mask and n_records must be non-NULL");
    if (capacity > 0 && !records) return fail(TRHIP_ERR_INVALID_ARG, "records is NULL with capacity > 0");
    const Kind kind = forward_kind(scene, render);
    uint32_t tile = 0, block = 0;
    if ((st = choose_shape(scene, render, kind, &tile, &block)) != TRHIP_OK) return st;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.film = film;
    L.steady = steady;
    L.oow = oow;
    L.record_mask = pixel_mask;
    L.records = reinterpret_cast<trhip::ContribRecord*>(records);
    L.record_cap = capacity;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d_count = nullptr;
    hipError_t e = hipMalloc(&d_count, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemsetAsync(d_count, 0, sizeof(unsigned long long), s);
    L.record_count = d_count;
    if (e == hipSuccess) e = launch_forward(scene, kind, L, block, s, nullptr);
    unsigned long long n = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&n, d_count, sizeof(n), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_count);
    if (e != hipSuccess) return hip_fail(e, "recording render");
    *n_records = n;
    return TRHIP_OK;
}

trhip_status trhip_numerics_probe(int32_t op, const void* in, void* out, uint64_t n, uint64_t first, void* stream)
{
    if (op < TRHIP_PROBE_SINCOS2PI || op > TRHIP_PROBE_SQRT) return fail(TRHIP_ERR_INVALID_ARG, "unknown probe %d", op);
    if (n == 0) return TRHIP_OK;
    if (!out) return fail(TRHIP_ERR_INVALID_ARG, "out is NULL");
    const bool uniforms = op == TRHIP_PROBE_SINCOS2PI || op == TRHIP_PROBE_LOG1M;
    if (!uniforms && !in) return fail(TRHIP_ERR_INVALID_ARG, "in is NULL");
    if (uniforms && (first > (1ull << 24) || n > (1ull << 24) - first))
        return fail(TRHIP_ERR_INVALID_ARG, "first + n must not exceed 2^24");
    if (n > (1ull << 40)) return fail(TRHIP_ERR_INVALID_ARG, "n too large");
    static_assert(TRHIP_PROBE_SINCOS2PI == trhip::kProbeSinCos2Pi && TRHIP_PROBE_SQRT == trhip::kProbeSqrt,
                  "probe numbering");
    hipError_t e = trhip::launch_probe(op, in, out, n, first, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "probe launch");
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
    const bool fixed = (render->flags & TRHIP_FLAG_DETERMINISTIC) != 0;
    const Kind kind = fixed ? (primal_film ? Kind::BackwardPrimalFixed : Kind::BackwardFixed)
                            : (primal_film ? Kind::BackwardPrimal : Kind::Backward);
    if ((st = choose_shape(scene, render, kind, &tile, &block)) !=
        TRHIP_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t nt = scene->view.n_tris;
    trhip::LaunchArgs L;
    fill_launch(scene, render, tile, &L);
    L.grad_film = grad_film;
    L.g_alb = scene->d_grad;
    L.g_rough = scene->d_grad + nt;
    L.g_fixed = fixed ? reinterpret_cast<unsigned long long*>(scene->d_grad) : nullptr;
    L.primal = primal_film;
    // single trace with a register stash when a path has few continuations,
    // path replay otherwise (or when asked for with TRHIP_KERNEL_PATH)
    const int vmax = (scene->view.sensor == TRHIP_SENSOR_CONFOCAL) ? (int)render->max_depth - 3
                                                                    : (int)render->max_depth - 1;
    int max_cont = 0;
    if (render->kernel != TRHIP_KERNEL_PATH) max_cont = (vmax - 1 <= 2) ? 2 : (vmax - 1 <= 7 ? 7 : 0);
    hipError_t e = trhip::launch_zero_f64(scene->d_grad, (fixed ? 4 : 2) * nt, s);
    if (e == hipSuccess) e = trhip::launch_backward(scene->view, L, block, max_cont, s);
    if (fixed) {
        if (e == hipSuccess) e = trhip::launch_fixed_to_f32(L.g_fixed, grad_albedo, nt, s);
        if (e == hipSuccess) e = trhip::launch_fixed_to_f32(L.g_fixed + 2 * nt, grad_roughness, nt, s);
    } else {
        if (e == hipSuccess) e = trhip::launch_f64_to_f32(scene->d_grad, grad_albedo, nt, s);
        if (e == hipSuccess) e = trhip::launch_f64_to_f32(scene->d_grad + nt, grad_roughness, nt, s);
    }
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return TRHIP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched persistent rendering
// ---------------------------------------------------------------------------
constexpr uint32_t kBatchMagic = 0x54524842u;  // "TRHB"
constexpr uint64_t kBatchKernelRevision = 4;   // bump when the persistent kernel's performance model changes

// The scenes of a batch are split into classes by stack-link width (16-bit
// links and buffer loads up to 32,768 triangles, 32-bit links above) and
// film length (up to kBatchLongFilm bins, or more).  Each class has its own
// persistent launch with its own shape, so that one large scene does not put
// every scene on 32-bit links and the longest film does not size every
// workgroup's LDS; the classes' launches follow one another in the batch's
// graph, the costliest first.
constexpr uint32_t kBatchLongFilm = 640;

struct BatchClass {
    std::vector<uint32_t> order;  // scene indices in processing order (largest cost first)
    double cost;
    bool short_links;
    uint32_t depth;               // deepest BVH of the class
    uint32_t* d_item_start;
    uint32_t* d_order;
    uint32_t* d_cursor;
    trhip::BatchTables tables;
    uint32_t block, tile, groups;  // groups: per CU while tuning, workgroups once captured
    bool deferred;
    size_t lds;
    uint32_t timed;
    float best_ms;
};

struct trhip_batch {
    uint32_t magic;
    std::vector<trhip_scene*> scenes;
    std::vector<trhip::SceneView> views;
    std::vector<trhip::LaunchArgs> args;  // tile_pixels filled by the shape of the scene's class
    trhip::SceneView* d_views;
    trhip::LaunchArgs* d_args;
    std::vector<BatchClass> classes;
    hipGraph_t graph;
    hipGraphExec_t exec;
    trhip_batch_info info;
};

namespace {

std::mutex g_batch_mutex;
std::unordered_set<const trhip_batch*> g_live_batches;
std::unordered_map<uint64_t, std::array<uint32_t, 4>> g_tune_cache;  // key -> block, tile, groups, deferred

// The tuner's choices also persist across processes, one line per class
// shape ("key block tile groups deferred", hex key) in the file named by
// TRHIP_TUNE_CACHE, else ~/.cache/trhip/batch_tune.txt; a missing or
// unreadable file is ignored.
std::string tune_cache_path()
{
    if (const char* p = getenv("TRHIP_TUNE_CACHE")) return p;
    const char* home = getenv("HOME");
    return home ? std::string(home) + "/.cache/trhip/batch_tune.txt" : std::string();
}

bool tune_cache_load(uint64_t key, std::array<uint32_t, 4>* out)
{
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return false;
    unsigned long long k = 0;
    unsigned a = 0, b = 0, c = 0, d = 0;
    bool found = false;
    while (fscanf(f, "%llx %u %u %u %u", &k, &a, &b, &c, &d) == 5)
        if (k == key && a && b && c) {
            *out = {a, b, c, d};  // the last line of a key wins
            found = true;
        }
    fclose(f);
    return found;
}

void tune_cache_store(uint64_t key, const std::array<uint32_t, 4>& v)
{
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        const std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    if (FILE* f = fopen(path.c_str(), "a")) {
        fprintf(f, "%016llx %u %u %u %u\n", (unsigned long long)key, v[0], v[1], v[2], v[3]);
        fclose(f);
    }
}

bool batch_live(const trhip_batch* b)
{
    std::lock_guard<std::mutex> lock(g_batch_mutex);
    return b && g_live_batches.count(b) && b->magic == kBatchMagic;
}

void free_batch(trhip_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_views);
    (void)hipFree(b->d_args);
    for (BatchClass& c : b->classes) {
        (void)hipFree(c.d_item_start);
        (void)hipFree(c.d_order);
        (void)hipFree(c.d_cursor);
    }
    b->magic = 0;
    delete b;
}

// A class's tile choice: a scale s (codes 1, 2, 4: a scene with T bins
// takes s * 1,026 floats of LDS film, a pixel of 1,024 bins, divided by its
// film floats per pixel, so that scenes with fewer bins take more pixels per
// item) or a pixel count p for every scene of the class (kFixedTile | p).
constexpr uint32_t kFixedTile = 0x100u;
uint32_t batch_tile(uint32_t code, uint32_t T)
{
    if (code & kFixedTile) return code & (kFixedTile - 1u);
    return std::max<uint32_t>(1u, (code * 1026u) / (T + 2u));
}

// a class's shape -> its tables on the device; *fits false if the LDS does
// not fit (nothing staged then)
hipError_t stage_shape(trhip_batch* b, BatchClass& c, uint32_t block, uint32_t tile_code, uint32_t groups,
                       bool deferred, hipStream_t s, bool* fits)
{
    const uint32_t n = (uint32_t)c.order.size();
    std::vector<uint32_t> start(n + 1, 0);
    uint32_t film_words = 0;
    *fits = true;
    for (uint32_t k = 0; k < n; ++k) {
        const uint32_t i = c.order[k];
        const uint32_t T = b->views[i].n_bins;
        const uint32_t tp = std::min<uint32_t>(batch_tile(tile_code, T), b->scenes[i]->n_pixels);
        b->args[i].tile_pixels = tp;
        film_words = std::max<uint32_t>(film_words, tp * T + 2 * tp);
        if ((uint64_t)tp * b->args[i].spp >= (1ull << 32)) *fits = false;
        start[k + 1] = start[k] + (b->scenes[i]->n_pixels + tp - 1) / tp;
    }
    const size_t lds = trhip::batch_lds_bytes(film_words, block, c.depth * (c.short_links ? 2u : 4u), deferred);
    *fits = *fits && lds <= kLdsBudget;
    if (!*fits) return hipSuccess;
    hipError_t e = hipMemcpyAsync(b->d_args, b->args.data(), b->args.size() * sizeof(trhip::LaunchArgs),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c.d_item_start, start.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    c.tables.views = b->d_views;
    c.tables.args = b->d_args;
    c.tables.item_start = c.d_item_start;
    c.tables.order = c.d_order;
    c.tables.n_scenes = n;
    c.tables.n_items = start[n];
    c.tables.film_words = film_words;
    c.tables.cursor = c.d_cursor;
    c.block = block;
    c.tile = b->args[c.order[0]].tile_pixels;  // pixels per item of the costliest scene
    c.groups = groups;
    c.deferred = deferred;
    c.lds = lds;
    return e;
}

uint64_t tune_key(const trhip_batch* b, const BatchClass& c, int device, const trhip_batch_opts& o)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    // the kernels' build and the GPU model: a cached shape is only reused
    // for the same library and device type
    for (const char* ch = trhip_version(); *ch; ++ch) mix((uint64_t)*ch);
    mix(kBatchKernelRevision);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess)
        for (const char* ch = prop.gcnArchName; *ch; ++ch) mix((uint64_t)*ch);
    mix((uint64_t)device);
    mix(o.block_size);
    mix(o.tile_pixels);
    mix(o.groups_per_cu);
    mix(o.kernel);
    for (uint32_t i : c.order) {
        mix(b->scenes[i]->n_pixels);
        mix(b->views[i].n_bins);
        mix(b->views[i].n_tris);
        mix(b->views[i].stack_depth);
        mix(b->args[i].spp);
        mix(b->args[i].max_depth);
        mix(b->args[i].flags);
    }
    return h;
}

// picks (tunes, or loads) the launch shape of one class and stages it
hipError_t shape_class(trhip_batch* b, BatchClass& c, const trhip_batch_opts& o, int device, int n_cu, hipStream_t s,
                       bool* ok)
{
    *ok = false;
    const std::vector<uint32_t> blocks = o.block_size ? std::vector<uint32_t>{o.block_size}
                                                      : std::vector<uint32_t>{64, 128, 256};
    // the tile choices (batch_tile): the caller's pixels per item, else three
    // scales and three pixel counts
    const std::vector<uint32_t> tiles =
        o.tile_pixels ? std::vector<uint32_t>{kFixedTile | o.tile_pixels}
                      : std::vector<uint32_t>{1, 2, 4, kFixedTile | 2, kFixedTile | 4, kFixedTile | 8};
    const std::vector<uint32_t> gpcs = o.groups_per_cu ? std::vector<uint32_t>{o.groups_per_cu}
                                                       : std::vector<uint32_t>{4, 5, 8};
    const std::vector<uint32_t> forms = o.kernel ? std::vector<uint32_t>{o.kernel}
                                                 : std::vector<uint32_t>{TRHIP_KERNEL_PATH, TRHIP_KERNEL_DEFERRED};
    std::array<uint32_t, 4> best{0, 0, 0, 0};
    const uint64_t key = tune_key(b, c, device, o);
    bool cached = false;
    {
        std::lock_guard<std::mutex> lock(g_batch_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            best = it->second;
            cached = true;
        } else if (o.autotune && tune_cache_load(key, &best)) {
            g_tune_cache[key] = best;
            cached = true;
        }
    }
    hipError_t e = hipSuccess;
    c.timed = 0;
    c.best_ms = 0.0f;
    if (!cached && o.autotune) {
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        e = hipEventCreate(&ev0);
        if (e == hipSuccess) e = hipEventCreate(&ev1);
        float best_t = 0.0f;
        for (uint32_t form : forms)
            for (uint32_t bs : blocks)
                for (uint32_t tp : tiles)
                    for (uint32_t g : gpcs) {
                        if (e != hipSuccess) break;
                        bool fits = false;
                        const bool dfr = form == TRHIP_KERNEL_DEFERRED;
                        e = stage_shape(b, c, bs, tp, g, dfr, s, &fits);
                        if (e != hipSuccess || !fits) continue;
                        const uint32_t groups = std::max<uint32_t>(1u, (uint32_t)n_cu * g);
                        e = trhip::launch_batch(c.tables, groups, bs, c.depth, c.short_links, dfr, s);  // warm-up
                        float ms = 0.0f;
                        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the faster of two launches
                            e = hipEventRecord(ev0, s);
                            if (e == hipSuccess) e = trhip::launch_batch(c.tables, groups, bs, c.depth, c.short_links,
                                                                         dfr, s);
                            if (e == hipSuccess) e = hipEventRecord(ev1, s);
                            if (e == hipSuccess) e = hipEventSynchronize(ev1);
                            float t = 0.0f;
                            if (e == hipSuccess) e = hipEventElapsedTime(&t, ev0, ev1);
                            ms = rep == 0 ? t : std::min(ms, t);
                        }
                        if (e != hipSuccess) break;
                        ++c.timed;
                        if (best[0] == 0 || ms < best_t) {
                            best_t = ms;
                            best = {bs, tp, g, dfr ? 1u : 0u};
                        }
                    }
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (e != hipSuccess) return e;
        c.best_ms = best_t;
        if (best[0]) {
            std::lock_guard<std::mutex> lock(g_batch_mutex);
            g_tune_cache[key] = best;
            tune_cache_store(key, best);
        }
    }
    if (best[0] == 0) {
        // untuned default: deferred form, the largest block whose LDS fits,
        // scale 1, 8 groups per CU
        const bool dfr = o.kernel != TRHIP_KERNEL_PATH;
        for (uint32_t bs : {256u, 128u, 64u}) {
            if (o.block_size && bs != o.block_size) continue;
            bool fits = false;
            const uint32_t g = o.groups_per_cu ? o.groups_per_cu : 8u;
            const uint32_t code = o.tile_pixels ? (kFixedTile | o.tile_pixels) : 1u;
            e = stage_shape(b, c, bs, code, g, dfr, s, &fits);
            if (e != hipSuccess) return e;
            if (fits) {
                best = {bs, code, g, dfr ? 1u : 0u};
                break;
            }
        }
    }
    if (!best[0]) return hipSuccess;
    bool fits = false;
    e = stage_shape(b, c, best[0], best[1], best[2], best[3] != 0, s, &fits);
    *ok = e == hipSuccess && fits;
    return e;
}

}  // namespace

extern "C" {

trhip_status trhip_batch_create(trhip_scene* const* scenes, const trhip_render_desc* renders, uint32_t n_scenes,
                                float* const* films, const trhip_batch_opts* opts, void* stream,
                                trhip_batch** out)
{
    if (!out) return fail(TRHIP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!scenes || !renders || !films || n_scenes == 0)
        return fail(TRHIP_ERR_INVALID_ARG, "scenes, renders and films must be non-empty arrays");
    trhip_batch_opts o{};
    if (opts) o = *opts;
    if (o.block_size != 0 && (o.block_size % 64 != 0 || o.block_size > kMaxBlock))
        return fail(TRHIP_ERR_INVALID_ARG, "block_size must be a multiple of 64 and <= %u", kMaxBlock);
    if (o.groups_per_cu > 64) return fail(TRHIP_ERR_INVALID_ARG, "groups_per_cu must be <= 64");
    if (o.kernel != 0 && o.kernel != TRHIP_KERNEL_PATH && o.kernel != TRHIP_KERNEL_DEFERRED)
        return fail(TRHIP_ERR_INVALID_ARG, "batch kernel must be PATH or DEFERRED");
    for (uint32_t i = 0; i < n_scenes; ++i) {
        trhip_status st = check_scene(scenes[i]);
        if (st != TRHIP_OK) return fail(st, "scene %u: invalid handle", i);
        if ((st = validate_render(scenes[i], &renders[i])) != TRHIP_OK) return st;
        if (renders[i].albedo_override || renders[i].roughness_override)
            return fail(TRHIP_ERR_INVALID_ARG, "scene %u: batched renders take no parameter overrides", i);
        if (renders[i].flags & ~(uint32_t)(TRHIP_FLAG_PIXEL_CENTRE | TRHIP_FLAG_NLOS_AREA_SAMPLING))
            return fail(TRHIP_ERR_INVALID_ARG,
                        "scene %u: batched renders accept only TRHIP_FLAG_PIXEL_CENTRE and TRHIP_FLAG_NLOS_AREA_SAMPLING", i);
        if (!films[i]) return fail(TRHIP_ERR_INVALID_ARG, "scene %u: film is NULL", i);
    }
    hipStream_t s = (hipStream_t)stream;
    trhip_batch* b = new (std::nothrow) trhip_batch();
    if (!b) return fail(TRHIP_ERR_OOM, "host allocation failed");
    b->magic = 0;
    b->scenes.assign(scenes, scenes + n_scenes);
    b->views.resize(n_scenes);
    b->args.resize(n_scenes);
    std::vector<double> cost(n_scenes);
    for (uint32_t i = 0; i < n_scenes; ++i) {
        b->views[i] = scenes[i]->view;
        fill_launch(scenes[i], &renders[i], 1, &b->args[i]);
        b->args[i].film = films[i];
        cost[i] = (double)scenes[i]->n_pixels * renders[i].spp * (double)(scenes[i]->view.stack_depth + 4);
    }
    // classes by link width and film length, scenes in decreasing cost
    std::vector<uint32_t> idx(n_scenes);
    for (uint32_t i = 0; i < n_scenes; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t c) { return cost[a] > cost[c]; });
    for (uint32_t i : idx) {
        const bool sl = trhip::short_stack(scenes[i]->view.n_tris);
        const bool lf = scenes[i]->view.n_bins > kBatchLongFilm;
        BatchClass* c = nullptr;
        for (BatchClass& k : b->classes)
            if (k.short_links == sl && (b->views[k.order[0]].n_bins > kBatchLongFilm) == lf) c = &k;
        if (!c) {
            b->classes.emplace_back();
            c = &b->classes.back();
            c->cost = 0.0;
            c->short_links = sl;
            c->depth = 1;
        }
        c->order.push_back(i);
        c->cost += cost[i];
        c->depth = std::max(c->depth, scenes[i]->view.stack_depth);
    }
    std::stable_sort(b->classes.begin(), b->classes.end(),
                     [](const BatchClass& x, const BatchClass& y) { return x.cost > y.cost; });
    int device = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = hipMalloc(&b->d_views, n_scenes * sizeof(trhip::SceneView));
    if (e == hipSuccess) e = hipMalloc(&b->d_args, n_scenes * sizeof(trhip::LaunchArgs));
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_views, b->views.data(), n_scenes * sizeof(trhip::SceneView), hipMemcpyHostToDevice, s);
    for (BatchClass& c : b->classes) {
        const size_t n = c.order.size();
        if (e == hipSuccess) e = hipMalloc(&c.d_item_start, (n + 1) * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&c.d_order, n * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&c.d_cursor, sizeof(uint32_t));
        if (e == hipSuccess)
            e = hipMemcpyAsync(c.d_order, c.order.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "batch tables");
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (BatchClass& c : b->classes) {
        bool ok = false;
        e = shape_class(b, c, o, device, n_cu, s, &ok);
        if (e != hipSuccess) {
            free_batch(b);
            return hip_fail(e, "batch autotune / staging");
        }
        if (!ok) {
            free_batch(b);
            return fail(TRHIP_ERR_UNSUPPORTED, "no batch launch shape fits in %zu bytes of LDS", kLdsBudget);
        }
    }
    const float tune_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // capture [cursor reset -> persistent kernel] of every class once
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        for (BatchClass& c : b->classes) {
            c.groups = std::max<uint32_t>(1u, (uint32_t)n_cu * c.groups);
            if (le == hipSuccess)
                le = trhip::launch_batch(c.tables, c.groups, c.block, c.depth, c.short_links, c.deferred, cs);
        }
        e = hipStreamEndCapture(cs, &b->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "batch graph capture");
    }
    const BatchClass& c0 = b->classes[0];
    b->info.n_scenes = n_scenes;
    b->info.n_items = 0;
    b->info.candidates = 0;
    b->info.best_ms = 0.0f;
    b->info.stack_depth = 1;
    b->info.lds_bytes = 0;
    for (const BatchClass& c : b->classes) {
        b->info.n_items += c.tables.n_items;
        b->info.candidates += c.timed;
        b->info.best_ms += c.best_ms;
        b->info.stack_depth = std::max(b->info.stack_depth, c.depth);
        b->info.lds_bytes = std::max(b->info.lds_bytes, c.lds);
    }
    b->info.block_size = c0.block;
    b->info.tile_pixels = c0.tile;
    b->info.groups = c0.groups;
    b->info.kernel = c0.deferred ? TRHIP_KERNEL_DEFERRED : TRHIP_KERNEL_PATH;
    b->info.tune_ms = b->info.candidates ? tune_ms : 0.0f;
    b->info.n_classes = (uint32_t)b->classes.size();
    b->magic = kBatchMagic;
    {
        std::lock_guard<std::mutex> lock(g_batch_mutex);
        g_live_batches.insert(b);
    }
    *out = b;
    return TRHIP_OK;
}

trhip_status trhip_batch_render(trhip_batch* batch, void* stream)
{
    if (!batch_live(batch)) return fail(TRHIP_ERR_BAD_HANDLE, "invalid batch handle");
    for (trhip_scene* sc : batch->scenes)
        if (!is_live(sc)) return fail(TRHIP_ERR_BAD_HANDLE, "a scene of the batch was destroyed");
    hipError_t e = hipGraphLaunch(batch->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "batch graph launch");
    return TRHIP_OK;
}

trhip_status trhip_batch_get_info(const trhip_batch* batch, trhip_batch_info* info)
{
    if (!batch_live(batch)) return fail(TRHIP_ERR_BAD_HANDLE, "invalid batch handle");
    if (!info) return fail(TRHIP_ERR_INVALID_ARG, "info is NULL");
    *info = batch->info;
    return TRHIP_OK;
}

trhip_status trhip_batch_destroy(trhip_batch* batch)
{
    if (!batch) return TRHIP_OK;
    {
        std::lock_guard<std::mutex> lock(g_batch_mutex);
        if (!g_live_batches.erase(batch)) return fail(TRHIP_ERR_BAD_HANDLE, "invalid batch handle");
    }
    (void)hipDeviceSynchronize();
    free_batch(batch);
    return TRHIP_OK;
}

}  // extern "C"

extern "C" {

trhip_status trhip_poisson_noise(const float* film, float* out, uint64_t n, float scale, uint64_t seed, void* stream)
{
    if (n == 0) return TRHIP_OK;
    if (!film || !out) return fail(TRHIP_ERR_INVALID_ARG, "film and out must be non-NULL");
    if (!(scale > 0.0f) || !std::isfinite(scale)) return fail(TRHIP_ERR_INVALID_ARG, "scale must be positive and finite");
    hipError_t e = trhip::launch_poisson(film, out, n, scale, seed, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "noise launch");
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
