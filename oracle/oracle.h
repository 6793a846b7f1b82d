/*
 * oracle.h -- interface of the CPU reference for transient path tracing.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_SENSOR_PINHOLE 0
#define ORC_SENSOR_CONFOCAL 1
#define ORC_MAT_LAMBERT 0
#define ORC_MAT_GGX 1
#define ORC_MAT_DIELECTRIC 2   /* smooth interface; inside = against e1 x e2 */
#define ORC_MAX_VERT 64

typedef struct {
    int n_tris;
    const float* tri;         /* [n_tris][3 vertices][xyz] */
    const uint8_t* mat;       /* ORC_MAT_* */
    const float* albedo;      /* Lambertian albedo or GGX reflectance F */
    const float* roughness;   /* GGX alpha */
    float light_pos[3];
    float light_intensity;    /* W/sr, isotropic point light */
    int sensor;               /* ORC_SENSOR_* */
    float cam_origin[3], cam_right[3], cam_up[3], cam_fwd[3];
    float tan_x, tan_y;
    int width, height;        /* film pixels (pinhole) or scan grid (confocal) */
    const float* scan_points; /* [width*height][3], confocal */
    float wall_normal[3];
    float wall_albedo, laser_power;
    float sigma_t, medium_albedo; /* sigma_t == 0: no medium */
    int n_bins;
    float bin_width, bin_start;
    int camera_unwarp;
    /* refractive indices and scattering delays (Eqs. 3 and 10) */
    const float* ior;         /* [n_tris] index inside dielectric triangles' meshes, or NULL */
    const float* delay;       /* [n_tris] mean scattering delay (metres of OPL), or NULL = none */
    float medium_ior;         /* index of the space around the meshes (0 means 1) */
} orc_scene;

typedef struct {
    int spp;
    uint32_t sample_offset;
    int max_depth;            /* path segments, device segments included */
    uint64_t seed;
    uint32_t stream_id;
    int pixel_centre;
    int frozen_proposal;      /* GGX: sample with scene roughness, evaluate with `roughness` */
    const float* albedo;      /* optional per-triangle overrides */
    const float* roughness;
    int nlos_area;            /* confocal: area-sample the hidden vertex (Sec. 4.5) */
} orc_render;

typedef struct {
    int tri;                  /* -1: medium vertex */
    int has_c, has_cont, bin;
    float c, opl_c;
    double dn_alb, dn_rough, dc_alb, dc_rough; /* d log f, NEE / continuation */
} orc_vertex;

typedef struct {
    int n_vert;
    orc_vertex v[ORC_MAX_VERT];
} orc_path;

/* one next-event contribution (orc_render_records) */
typedef struct {
    uint32_t pixel, sample;
    int32_t vertex, bin;
    float value, tof;
    int32_t tri;
    uint32_t reserved;
} orc_record;

typedef struct orc_prepared orc_prepared;

orc_prepared* orc_prepare(const orc_scene* sc);
void orc_release(orc_prepared* p);
float orc_pad(const orc_prepared* p);
double orc_area_total(const orc_prepared* p);
float orc_fresnel(float ci, float eta_i, float eta_t); /* unpolarised dielectric reflectance */

int orc_trace_path(const orc_prepared* p, const orc_render* r, uint32_t pix, uint32_t sample, orc_path* rec);
int64_t orc_render_records(const orc_prepared* p, const orc_render* r, const int32_t* pixels, int n_pix,
                           orc_record* out, int64_t cap);
int orc_render_film(const orc_prepared* p, const orc_render* r, const int32_t* pixels, int n_pix,
                    double* film, double* steady, double* oow, int nthreads);
/* forward-mode derivative (Sec. 4.4): film and dfilm [n_pix][T], dfilm the
 * derivative along (v_alb, v_rough) (either may be NULL) */
int orc_render_tangent(const orc_prepared* p, const orc_render* r, const int32_t* pixels, int n_pix,
                       const double* v_alb, const double* v_rough, double* film, double* dfilm, double* steady,
                       int nthreads);
/* phasor film of Sec. 4.3 (Eq. 14): phasor[n_pix][n_freq][2] = (re, im) of
 * (1/N) sum c exp(-2 pi i f tof), f in cycles per metre of optical path */
int orc_render_phasor(const orc_prepared* p, const orc_render* r, const int32_t* pixels, int n_pix,
                      const double* freqs, int n_freq, double* phasor, double* steady, int nthreads);
int orc_backward(const orc_prepared* p, const orc_render* r, const int32_t* pixels, int n_pix,
                 const float* grad_film, double* g_alb, double* g_rough, double* primal_film, int nthreads);

int orc_closest_hit(const orc_prepared* p, const float o[3], const float d[3], int exclude, int use_bvh,
                    float* t, int* prim);

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_uniform(uint32_t x);
void orc_sincos2pi(float u, float* s, float* c);
float orc_log1m(float u);
void orc_cosine_sample(float u0, float u1, float out[3]);
void orc_phase_sample(float u0, float u1, float out[3]);
float orc_ggx_f(const float wo[3], const float wi[3], float alpha, float F);
float orc_ggx_pdf(const float wo[3], const float wi[3], float alpha);
void orc_ggx_sample(const float wo[3], float alpha, float u0, float u1, float wi[3]);
double orc_ggx_dlogf_dalpha(const float wo[3], const float wi[3], double alpha);

void orc_sincos2pi_n(int64_t n, const float* u, float* s, float* c);
void orc_log1m_n(int64_t n, const float* u, float* out);
void orc_ggx_eval_n(int64_t n, const float* wo, const float* wi, const float* alpha, const float* F,
                    float* f_out, float* pdf_out);
void orc_ggx_sample_n(int64_t n, const float* wo, const float* alpha, const float* alpha_s, const float* F,
                      int frozen, const float* u0, const float* u1, float* wi_out, float* w_out);
void orc_cosine_sample_n(int64_t n, const float* u0, const float* u1, float* out);
void orc_phase_sample_n(int64_t n, const float* u0, const float* u1, float* out);
void orc_philox_n(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out);

#ifdef __cplusplus
}
#endif
#endif
