/*
 * msst_oracle.h -- FP64 CPU oracle for learned sphere tracing of volumetric
 * subsurface scattering (Leonard, Hoehlein, Westermann, arXiv 2011.03082).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct CPU
 * implementation that the HIP library is checked against.  It shares no
 * source, header, table or helper with the GPU library, and the product
 * path never links, loads or calls it: only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg do.
 *
 * Everything is scalar double precision.  Random numbers come from the
 * oracle's own Philox4x32-10, written from Salmon, Moraes, Dror and Shaw,
 * "Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11); the GPU library has
 * an independent implementation of the same published generator, so both
 * sides consume identical uniforms.
 *
 * Counter layout of every draw: (c0 = draw index, c1 = id low word,
 * c2 = id high word, c3 = stream tag); key = (seed low word, seed high word).
 */
#ifndef MSST_ORACLE_H
#define MSST_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Stream tags (word c3 of the Philox counter). */
enum {
    OR_TAG_WALK_EVENT = 0,
    OR_TAG_WALK_PARAM = 1,
    OR_TAG_CVAE_INIT = 2,
    OR_TAG_CVAE_BATCH = 3,
    OR_TAG_CVAE_REPARAM = 4,
    OR_TAG_CVAE_SAMPLE = 5,
    OR_TAG_RENDER_PIXEL = 6,
    OR_TAG_RENDER_PATH = 7,
    OR_TAG_SCENE = 8,
    OR_TAG_DEQUANT = 9
};

/* ---------------- randomness (rng.c) ---------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Fills out[4*n] with the Philox blocks of counters (c0 + j, id, tag), j < n. */
void or_philox_blocks(uint64_t seed, uint32_t tag, uint64_t id, uint32_t c0, int n, uint32_t* out);
double or_u01(uint32_t word);
void or_uniform4(uint64_t seed, uint32_t tag, uint64_t id, uint32_t c0, double u[4]);
void or_normal4(uint64_t seed, uint32_t tag, uint64_t id, uint32_t c0, double nrm[4]);

/* ---------------- scattering primitives (walk.c) ---------------- */
double or_hg_eval(double g, double cos_theta);
double or_hg_sample(double g, double xi);
void or_onb(const double n[3], double b1[3], double b2[3]);
void or_scatter_dir(double d[3], double mu, double azimuth);

/* ---------------- random walk (walk.c) ---------------- */
enum { OR_WALK_ANALOG = 0, OR_WALK_TRAINING = 1 };
enum { OR_EVENT_ALBEDO_POWER = 0, OR_EVENT_UNIFORM = 1 };

typedef struct {
    uint64_t seed, photon_offset, n_photons;
    int32_t mode, event_weighting;
    double sigma_t, g, albedo, radius;
    double st_range[2], g_range[2], albedo_range[2];
    uint32_t max_events;
    int32_t n_threads;
    /* TRAINING: with probability focus_fraction (fourth uniform of the
     * parameter block) sigma_t r and g come from the focus ranges */
    double focus_fraction;
    double focus_st_range[2], focus_g_range[2];
} or_walk_desc;

/* Planar (component-major) outputs, any pointer may be NULL. */
typedef struct {
    double* params;       /* [3][n] sigma_t*r, g, albedo                  */
    uint32_t* n_scatter;  /* [n]                                           */
    uint32_t* event_index;/* [n] representative event k (TRAINING)         */
    uint8_t* absorbed;    /* [n]                                           */
    uint8_t* truncated;   /* [n]                                           */
    double* exit_pos;     /* [3][n]                                        */
    double* exit_dir;     /* [3][n]                                        */
    double* exit_param;   /* [3][n] cos(theta), alpha, beta                */
    double* event_pos;    /* [3][n] X in the psi = 0 frame, units of r     */
    double* event_dir;    /* [3][n] W in the psi = 0 frame                 */
} or_walk_out;

int or_random_walk(const or_walk_desc* d, const or_walk_out* o);

/* ---------------- CVAE (cvae.c) ---------------- */
/* Widest layer (hidden units, network inputs or outputs) of any shape. */
#define OR_MAX_WIDTH 32

typedef struct {
    int32_t model;   /* 0 LengthGen, 1 PathGen, 2 EventGen */
    int32_t p_in, p_out, latent, width, n_linear;
} or_cvae_shape;

enum { OR_PREC_FP64 = 0, OR_PREC_BF16 = 1, OR_PREC_FP8 = 2 };

double or_softplus(double x);
double or_round_bf16(double x);
double or_round_fp8_e4m3(double x);

/* Parameters of a shape: 2 n_linear layers of S x S weights and S biases,
 * S = 16 if every network width is at most 16, else 32 (see cvae.c). */
int64_t or_cvae_param_count(const or_cvae_shape* s);
void or_cvae_init(const or_cvae_shape* s, uint64_t seed, double* params);

/* Mean KL + NLL over the batch; grad (may be NULL) receives the gradient of
 * NLL + kl_weight * KL with respect to the parameters. */
double or_cvae_loss_grad(const or_cvae_shape* s, const double* params, int32_t batch,
                         const double* cond, const double* target, uint64_t seed, int64_t step,
                         uint64_t id_offset, double kl_weight, double* grad, double* kl_out,
                         double* nll_out);

void or_adamw_step(int32_t n, double* params, double* m, double* v, const double* grad,
                   double lr, double beta1, double beta2, double eps, double weight_decay,
                   int64_t step);

/* Decoder-only sampling, de-standardised outputs.
 * stats = [mean_c(16), std_c(16), mean_y(16), std_y(16)].
 * precision: OR_PREC_FP64 or OR_PREC_BF16 (weights and layer inputs rounded
 * to bfloat16, the rest in double). */
void or_cvae_sample(const or_cvae_shape* s, const double* params, const double* stats,
                    int32_t precision, const double* act_scales, const double* cond, int64_t n,
                    uint64_t seed, uint64_t id_offset, double* out);

/* Decoder-only evaluation with explicit standardised z, eps. */
/* FP8 activation scales of decoder layers 0 .. n_linear - 1 (powers of two)
 * from n raw calibration conditions (see cvae.c). */
void or_cvae_act_scales(const or_cvae_shape* s, const double* params, const double* stats,
                        const double* cond, int64_t n, double* scales);
void or_cvae_decode(const or_cvae_shape* s, const double* params, int32_t precision,
                    const double* act_scales, const double* z, const double* cond_std,
                    double* mu, double* logvar);

/* Raw (unstandardised) features of walk tuples for one model. */
void or_cvae_features(int32_t model, int64_t n, const double* params3, const uint32_t* n_scatter,
                      const double* exit_param, const double* event_pos, const double* event_dir,
                      uint64_t seed, uint64_t id_offset, double* cond, double* target);

/* ---------------- geometry and rendering (render.c) ---------------- */
enum { OR_PRIM_SPHERE = 0, OR_PRIM_BOX = 1 };

typedef struct {
    const float* prims; /* n_prims x 8: type, cx, cy, cz, a, b, c, unused */
    int32_t n_prims;
    const uint16_t* sdf_fp16; /* optional conservative grid, res^3, x fastest */
    int32_t res;
    float lo[3], hi[3];
    /* Optional closed triangle mesh (n_tris x 9 floats: three vertices, any
     * winding); when n_tris > 0 the body is the mesh interior and prims are
     * ignored. */
    const float* tris;
    int32_t n_tris;
} or_scene;

typedef struct {
    double eye[3], look_at[3], up[3];
    double vfov_deg;
    int32_t width, height;
} or_camera;

typedef struct {
    double pos[3];
    double intensity;
} or_light;

typedef struct {
    double sigma_t, g, albedo;
} or_medium;

enum { OR_METHOD_PLAIN_NEE = 1, OR_METHOD_ST = 2 };
enum { OR_SAMPLER_CVAE = 0, OR_SAMPLER_EXACT_WALK = 1 };

typedef struct {
    int32_t method, sampler, precision;
    or_cvae_shape shapes[3];  /* LengthGen, PathGen, EventGen */
    const double* params[3]; /* master weights, one per model */
    const double* stats[3];  /* feature standardisation per model */
    const double* act_scales[3];
    double tau_min, st_max;
    int32_t spp;
    uint64_t seed, sample_offset;
    uint32_t max_events;
    const int32_t* pixels; /* optional subset of pixel indices */
    int64_t n_pixels;      /* number of entries in pixels (or 0 = all) */
    int32_t n_threads;
    int32_t nee_samples;   /* representative events per CVAE step (0 = 1), at most 16 */
    int32_t flags;         /* OR_NEE_BEFORE_ABSORPTION */
    int32_t nee_chain;     /* > 0: a step of N events takes min(nee_samples,
                            * 1 + floor((N - 1) / nee_chain)) representative
                            * events; 0: nee_samples for every step */
} or_render_desc;

/* CVAE steps estimate their direct light before the absorption test, with
 * weight sum_{i<=N} albedo^i, for every step (default: survivors only, with
 * that sum divided by albedo^N).  OR_STEP_PAPER: the learned step as the
 * paper prints it -- PathGen for every lit step (also N = 1) and EventGen
 * for every representative event (no exact first event). */
enum { OR_NEE_BEFORE_ABSORPTION = 1, OR_STEP_PAPER = 2 };

#define OR_MAX_NEE 16

/* Outcome of one sphere step (world frame). */
typedef struct {
    double x[3], w[3];        /* exit position and direction */
    double X[OR_MAX_NEE][3];  /* representative events */
    double W[OR_MAX_NEE][3];
    int first[OR_MAX_NEE];    /* 1 where the event is the exact first one */
    int n_rep;                /* events whose direct light is added */
    double nee_w;             /* weight of each of them */
    double N;
    int survived;
    double psi;               /* azimuth of the exit about w_in */
} or_step_result;

uint32_t or_sphere_step(const or_render_desc* rd, const or_medium* md, uint64_t id, uint32_t c0,
                        const double p[3], const double d[3], double r, or_step_result* out);

typedef struct {
    double* sum;     /* per listed pixel */
    double* sumsq;
    double* events;  /* plain scattering events, summed over samples */
    double* steps;   /* CVAE (or exact-walk) sphere steps, summed */
} or_image_out;

double or_scene_sdf(const or_scene* sc, const double p[3]);
int or_ray_intervals(const or_scene* sc, const double o[3], const double d[3], double* t0,
                     double* t1, int cap);
double or_conservative_radius(const or_scene* sc, const double p[3]);
void or_build_sdf_grid(const or_scene* sc, int32_t res, const float lo[3], const float hi[3],
                       uint16_t* out);
int or_render(const or_scene* sc, const or_camera* cam, const or_light* light,
              const or_medium* med, const or_render_desc* rd, const or_image_out* img);

#ifdef __cplusplus
}
#endif
#endif
