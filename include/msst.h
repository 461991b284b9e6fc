/*
 * msst.h -- C ABI of libmsst, an MI355X (gfx950) implementation of learned
 * sphere tracing for volumetric subsurface scattering
 * (L. Leonard, K. Hoehlein, R. Westermann, arXiv 2011.03082).
 *
 * Conventions shared by every call
 *  - Every call returns an ms_status: MS_OK (0) or a negative error code.
 *    ms_last_error() returns a thread-local description of the last error.
 *  - Arguments are validated completely on the host before any device work
 *    is queued; on error nothing is launched and no output is written.
 *  - Pointers named *_dev, and every array pointer inside the descriptor
 *    structs, are device pointers (HIP device memory, 16-byte aligned,
 *    contiguous).  Descriptor structs themselves live in host memory and are
 *    read only during the call.
 *  - Work is queued asynchronously on the caller's stream (a hipStream_t
 *    passed as void*, NULL = the default stream).  The caller owns every
 *    buffer and keeps it alive until the stream work has finished; the
 *    library keeps no pointer after returning and allocates no device memory:
 *    scratch space comes from a caller-provided workspace whose size the
 *    matching *_workspace_size call reports.
 *  - Arrays of 3-vectors are planar: component c of element i sits at
 *    [c * n + i].
 *  - Randomness is Philox4x32-10 (Salmon et al., SC'11), counter =
 *    (draw index, id low word, id high word, stream tag), key = seed; so any
 *    split of an id range over calls or devices gives identical results.
 *  - Numerical events at run time do not change the status: truncated
 *    walks and paths are counted in the optional counters, and non-finite
 *    inputs or weights propagate to the outputs (cvae_train_step's loss and
 *    gradient, an image's sums and with them ms_image_stats's mean), where
 *    the caller tests for them.
 */
#ifndef MSST_H
#define MSST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MS_ABI_VERSION 1

typedef int32_t ms_status;
enum {
    MS_OK = 0,
    MS_ERR_INVALID_ARGUMENT = -1,
    MS_ERR_DEVICE = -2,
    MS_ERR_UNSUPPORTED = -3,
    MS_ERR_WORKSPACE_TOO_SMALL = -4
};

/* Philox stream tags (counter word 3). */
enum {
    MS_TAG_WALK_EVENT = 0,
    MS_TAG_WALK_PARAM = 1,
    MS_TAG_CVAE_INIT = 2,
    MS_TAG_CVAE_BATCH = 3,
    MS_TAG_CVAE_REPARAM = 4,
    MS_TAG_CVAE_SAMPLE = 5,
    MS_TAG_RENDER_PIXEL = 6,
    MS_TAG_RENDER_PATH = 7,
    MS_TAG_SCENE = 8,
    MS_TAG_DEQUANT = 9
};

int32_t ms_abi_version(void);
const char* ms_last_error(void);

/* ------------------------------------------------------------------------
 * Randomness.  The paper draws uniform xi for flights and phase sampling
 * (Sec. 3.1) and Gaussian z, epsilon for the CVAEs (Sec. 3.2, Sec. 4.2).
 *
 * ms_philox_fill: out_dev[(i * n_draws + j) * 4 + w] = word w of the Philox
 * block of counter (c0 + j, id0 + i, tag) under key seed, for i < n_ids,
 * j < n_draws.  n_ids * n_draws must be positive and below 2^31.
 */
ms_status ms_philox_fill(uint64_t seed, uint32_t tag, uint64_t id0, int64_t n_ids, uint32_t c0,
                         int32_t n_draws, uint32_t* out_dev, void* stream);

/* ------------------------------------------------------------------------
 * Random walk in a homogeneous sphere (Sec. 3.1; method overview figure of
 * Sec. 3).  A photon starts at the centre heading along +z; the first
 * scattering event is at the centre; free flights l = -log(1 - xi)/sigma_t;
 * Henyey-Greenstein scattering (Eq. 1); the walk ends at the first crossing
 * of the sphere.
 *  ANALOG:   fixed (sigma_t, g, albedo, radius); absorption at each event
 *            with probability 1 - albedo (the Russian roulette of Sec. 3.1).
 *  TRAINING: per photon sigma_t*r log-uniform in st_range, g and albedo
 *            uniform in their ranges, r = 1, no absorption (the learned
 *            models take absorption separately, Sec. 3.2); a representative
 *            event k is kept with probability albedo^k / sum_i albedo^i
 *            (ALBEDO_POWER, Sec. 4.3) or 1/N (UNIFORM).  Outputs use the
 *            exit parameterisation of Sec. 4.1: cos(theta), alpha, beta and
 *            (X, W) rotated into the frame where psi = 0.
 * Photon i uses Philox id photon_offset + i.  Invalid: n_photons == 0 or
 * >= 2^40, sigma_t <= 0, |g| >= 1, albedo outside [0, 1], radius <= 0
 * (ANALOG); empty or inverted ranges, st_range[0] <= 0 (TRAINING).
 */
enum { MS_WALK_ANALOG = 0, MS_WALK_TRAINING = 1 };
enum { MS_EVENT_ALBEDO_POWER = 0, MS_EVENT_UNIFORM = 1 };

typedef struct {
    uint64_t seed, photon_offset, n_photons;
    int32_t mode, event_weighting;
    double sigma_t, g, albedo, radius;                 /* ANALOG */
    double st_range[2], g_range[2], albedo_range[2];   /* TRAINING */
    uint32_t max_events;                               /* 0 = 2^20 */
    int32_t blocks_per_cu;                             /* 256-thread blocks per CU, 1..64; 0 = 2 */
    /* TRAINING: (sigma_t r, g)-weighted data (Sec. 5.3 names over-weighting
     * parameter regions as a lever for quality).  With probability
     * focus_fraction (decided by the fourth uniform of the photon's parameter
     * block) sigma_t r and g are drawn from the focus ranges instead, with
     * the same uniforms; 0 disables it. */
    double focus_fraction;
    double focus_st_range[2], focus_g_range[2];
} ms_walk_desc;

/* Any pointer may be NULL.  Planar [3][n] for the 3-vectors. */
typedef struct {
    float* params;         /* [3][n] sigma_t * r, g, albedo */
    uint32_t* n_scatter;   /* [n] N, events including the centre one */
    uint32_t* event_index; /* [n] representative event k (TRAINING) */
    uint8_t* absorbed;     /* [n] (ANALOG) */
    uint8_t* truncated;    /* [n] max_events reached */
    float* exit_pos;       /* [3][n] exit (or absorption) position */
    float* exit_dir;       /* [3][n] direction there */
    float* exit_param;     /* [3][n] cos(theta), alpha, beta */
    float* event_pos;      /* [3][n] X / r in the psi = 0 frame (TRAINING) */
    float* event_dir;      /* [3][n] W in the psi = 0 frame (TRAINING) */
    uint64_t* counters;    /* [4] += total events, absorbed, truncated, max N */
} ms_walk_out;

ms_status ms_random_walk_workspace_size(const ms_walk_desc* desc, size_t* bytes);
ms_status ms_random_walk(const ms_walk_desc* desc, const ms_walk_out* out, void* workspace_dev,
                         size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Conditional VAEs (Sec. 3.2, Fig. 3b; model signatures of Sec. 4.2).
 * Encoder and decoder are MLPs of n_linear linear maps (n_linear - 1 hidden
 * layers of `width` units) with Softplus between hidden layers and linear
 * (mean, log variance) outputs.
 *   LengthGen  cond (log sigma_t r, g)                                -> log N
 *   PathGen    cond (log sigma_t r, g, log N)                         -> (cos theta, alpha, beta)
 *   EventGen   cond (log sigma_t r, g, albedo, cos theta, alpha, beta, log N) -> (X, W)
 * Limits: 2 <= n_linear <= 4 (Table 1's depths D = 1..3), width <= 32,
 * p_in <= 16, p_out + p_in <= 32, latent + p_in <= 32, 2 * p_out <= 32,
 * 2 * latent <= 32 (all of Table 1's settings).
 *
 * Master parameter layout (FP32, cvae_param_count floats): 2 * n_linear
 * layers, encoder first; each layer = S x S row-major weights (row = output
 * unit) then S biases, S = 16 when width, p_out + p_in, latent + p_in,
 * 2 p_out and 2 latent are all <= 16 (one MFMA tile per layer) and S = 32
 * otherwise (a 2 x 2 grid of tiles); unused rows and columns are zero and
 * stay zero.  Encoder input is (target, cond); decoder input is (z, cond);
 * output rows are (mean[0..k), log variance[0..k)); log variances are
 * clamped to [-12, 8].
 */
enum { MS_MODEL_LENGTH = 0, MS_MODEL_PATH = 1, MS_MODEL_EVENT = 2 };
enum { MS_PREC_BF16 = 1, MS_PREC_FP8 = 2 };

typedef struct {
    int32_t model, p_in, p_out, latent, width, n_linear;
} ms_cvae_shape;

typedef struct {
    double lr, beta1, beta2, eps, weight_decay;
    int64_t step; /* 1-based AdamW step number */
} ms_adam;

ms_status cvae_param_count(const ms_cvae_shape* shape, size_t* n_floats);

/* Deterministic initialisation: each real weight and bias is
 * (2u - 1) / sqrt(fan_in), u from tag CVAE_INIT, id = model,
 * c0 = flat index / 4, word = flat index % 4. */
ms_status cvae_init(const ms_cvae_shape* shape, uint64_t seed, float* master_dev, void* stream);

/* Condition / target rows of one model from TRAINING walk outputs, row-major
 * [n][p_in] and [n][p_out].  Output row i is built from walk record
 * rows_dev[i] (or record i when rows_dev is NULL); n_records is the length of
 * the walk arrays.  LengthGen's target is log(N + u - 1/2), u from tag
 * DEQUANT (id = id_offset + record, c0 = 0, word 0).  If stats_dev is not
 * NULL ([64] doubles: mean_c[16], std_c[16], mean_y[16], std_y[16]) the rows
 * are standardised. */
ms_status cvae_features(int32_t model, int64_t n, const int64_t* rows_dev, int64_t n_records,
                        const float* params3_dev, const uint32_t* n_scatter_dev,
                        const float* exit_param_dev, const float* event_pos_dev,
                        const float* event_dir_dev, uint64_t seed, uint64_t id_offset,
                        const double* stats_dev, float* cond_dev, float* target_dev, void* stream);

/* Deterministic stream compaction of walk records: rows_dev receives, in
 * increasing order, the indices i < n with n_scatter[i] >= min_scatter and
 * (event_index_dev NULL or event_index[i] >= min_event); *count_dev (device)
 * their number.  Used to train PathGen on N >= 2 and EventGen on k >= 2
 * records, whose single-event cases the renderer samples exactly. */
ms_status ms_select_rows_workspace_size(int64_t n, size_t* bytes);
ms_status ms_select_rows(int64_t n, const uint32_t* n_scatter_dev, const uint32_t* event_index_dev,
                         uint32_t min_scatter, uint32_t min_event, int64_t* rows_dev,
                         int64_t* count_dev, void* workspace_dev, size_t workspace_bytes,
                         void* stream);

/* FP64 column mean and standard deviation of a row-major [n][dim] matrix,
 * written to out_dev[0..dim) and out_dev[16..16+dim) (dim <= 16), by a
 * deterministic two-pass reduction. */
ms_status ms_column_moments_workspace_size(int64_t n, int32_t dim, size_t* bytes);
ms_status ms_column_moments(const float* x_dev, int64_t n, int32_t dim, double* out_dev,
                            void* workspace_dev, size_t workspace_bytes, void* stream);

/* One AdamW step of one CVAE on one minibatch (ELBO of Sec. 3.2: KL to
 * N(0, I) plus the Gaussian NLL, one reparameterised sample).  Forward and
 * backward run on bfloat16 MFMA with FP32 accumulation; the master weights
 * and the AdamW moments stay FP32.
 *  rows: sample_rows == 0 takes rows [0, batch) of cond/target; otherwise
 *        row of sample b = (w * n_rows) >> 32 with w word 0 of tag
 *        CVAE_BATCH (id = b, c0 = step): uniform with replacement.
 *  noise: eps of sample b from tag CVAE_REPARAM, id = id_offset + b,
 *        c0 = 4 * step + j.
 *  kl_weight: weight of the KL term in the gradient (1 = the ELBO; a
 *        warm-up from 0 is the usual guard against an unused latent).
 *  adam == NULL computes the gradient without updating.
 *  loss_dev (nullable, [3] doubles): batch-mean KL + NLL, KL, NLL (unweighted).
 *  grad_dev (nullable, cvae_param_count floats): batch-mean gradient.
 * batch must be a positive multiple of 16, at most 2^20. */
ms_status cvae_workspace_size(const ms_cvae_shape* shape, int32_t batch, size_t* bytes);
ms_status cvae_train_step(const ms_cvae_shape* shape, float* master_dev, float* adam_m_dev,
                          float* adam_v_dev, const ms_adam* adam, const float* cond_dev,
                          const float* target_dev, int64_t n_rows, int32_t batch,
                          int32_t sample_rows, uint64_t seed, int64_t step, uint64_t id_offset,
                          double kl_weight, void* workspace_dev, size_t workspace_bytes,
                          double* loss_dev, float* grad_dev, void* stream);

/* cvae_train_step without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * cvae_train_step; the per-block partials live in a static device array of
 * the library (about 8.7 MB per device, held until the process ends, sized
 * for the largest batch (2^20) and network (n_linear 4) accepted; a
 * larger batch fails with MS_ERR_INVALID_ARGUMENT and a larger network with
 * MS_ERR_UNSUPPORTED before anything is launched).
 * Nothing is allocated: the array's device address is looked up once per
 * device on the first call with that device current.  Calls on one device
 * share the array, so calls that overlap in time on one device (several
 * streams, several threads) race; serialise them on one stream. */
ms_status cvae_train_step_noalloc(const ms_cvae_shape* shape, float* master_dev, float* adam_m_dev,
                                  float* adam_v_dev, const ms_adam* adam, const float* cond_dev,
                                  const float* target_dev, int64_t n_rows, int32_t batch,
                                  int32_t sample_rows, uint64_t seed, int64_t step,
                                  uint64_t id_offset, double kl_weight, double* loss_dev,
                                  float* grad_dev, void* stream);

/* Inference copy of one model's decoder (Sec. 3.2: the encoder is dropped;
 * the paper's shader re-implements the decoders in reduced precision):
 * bfloat16 weights, or FP8 E4M3 weights with a per-layer weight scale
 * s_w = max|W| / 448 and a per-layer activation scale s_a (FP32
 * accumulation either way), plus the standardisation constants (stats_dev
 * as for cvae_features).  FP8 layer j computes
 * s_w s_a * (E4M3(W / s_w) . E4M3(a / s_a)) + b.  s_a comes from
 * calibration: calib_cond_dev holds n_calib raw conditions [n_calib][p_in];
 * for each decoder layer, s_a is the smallest power of two with
 * max|a| / s_a <= 448 over those rows, a being the layer's FP32 input from
 * the master weights with latent z the first L normals of cvae_sample's
 * stream for seed 0, id = row.  n_calib = 0 (or BF16) gives s_a = 1.
 * n_calib <= 2^20; stats_dev is required with calibration rows. */
size_t cvae_packed_bytes(void);
ms_status cvae_pack(const ms_cvae_shape* shape, const float* master_dev, const double* stats_dev,
                    int32_t precision, const float* calib_cond_dev, int64_t n_calib,
                    void* packed_dev, size_t packed_bytes, void* stream);

/* Decoder-only sampling (Sec. 3.2 inference): z ~ N(0, I), then
 * y = mu_Dec(z, c) + exp(logvar / 2) eps, de-standardised.  Path i draws its
 * L + p_out normals from tag CVAE_SAMPLE, id = id_offset + i, blocks
 * c0 = 0, 1, ... (Box-Muller on word pairs), z first.  cond_dev is raw
 * [n][p_in], out_dev raw [n][p_out]. */
ms_status cvae_sample(const void* packed_dev, const float* cond_dev, int64_t n, uint64_t seed,
                      uint64_t id_offset, float* out_dev, void* stream);

/* ------------------------------------------------------------------------
 * Rendering (Sec. 3, Fig. 2; Sec. 4.1 radius rescale; Sec. 4.3 direct light).
 * A pinhole camera traces paths into a homogeneous medium bounded by the
 * union of primitives (no refraction, black background) lit by one point
 * light.  PLAIN_NEE: plain path tracing with next-event estimation at
 * every scattering event.  ST: at a collision, r = min(conservative
 * distance, st_max / sigma_t); if sigma_t r >= tau_min one learned sphere
 * step (LengthGen, absorption with probability 1 - albedo^N, PathGen,
 * EventGen, NEE at the representative event with weight
 * sum_{i<=N} albedo^i / albedo^N), else a plain event.  The single-event
 * parts of the step are sampled exactly: N = 1 is one HG scatter at the
 * centre (no PathGen), and for N >= 2 the representative event is the
 * centre with probability albedo / sum_{i<=N} albedo^i (no EventGen);
 * PathGen and EventGen are trained on the remaining records (see
 * ms_select_rows).  sampler EXACT_WALK replaces the learned step by the
 * actual walk inside the sphere.
 * Path (pixel, s) uses Philox id pixel | (sample_offset + s) << 32.
 * Results are ADDED to the caller-zeroed image buffers, so renders can be
 * resumed with sample_offset.  Primitive record: 8 floats
 * (type, cx, cy, cz, a, b, c, 0): sphere radius a, box half sizes a, b, c.
 */
enum { MS_PRIM_SPHERE = 0, MS_PRIM_BOX = 1 };
enum { MS_METHOD_PLAIN_NEE = 1, MS_METHOD_ST = 2 };
enum { MS_SAMPLER_CVAE = 0, MS_SAMPLER_EXACT_WALK = 1 };

typedef struct {
    const float* prims;       /* device [n_prims][8] */
    int32_t n_prims;          /* 1..256 (up to 4 are held in registers); 0 with a mesh */
    const uint16_t* sdf_fp16; /* optional device grid [res^3], x fastest (required with a mesh) */
    int32_t res;
    float lo[3], hi[3];
    /* Optional closed triangle mesh (the polygon-mesh boundary the paper
     * renders): when n_tris > 0 the body is the mesh interior and prims are
     * ignored.  tris: device [n_tris][9] vertex triples in the order
     * ms_build_mesh_bvh returns, bvh: its device node array.  Camera rays
     * start outside the body and every other ray inside it (at a collision
     * or a sphere-step exit), so the crossings ahead of a ray's origin
     * alternate entry / exit (resp. exit / entry); up to 8 are kept, the
     * nearest first. */
    const float* tris;
    int32_t n_tris;
    const void* bvh;
    int32_t n_nodes;
} ms_scene;

/* Bounding-volume hierarchy of a closed triangle mesh, built on the host:
 * binned surface-area-heuristic splits (median splits where the bins cannot
 * separate the triangles), leaves of up to 4 triangles,
 * 32-byte nodes in depth-first order with skip links (stackless traversal).
 * tris_host: [n_tris][9] floats; writes the nodes (at most 2 n_tris, size
 * from ms_mesh_bvh_size) and the triangles reordered to the leaves' order
 * (tris_sorted_host, [n_tris][9]); the caller copies both to the device.
 * Host memory only; nothing is launched. */
ms_status ms_mesh_bvh_size(int32_t n_tris, size_t* node_bytes);
ms_status ms_build_mesh_bvh(const float* tris_host, int32_t n_tris, void* nodes_host, size_t node_bytes,
                            float* tris_sorted_host, int32_t* n_nodes);

typedef struct {
    float eye[3], look_at[3], up[3];
    float vfov_deg;
    int32_t width, height;
} ms_camera;

typedef struct {
    float pos[3];
    float intensity;
} ms_light;

typedef struct {
    float sigma_t, g, albedo;
} ms_medium;

typedef struct {
    int32_t method, sampler;
    const void* packed[3];   /* LengthGen, PathGen, EventGen (ST with CVAE); one-tile
                              * models (S = 16, latent <= 8); other models leave the
                              * image's sum NaN and trace nothing */
    /* learned steps where sigma_t r >= tau_min (> 0); r capped at st_max / sigma_t.
     * The decoders are trained on sigma_t r in [0.1, 200] (the training walk's
     * st_range): tau_min below 0.1 or st_max above 200 asks them to extrapolate. */
    float tau_min, st_max;
    int32_t spp;
    int32_t chunk;           /* samples per work unit; 0 = min(64, ceil(pixels spp / 2^23)), or
                              * ceil(pixels spp / 2^24) where that leaves more than 2^24 units,
                              * at least 2 and at most spp; at most 2^32 units */
    uint64_t seed, sample_offset;
    uint32_t max_events;     /* collisions per path (plain events plus sphere
                              * steps, a step counting once); a path ends at
                              * the next collision, keeping the light gathered
                              * so far, and is counted as truncated; 0 = 2^20 */
    int32_t blocks_per_cu;   /* 256-thread blocks per CU, 1..64; 0 = 4 */
    int32_t cvae_batch_min;  /* waiting lanes that trigger a decoder pass, 1..64; 0 = 20 */
    int32_t restart_min;     /* lanes waiting for a new path that trigger a restart pass, 1..64; 0 = 16 */
    int32_t max_wait;        /* loop iterations after which waiting lanes force a pass anyway; 0 = 10 */
    int32_t nee_samples;     /* representative events per learned step, 1..16 (0 = 1) */
    int32_t flags;           /* MS_RENDER_NEE_BEFORE_ABSORPTION | MS_RENDER_STEP_PAPER */
    /* Cost rule for a launch (0 = off): learned steps are taken only if the
     * deepest sphere the scene allows, of optical radius T = sigma_t *
     * min(deepest interior distance, st_max / sigma_t), holds a chain of
     * about T^2 (1 - g) / 2 collisions (the diffusion estimate of E[N]) of at
     * least min_chain; otherwise the launch traces plainly (the same paths as
     * PLAIN_NEE).  Scenes whose deepest distance is not known in closed form
     * (a distance grid, many primitives, a mesh) always allow steps. */
    float min_chain;
    /* Representative events per learned step by chain length (0 = off:
     * nee_samples for every step).  A step's direct-light estimate weights
     * one event by sum_{i<=N} albedo^i, so its variance grows with the square
     * of that sum; with nee_chain > 0 a step of N events draws
     * K = min(nee_samples, 1 + floor((N - 1) / nee_chain)) events, each
     * weighted by 1/K of it: more events where the chain is long, one where
     * it is short.  K depends on N only (drawn before the events), so the
     * estimate stays unbiased.  At most 2^24. */
    int32_t nee_chain;
} ms_render_desc;

/* MS_RENDER_NEE_BEFORE_ABSORPTION: direct light of a learned step estimated
 * before its absorption test, with weight sum_{i<=N} albedo^i, for every
 * step (the paper's order rejects first and weights survivors by that sum /
 * albedo^N); both are unbiased for sum_i albedo^i f_i.  K = nee_samples
 * representative events average K independent EventGen samples (each its
 * own first-event test).
 * MS_RENDER_STEP_PAPER: the learned step as the paper prints it (Sec. 3.2,
 * Sec. 4.2, Sec. 4.3): PathGen for every lit step, also N = 1, and EventGen
 * for every representative event, also the first one; the models are then
 * meant to be trained on every walk record.  The same Philox blocks are
 * drawn as without the flag (the HG and first-event uniforms go unused). */
enum { MS_RENDER_NEE_BEFORE_ABSORPTION = 1, MS_RENDER_STEP_PAPER = 2 };

typedef struct {
    float* sum;          /* [width * height] sum of path radiance */
    float* comp;         /* [width * height] compensation term of sum */
    float* sumsq;        /* [width * height] sum of squares */
    uint32_t* events;    /* [width * height] plain scattering events */
    uint32_t* steps;     /* [width * height] sphere steps */
    uint64_t* counters;  /* optional [4] += paths, events, steps, truncated */
} ms_image_out;

ms_status sphere_trace_render_workspace_size(const ms_camera* cam, const ms_render_desc* desc,
                                             size_t* bytes);
ms_status sphere_trace_render(const ms_scene* scene, const ms_camera* cam, const ms_light* light,
                              const ms_medium* medium, const ms_render_desc* desc,
                              const ms_image_out* out, void* workspace_dev, size_t workspace_bytes,
                              void* stream);

/* Conservative distance grid of a scene (the voxel-grid distance pre-process
 * of Sec. 3, with a Euclidean lower bound in place of the Chebyshev
 * distance): grid_dev[(k * res + j) * res + i] = binary16 bits of
 * min_prims sdf(lo + (i + 1/2, j + 1/2, k + 1/2) h), evaluated in FP64 and
 * rounded toward zero, h = (hi - lo) / res, over scene->lo .. scene->hi
 * (scene->sdf_fp16 and scene->res are ignored).  Passing the grid back in
 * ms_scene makes the renderer take sphere radii from the nearest voxel
 * minus half a voxel diagonal.  1..256 primitives, res <= 4096.  For a mesh
 * scene (n_tris > 0, tris on the device) the distance is the FP64 distance
 * to the nearest triangle, negative where a ray from the voxel centre along
 * (1, 2, 3) / sqrt(14) crosses the mesh an odd number of times (every
 * triangle is tested: a pre-process, not a per-frame cost). */
ms_status ms_build_sdf_grid(const ms_scene* scene, int32_t res, uint16_t* grid_dev, void* stream);

/* FP64 image statistics (deterministic): out_dev[0] mean radiance,
 * [1] RMSE against ref_dev (per-pixel means), [2] mean per-pixel variance
 * of one sample, [3] mean of ref.  Images are per-pixel sums over spp
 * samples (sum + comp); ref_dev holds per-pixel means (nullable). */
ms_status ms_image_stats_workspace_size(int64_t n_pixels, size_t* bytes);
ms_status ms_image_stats(const float* sum_dev, const float* comp_dev, const float* sumsq_dev,
                         const float* ref_dev, int64_t n_pixels, int32_t spp, double* out_dev,
                         void* workspace_dev, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif
