/*
 * oracle_sanitize.c -- drives every entry point of the FP64 oracle on small
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitizers.py).  Exits 0 when every call returns and
 * every output is finite; the sanitizers abort on any invalid access,
 * leak, overflow or undefined operation on the way.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "msst_oracle.h"

static int bad = 0;

static void check_finite(const char* what, const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) {
            fprintf(stderr, "%s[%zu] is not finite\n", what, i);
            bad = 1;
            return;
        }
}

static void* zalloc(size_t bytes) {
    void* p = calloc(1, bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

static void walks(void) {
    for (int mode = 0; mode < 2; ++mode) {
        const uint64_t n = 2000;
        or_walk_desc d;
        memset(&d, 0, sizeof d);
        d.seed = 3;
        d.n_photons = n;
        d.mode = mode;
        d.sigma_t = 10.0;
        d.g = 0.8;
        d.albedo = 0.99;
        d.radius = 1.0;
        d.st_range[0] = 0.1, d.st_range[1] = 200.0;
        d.g_range[0] = -0.9, d.g_range[1] = 0.95;
        d.albedo_range[0] = 0.9, d.albedo_range[1] = 1.0;
        d.max_events = 1u << 20;
        d.n_threads = 4;
        d.focus_fraction = mode ? 0.5 : 0.0;
        d.focus_st_range[0] = 10.0, d.focus_st_range[1] = 200.0;
        d.focus_g_range[0] = 0.7, d.focus_g_range[1] = 0.9;
        or_walk_out o;
        memset(&o, 0, sizeof o);
        o.params = zalloc(3 * n * sizeof(double));
        o.n_scatter = zalloc(n * sizeof(uint32_t));
        o.event_index = zalloc(n * sizeof(uint32_t));
        o.absorbed = zalloc(n);
        o.truncated = zalloc(n);
        o.exit_pos = zalloc(3 * n * sizeof(double));
        o.exit_dir = zalloc(3 * n * sizeof(double));
        o.exit_param = zalloc(3 * n * sizeof(double));
        o.event_pos = zalloc(3 * n * sizeof(double));
        o.event_dir = zalloc(3 * n * sizeof(double));
        if (or_random_walk(&d, &o) != 0) bad = 1;
        check_finite("walk exit_pos", o.exit_pos, 3 * n);
        if (mode == OR_WALK_TRAINING) {
            /* the walk's records as CVAE features of each model */
            for (int m = 0; m < 3; ++m) {
                const int pin[3] = {2, 3, 7}, pout[3] = {1, 3, 6};
                double* cond = zalloc(n * pin[m] * sizeof(double));
                double* target = zalloc(n * pout[m] * sizeof(double));
                or_cvae_features(m, (int64_t)n, o.params, o.n_scatter, o.exit_param, o.event_pos, o.event_dir, 5,
                                 0, cond, target);
                check_finite("features", cond, n * pin[m]);
                free(cond);
                free(target);
            }
        }
        free(o.params), free(o.n_scatter), free(o.event_index), free(o.absorbed), free(o.truncated);
        free(o.exit_pos), free(o.exit_dir), free(o.exit_param), free(o.event_pos), free(o.event_dir);
    }
}

static void fill_stats(int p_in, int p_out, double* stats) {
    memset(stats, 0, 64 * sizeof(double));
    for (int k = 0; k < 16; ++k) {
        stats[k] = 0.1 * k;
        stats[16 + k] = 1.0 + 0.05 * k;
        stats[32 + k] = -0.1 * k;
        stats[48 + k] = 0.5 + 0.1 * k;
    }
    (void)p_in;
    (void)p_out;
}

static void cvae(const or_cvae_shape* s) {
    const int64_t np = or_cvae_param_count(s);
    double* p = zalloc((size_t)np * sizeof(double));
    double* g = zalloc((size_t)np * sizeof(double));
    double* m = zalloc((size_t)np * sizeof(double));
    double* v = zalloc((size_t)np * sizeof(double));
    or_cvae_init(s, 11, p);
    const int B = 8;
    double cond[8 * 16], target[8 * 16];
    for (int i = 0; i < B * 16; ++i) {
        cond[i] = sin(0.37 * i);
        target[i] = cos(0.21 * i);
    }
    double kl = 0, nll = 0;
    double loss = or_cvae_loss_grad(s, p, B, cond, target, 9, 2, 0, 0.5, g, &kl, &nll);
    check_finite("loss", &loss, 1);
    check_finite("grad", g, (size_t)np);
    or_adamw_step((int32_t)np, p, m, v, g, 1e-3, 0.9, 0.999, 1e-8, 0.01, 1);
    double stats[64];
    fill_stats(s->p_in, s->p_out, stats);
    double scales[8];
    or_cvae_act_scales(s, p, stats, cond, B, scales);
    check_finite("act scales", scales, (size_t)s->n_linear);
    double out[8 * 16];
    for (int prec = 0; prec < 3; ++prec) {
        or_cvae_sample(s, p, stats, prec, prec == OR_PREC_FP8 ? scales : NULL, cond, B, 4, 0, out);
        check_finite("sample", out, (size_t)(B * s->p_out));
    }
    free(p), free(g), free(m), free(v);
}

static void renders(void) {
    const float prims[16] = {OR_PRIM_SPHERE, 0, 0, 0, 1, 0, 0, 0, OR_PRIM_BOX, 1.2f, 0, 0, 0.8f, 0.4f, 0.4f, 0};
    or_scene sc;
    memset(&sc, 0, sizeof sc);
    sc.prims = prims;
    sc.n_prims = 2;
    const int res = 16;
    uint16_t* grid = zalloc((size_t)res * res * res * sizeof(uint16_t));
    const float lo[3] = {-1.2f, -1.2f, -1.2f}, hi[3] = {2.2f, 1.2f, 1.2f};
    or_build_sdf_grid(&sc, res, lo, hi, grid);
    or_camera cam = {{0.5, 0.3, 4.0}, {0.5, 0.0, 0.0}, {0, 1, 0}, 40.0, 8, 8};
    or_light light = {{2.0, 3.0, 2.0}, 20.0};
    or_medium med = {40.0, 0.8, 0.995};
    const or_cvae_shape shapes[3] = {{0, 2, 1, 4, 16, 3}, {1, 3, 3, 4, 16, 3}, {2, 7, 6, 4, 16, 3}};
    double* params[3];
    double stats[3][64];
    for (int m = 0; m < 3; ++m) {
        params[m] = zalloc((size_t)or_cvae_param_count(&shapes[m]) * sizeof(double));
        or_cvae_init(&shapes[m], 50 + m, params[m]);
        fill_stats(shapes[m].p_in, shapes[m].p_out, stats[m]);
    }
    const int npix = cam.width * cam.height;
    double* sum = zalloc(npix * sizeof(double));
    double* sumsq = zalloc(npix * sizeof(double));
    double* ev = zalloc(npix * sizeof(double));
    double* st = zalloc(npix * sizeof(double));
    or_image_out img = {sum, sumsq, ev, st};
    for (int with_grid = 0; with_grid < 2; ++with_grid) {
        sc.sdf_fp16 = with_grid ? grid : NULL;
        sc.res = with_grid ? res : 0;
        memcpy(sc.lo, lo, sizeof lo);
        memcpy(sc.hi, hi, sizeof hi);
        for (int c = 0; c < 5; ++c) {
            or_render_desc rd;
            memset(&rd, 0, sizeof rd);
            rd.method = c == 0 ? OR_METHOD_PLAIN_NEE : OR_METHOD_ST;
            rd.sampler = c == 1 ? OR_SAMPLER_EXACT_WALK : OR_SAMPLER_CVAE;
            rd.precision = c == 4 ? OR_PREC_BF16 : OR_PREC_FP64;
            for (int m = 0; m < 3; ++m) {
                rd.shapes[m] = shapes[m];
                rd.params[m] = params[m];
                rd.stats[m] = stats[m];
            }
            rd.tau_min = 2.0;
            rd.st_max = 200.0;
            rd.spp = 2;
            rd.seed = 7;
            rd.max_events = 1u << 16;
            rd.n_threads = 2;
            rd.nee_samples = c == 3 ? 3 : 1;
            rd.flags = c == 2 ? OR_NEE_BEFORE_ABSORPTION : (c == 3 ? OR_NEE_BEFORE_ABSORPTION | OR_STEP_PAPER : 0);
            memset(sum, 0, npix * sizeof(double));
            if (or_render(&sc, &cam, &light, &med, &rd, &img) != 0) bad = 1;
            check_finite("render sum", sum, (size_t)npix);
        }
    }
    /* a closed mesh: a tetrahedron */
    const float tris[4 * 9] = {0, 0, 1, 0.94f, 0, -0.33f, -0.47f, 0.82f, -0.33f,
                               0, 0, 1, -0.47f, 0.82f, -0.33f, -0.47f, -0.82f, -0.33f,
                               0, 0, 1, -0.47f, -0.82f, -0.33f, 0.94f, 0, -0.33f,
                               0.94f, 0, -0.33f, -0.47f, -0.82f, -0.33f, -0.47f, 0.82f, -0.33f};
    or_scene ms;
    memset(&ms, 0, sizeof ms);
    ms.tris = tris;
    ms.n_tris = 4;
    const float mlo[3] = {-1.1f, -1.1f, -1.1f}, mhi[3] = {1.1f, 1.1f, 1.1f};
    or_build_sdf_grid(&ms, res, mlo, mhi, grid);
    ms.sdf_fp16 = grid;
    ms.res = res;
    memcpy(ms.lo, mlo, sizeof mlo);
    memcpy(ms.hi, mhi, sizeof mhi);
    or_render_desc rd;
    memset(&rd, 0, sizeof rd);
    rd.method = OR_METHOD_ST;
    rd.sampler = OR_SAMPLER_EXACT_WALK;
    rd.tau_min = 2.0;
    rd.st_max = 200.0;
    rd.spp = 2;
    rd.max_events = 1u << 16;
    rd.n_threads = 1;
    if (or_render(&ms, &cam, &light, &med, &rd, &img) != 0) bad = 1;
    check_finite("mesh render sum", sum, (size_t)npix);
    for (int m = 0; m < 3; ++m) free(params[m]);
    free(grid), free(sum), free(sumsq), free(ev), free(st);
}

int main(void) {
    walks();
    const or_cvae_shape shapes[] = {
        {0, 2, 1, 4, 16, 3}, {1, 3, 3, 4, 16, 3}, {2, 7, 6, 4, 16, 3},  /* the defaults */
        {0, 2, 1, 2, 8, 3},                                             /* LengthGen final */
        {2, 7, 6, 5, 20, 3}, {1, 3, 3, 9, 8, 2}, {2, 7, 6, 9, 20, 4},  /* row stride 32 */
    };
    for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; ++i) cvae(&shapes[i]);
    renders();
    if (bad) return 1;
    printf("oracle sanitizer run ok\n");
    return 0;
}
