/*
 * walk.c -- oracle random walk in a homogeneous sphere.
 * TEST INFRASTRUCTURE ONLY (see msst_oracle.h).
 *
 * Follows the paper's training-data process (Sec. 3.1 and the method
 * overview figure of Sec. 3): a photon starts at the centre of a sphere,
 * heading along w_in = (0, 0, 1); the first scattering event happens at the
 * centre; free flights are l = -log(1 - xi) / sigma_t; at each event the path
 * is absorbed with probability 1 - albedo, otherwise a new direction is drawn
 * from the Henyey-Greenstein phase function (Eq. 1); the walk ends at the
 * first crossing of the sphere.  The exit is parameterised as in Sec. 4.1
 * (cos theta, psi, alpha, beta) and the representative event of Sec. 4.3 is
 * chosen with probability albedo^k / Lambda^(N).
 */
#include "msst_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288
#define OR_U24 16777216.0

/* Henyey-Greenstein phase function, Eq. 1 of Sec. 3.1. */
double or_hg_eval(double g, double cos_theta) {
    double denom = 1.0 + g * g - 2.0 * g * cos_theta;
    return (1.0 / (4.0 * OR_PI)) * (1.0 - g * g) / (denom * sqrt(denom));
}

/* Inverse of the HG cosine CDF
 *   F(mu) = (1 - g^2) / (2 g) * [(1 + g^2 - 2 g mu)^(-1/2) - (1 + g)^(-1)],
 * solved for mu at F = xi.  The paper importance-samples HG (Sec. 3.1) but
 * prints no inversion; this is the textbook one, isotropic when g == 0. */
double or_hg_sample(double g, double xi) {
    if (fabs(g) < 1e-12) return 2.0 * xi - 1.0;
    double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * xi);
    double mu = (1.0 + g * g - s * s) / (2.0 * g);
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* Orthonormal basis (b1, b2, n), right-handed, after Duff, Burgess,
 * Christensen, Hery, Kensler, Liani and Villemin, "Building an Orthonormal
 * Basis, Revisited", JCGT 6(1), 2017.  It fixes the azimuth origin that
 * phase sampling and the CVAE frame rotation use. */
void or_onb(const double n[3], double b1[3], double b2[3]) {
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a;
    b1[1] = sign * b;
    b1[2] = -sign * n[0];
    b2[0] = b;
    b2[1] = sign + n[1] * n[1] * a;
    b2[2] = -n[1];
}

/* New direction at polar cosine mu and azimuth phi around d. */
void or_scatter_dir(double d[3], double mu, double azimuth) {
    double b1[3], b2[3];
    or_onb(d, b1, b2);
    double s = sqrt(fmax(0.0, 1.0 - mu * mu));
    double ca = cos(azimuth), sa = sin(azimuth);
    double nd[3];
    for (int i = 0; i < 3; ++i) nd[i] = mu * d[i] + s * (ca * b1[i] + sa * b2[i]);
    double len = sqrt(nd[0] * nd[0] + nd[1] * nd[1] + nd[2] * nd[2]);
    for (int i = 0; i < 3; ++i) d[i] = nd[i] / len;
}

static void or_put3(double* base, uint64_t n, uint64_t i, const double v[3]) {
    if (!base) return;
    base[i] = v[0];
    base[n + i] = v[1];
    base[2 * n + i] = v[2];
}

/* Exit parameterisation of Sec. 4.1: cos theta = cos(w_in, x); psi the
 * azimuth of x about w_in; e_b = w_in x x_hat (normalised), e_t = e_b x e_n;
 * alpha = w.e_b, beta = w.e_t.  Evaluated after rotating by -psi about z so
 * that x lies in the xz-plane, where e_b = (0, 1, 0) and
 * e_t = (cos theta, 0, -sin theta). */
static void or_exit_frame(const double xh[3], double* cpsi, double* spsi, double* cos_t,
                          double* sin_t) {
    double psi = atan2(xh[1], xh[0]);
    *cpsi = cos(psi);
    *spsi = sin(psi);
    *cos_t = xh[2];
    *sin_t = sqrt(xh[0] * xh[0] + xh[1] * xh[1]);
}

static void or_rot_z_neg(double c, double s, const double v[3], double out[3]) {
    out[0] = c * v[0] + s * v[1];
    out[1] = -s * v[0] + c * v[1];
    out[2] = v[2];
}

static void or_walk_one(const or_walk_desc* d, const or_walk_out* o, uint64_t i) {
    const uint64_t n = d->n_photons;
    const uint64_t id = d->photon_offset + i;
    double st, g, phi, r;
    if (d->mode == OR_WALK_TRAINING) {
        double u[4];
        or_uniform4(d->seed, OR_TAG_WALK_PARAM, id, 0, u);
        /* (sigma_t r, g)-weighted data (Sec. 5.3): the focus region with
         * probability focus_fraction, decided exactly on the 24-bit integer
         * k = U 2^24 against floor(focus_fraction 2^24) */
        const double* sr = d->st_range;
        const double* gr = d->g_range;
        if (u[3] * 16777216.0 <= floor(d->focus_fraction * 16777216.0)) {
            sr = d->focus_st_range;
            gr = d->focus_g_range;
        }
        st = sr[0] * pow(sr[1] / sr[0], u[0]);
        g = gr[0] + (gr[1] - gr[0]) * u[1];
        phi = d->albedo_range[0] + (d->albedo_range[1] - d->albedo_range[0]) * u[2];
        r = 1.0;
    } else {
        /* flights are in world units; sigma_t * r is what the CVAEs see */
        st = d->sigma_t;
        g = d->g;
        phi = d->albedo;
        r = d->radius;
    }
    /* Survival at an event iff U3 <= albedo, with U3 = k 2^-24, i.e. iff
     * k <= floor(albedo 2^24): an exact integer decision. */
    const uint64_t surv_thr = (uint64_t)floor(phi * OR_U24);

    double x[3] = {0.0, 0.0, 0.0};
    double dir[3] = {0.0, 0.0, 1.0};
    double xk[3] = {0.0, 0.0, 0.0}, wk[3] = {0.0, 0.0, 1.0};
    uint32_t k = 1;
    double resv = 0.0; /* Lambda_i / albedo^i for the albedo-power reservoir */
    uint32_t nev = 0, c0 = 0;
    int absorbed = 0, truncated = 0;
    double xe[3] = {0, 0, 0};

    for (;;) {
        ++nev;
        uint32_t w[4];
        or_philox_blocks(d->seed, OR_TAG_WALK_EVENT, id, c0++, 1, w);
        uint64_t k3 = (uint64_t)(w[3] >> 8) + 1u;
        if (d->mode == OR_WALK_ANALOG) {
            if (k3 > surv_thr) {
                absorbed = 1;
                memcpy(xe, x, sizeof xe);
                break;
            }
        } else {
            /* Weighted single-item reservoir: event i replaces the kept one
             * with probability w_i / sum_{j<=i} w_j, so event k is kept with
             * probability w_k / sum_j w_j (Sec. 4.3 with w_i = albedo^i). */
            int keep;
            if (d->event_weighting == OR_EVENT_UNIFORM) {
                keep = k3 * (uint64_t)nev <= (uint64_t)OR_U24;
            } else {
                resv = (nev == 1) ? 1.0 : 1.0 + resv / phi;
                keep = or_u01(w[3]) * resv <= 1.0;
            }
            if (keep) {
                memcpy(xk, x, sizeof xk);
                memcpy(wk, dir, sizeof wk);
                k = nev;
            }
        }
        double mu = or_hg_sample(g, or_u01(w[1]));
        or_scatter_dir(dir, mu, 2.0 * OR_PI * or_u01(w[2]));
        double l = -log(or_u01(w[0])) / st;
        double xn[3] = {x[0] + l * dir[0], x[1] + l * dir[1], x[2] + l * dir[2]};
        if (xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2] >= r * r) {
            double b = x[0] * dir[0] + x[1] * dir[1] + x[2] * dir[2];
            double c = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] - r * r;
            double t = -b + sqrt(fmax(0.0, b * b - c));
            for (int j = 0; j < 3; ++j) xe[j] = x[j] + t * dir[j];
            break;
        }
        memcpy(x, xn, sizeof x);
        if (d->max_events && nev >= d->max_events) {
            truncated = 1;
            memcpy(xe, x, sizeof xe);
            break;
        }
    }

    if (o->params) {
        double p3[3] = {st * r, g, phi};
        or_put3(o->params, n, i, p3);
    }
    if (o->n_scatter) o->n_scatter[i] = nev;
    if (o->absorbed) o->absorbed[i] = (uint8_t)absorbed;
    if (o->truncated) o->truncated[i] = (uint8_t)truncated;
    or_put3(o->exit_pos, n, i, xe);
    or_put3(o->exit_dir, n, i, dir);

    double xh[3] = {xe[0] / r, xe[1] / r, xe[2] / r};
    double cpsi, spsi, cos_t, sin_t;
    or_exit_frame(xh, &cpsi, &spsi, &cos_t, &sin_t);
    if (o->exit_param) {
        double wp[3];
        or_rot_z_neg(cpsi, spsi, dir, wp);
        double ep[3] = {cos_t, wp[1], wp[0] * cos_t - wp[2] * sin_t};
        or_put3(o->exit_param, n, i, ep);
    }
    if (d->mode == OR_WALK_TRAINING) {
        if (o->event_index) o->event_index[i] = k;
        double xs[3] = {xk[0] / r, xk[1] / r, xk[2] / r}, xc[3], wc[3];
        or_rot_z_neg(cpsi, spsi, xs, xc);
        or_rot_z_neg(cpsi, spsi, wk, wc);
        or_put3(o->event_pos, n, i, xc);
        or_put3(o->event_dir, n, i, wc);
    }
}

typedef struct {
    const or_walk_desc* d;
    const or_walk_out* o;
    int t, nt;
} or_walk_job;

static void* or_walk_worker(void* arg) {
    or_walk_job* j = (or_walk_job*)arg;
    for (uint64_t i = (uint64_t)j->t; i < j->d->n_photons; i += (uint64_t)j->nt)
        or_walk_one(j->d, j->o, i);
    return NULL;
}

int or_random_walk(const or_walk_desc* d, const or_walk_out* o) {
    if (!d || !o) return -1;
    int nt = d->n_threads > 0 ? d->n_threads : 1;
    if (nt > 256) nt = 256;
    pthread_t th[256];
    or_walk_job jobs[256];
    for (int t = 0; t < nt; ++t) {
        jobs[t].d = d;
        jobs[t].o = o;
        jobs[t].t = t;
        jobs[t].nt = nt;
        if (nt == 1) {
            or_walk_worker(&jobs[t]);
        } else {
            pthread_create(&th[t], NULL, or_walk_worker, &jobs[t]);
        }
    }
    if (nt > 1)
        for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    return 0;
}
