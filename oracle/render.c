/*
 * render.c -- oracle geometry, plain path tracer with next-event estimation
 * and the sphere-tracing renderer.  TEST INFRASTRUCTURE ONLY (see
 * msst_oracle.h).
 *
 * Method (Sec. 3 and its overview figure): a camera path enters the
 * translucent body and moves by free flights l = -log(1 - xi) / sigma_t
 * (delta tracking in a homogeneous medium).  At a collision the plain path
 * tracer scatters once (absorption roulette, HG direction).  The sphere
 * tracer instead asks a signed distance for the largest sphere around the
 * collision that stays inside the body, rescales sigma_t -> sigma_t r
 * (Sec. 4.1) and replaces the whole scattering chain inside that sphere by
 * one learned step: LengthGen gives N, the path survives with probability
 * albedo^N (Sec. 3.2), PathGen gives the exit (theta, alpha, beta) placed by
 * the rotation of Eq. (transform), EventGen a representative event (X, W).
 * Direct light from a point light is added by next-event estimation
 * (Sec. 4.3, Eq. directLighting): at every plain event with weight albedo,
 * at the representative event of a sphere step with weight
 * Lambda^(N) / albedo^N.  There is no refraction at the boundary (Sec. 4.3),
 * so rays cross it unchanged; the background is black.
 */
#include "msst_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288
#define OR_U24 16777216.0
#define OR_MAX_IV 16

/* ---------------- primitives ---------------- */

static double or_dot(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void or_normalize(double v[3]) {
    double l = sqrt(or_dot(v, v));
    v[0] /= l;
    v[1] /= l;
    v[2] /= l;
}

static double or_prim_sdf(const float* pr, const double p[3]) {
    double q[3] = {p[0] - pr[1], p[1] - pr[2], p[2] - pr[3]};
    if ((int)pr[0] == OR_PRIM_SPHERE) return sqrt(or_dot(q, q)) - pr[4];
    double e[3] = {fabs(q[0]) - pr[4], fabs(q[1]) - pr[5], fabs(q[2]) - pr[6]};
    double out[3] = {fmax(e[0], 0.0), fmax(e[1], 0.0), fmax(e[2], 0.0)};
    double inside = fmin(fmax(e[0], fmax(e[1], e[2])), 0.0);
    return sqrt(or_dot(out, out)) + inside;
}

/* ---------------- triangle meshes ---------------- */

/* Line parameter t of the crossing of o + t d with triangle (a, b, c), any t
 * (Moller and Trumbore, "Fast, Minimum Storage Ray/Triangle Intersection",
 * JGT 1997, without back-face culling); 0 if the line misses it. */
static int or_tri_cross(const float* tr, const double o[3], const double d[3], double* t) {
    double a[3] = {tr[0], tr[1], tr[2]}, e1[3], e2[3], s[3], pv[3], qv[3];
    for (int i = 0; i < 3; ++i) {
        e1[i] = (double)tr[3 + i] - a[i];
        e2[i] = (double)tr[6 + i] - a[i];
        s[i] = o[i] - a[i];
    }
    pv[0] = d[1] * e2[2] - d[2] * e2[1];
    pv[1] = d[2] * e2[0] - d[0] * e2[2];
    pv[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = or_dot(e1, pv);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    double u = or_dot(s, pv) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    qv[0] = s[1] * e1[2] - s[2] * e1[1];
    qv[1] = s[2] * e1[0] - s[0] * e1[2];
    qv[2] = s[0] * e1[1] - s[1] * e1[0];
    double v = or_dot(d, qv) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    *t = or_dot(e2, qv) * inv;
    return 1;
}

/* All crossings of the whole line with the mesh, sorted; returns their
 * number (at most cap). */
static int or_mesh_crossings(const or_scene* sc, const double o[3], const double d[3], double* tc, int cap) {
    int n = 0;
    for (int i = 0; i < sc->n_tris; ++i) {
        double t;
        if (!or_tri_cross(sc->tris + 9 * i, o, d, &t)) continue;
        if (n == cap) return cap + 1;
        int k = n++;
        while (k > 0 && tc[k - 1] > t) {
            tc[k] = tc[k - 1];
            --k;
        }
        tc[k] = t;
    }
    return n;
}

/* Distance from p to triangle tr (closest point by region tests, after
 * Ericson, "Real-Time Collision Detection", Sec. 5.1.5). */
static double or_tri_distance(const float* tr, const double p[3]) {
    double a[3], b[3], c[3], ab[3], ac[3], ap[3], bp[3], cp[3], q[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = tr[i];
        b[i] = tr[3 + i];
        c[i] = tr[6 + i];
        ab[i] = b[i] - a[i];
        ac[i] = c[i] - a[i];
        ap[i] = p[i] - a[i];
        bp[i] = p[i] - b[i];
        cp[i] = p[i] - c[i];
    }
    double d1 = or_dot(ab, ap), d2 = or_dot(ac, ap);
    double d3 = or_dot(ab, bp), d4 = or_dot(ac, bp);
    double d5 = or_dot(ab, cp), d6 = or_dot(ac, cp);
    double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    if (d1 <= 0.0 && d2 <= 0.0) {
        for (int i = 0; i < 3; ++i) q[i] = a[i];
    } else if (d3 >= 0.0 && d4 <= d3) {
        for (int i = 0; i < 3; ++i) q[i] = b[i];
    } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int i = 0; i < 3; ++i) q[i] = a[i] + v * ab[i];
    } else if (d6 >= 0.0 && d5 <= d6) {
        for (int i = 0; i < 3; ++i) q[i] = c[i];
    } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double w = d2 / (d2 - d6);
        for (int i = 0; i < 3; ++i) q[i] = a[i] + w * ac[i];
    } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int i = 0; i < 3; ++i) q[i] = b[i] + w * (c[i] - b[i]);
    } else {
        double den = 1.0 / (va + vb + vc), v = vb * den, w = vc * den;
        for (int i = 0; i < 3; ++i) q[i] = a[i] + ab[i] * v + ac[i] * w;
    }
    double e[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    return sqrt(or_dot(e, e));
}

/* A fixed direction for inside tests, away from the axes and diagonals. */
static const double OR_PARITY_DIR[3] = {0.2672612419124244, 0.5345224838248488, 0.8017837257372732};

static double or_mesh_sdf(const or_scene* sc, const double p[3]) {
    double dmin = INFINITY;
    int odd = 0;
    for (int i = 0; i < sc->n_tris; ++i) {
        dmin = fmin(dmin, or_tri_distance(sc->tris + 9 * i, p));
        double t;
        if (or_tri_cross(sc->tris + 9 * i, p, OR_PARITY_DIR, &t) && t > 0.0) odd ^= 1;
    }
    return odd ? -dmin : dmin;
}

double or_scene_sdf(const or_scene* sc, const double p[3]) {
    if (sc->n_tris > 0) return or_mesh_sdf(sc, p);
    double s = INFINITY;
    for (int i = 0; i < sc->n_prims; ++i) s = fmin(s, or_prim_sdf(sc->prims + 8 * i, p));
    return s;
}

/* Parametric interval [t0, t1] of a ray inside one convex primitive. */
static int or_prim_interval(const float* pr, const double o[3], const double d[3], double* t0,
                            double* t1) {
    double q[3] = {o[0] - pr[1], o[1] - pr[2], o[2] - pr[3]};
    if ((int)pr[0] == OR_PRIM_SPHERE) {
        double b = or_dot(q, d);
        double c = or_dot(q, q) - (double)pr[4] * pr[4];
        double disc = b * b - c;
        if (disc <= 0.0) return 0;
        double s = sqrt(disc);
        *t0 = -b - s;
        *t1 = -b + s;
        return 1;
    }
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double h = pr[4 + a];
        if (d[a] == 0.0) {
            if (q[a] < -h || q[a] > h) return 0;
            continue;
        }
        double ta = (-h - q[a]) / d[a], tb = (h - q[a]) / d[a];
        if (ta > tb) {
            double tmp = ta;
            ta = tb;
            tb = tmp;
        }
        lo = fmax(lo, ta);
        hi = fmin(hi, tb);
    }
    if (lo >= hi) return 0;
    *t0 = lo;
    *t1 = hi;
    return 1;
}

/* Sorted, merged intervals of the ray inside the union of all primitives. */
int or_ray_intervals(const or_scene* sc, const double o[3], const double d[3], double* t0,
                     double* t1, int cap) {
    if (sc->n_tris > 0) {
        /* a closed mesh: consecutive crossings of the whole line pair up as
         * (entry, exit); an odd count (a crossing lost on an edge) drops the
         * last one */
        double tc[2 * OR_MAX_IV];
        int n = or_mesh_crossings(sc, o, d, tc, 2 * OR_MAX_IV);
        if (n > 2 * OR_MAX_IV) n = 2 * OR_MAX_IV;
        int m = 0;
        for (int i = 0; i + 1 < n && m < cap; i += 2, ++m) {
            t0[m] = tc[i];
            t1[m] = tc[i + 1];
        }
        return m;
    }
    double a[OR_MAX_IV * 8], b[OR_MAX_IV * 8];
    int n = 0;
    for (int i = 0; i < sc->n_prims && n < OR_MAX_IV * 8; ++i) {
        double x0, x1;
        if (or_prim_interval(sc->prims + 8 * i, o, d, &x0, &x1)) {
            int k = n++;
            while (k > 0 && a[k - 1] > x0) {
                a[k] = a[k - 1];
                b[k] = b[k - 1];
                --k;
            }
            a[k] = x0;
            b[k] = x1;
        }
    }
    int m = 0;
    for (int i = 0; i < n; ++i) {
        if (m > 0 && a[i] <= t1[m - 1]) {
            if (b[i] > t1[m - 1]) t1[m - 1] = b[i];
        } else if (m < cap) {
            t0[m] = a[i];
            t1[m] = b[i];
            ++m;
        }
    }
    return m;
}

/* fp16 bit pattern of x rounded toward zero (finite range only). */
static uint16_t or_fp16_rtz(double x) {
    uint16_t sign = x < 0 ? 0x8000u : 0;
    double a = fabs(x);
    if (a >= 65504.0) return (uint16_t)(sign | 0x7bffu);
    if (a < ldexp(1.0, -24)) return sign;
    int e;
    frexp(a, &e);
    int ex = e - 1; /* a in [2^ex, 2^(ex+1)) */
    if (ex < -14) {
        uint32_t m = (uint32_t)floor(a / ldexp(1.0, -24));
        return (uint16_t)(sign | m);
    }
    uint32_t mant = (uint32_t)floor((a / ldexp(1.0, ex) - 1.0) * 1024.0);
    return (uint16_t)(sign | ((uint32_t)(ex + 15) << 10) | mant);
}

static double or_fp16_value(uint16_t h) {
    int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
    double v = e == 0 ? ldexp((double)m, -24) : ldexp(1.0 + m / 1024.0, e - 15);
    return s ? -v : v;
}

/* Grid of signed distances at voxel centres lo + (i + 1/2) h, rounded toward
 * zero to binary16 so that |stored| <= |exact|: the voxel-grid distance
 * pre-process of Sec. 3, with a Euclidean lower bound in place of the
 * Chebyshev distance. */
void or_build_sdf_grid(const or_scene* sc, int32_t res, const float lo[3], const float hi[3],
                       uint16_t* out) {
    for (int64_t k = 0; k < res; ++k)
        for (int64_t j = 0; j < res; ++j)
            for (int64_t i = 0; i < res; ++i) {
                double p[3] = {lo[0] + (i + 0.5) * ((double)hi[0] - lo[0]) / res,
                               lo[1] + (j + 0.5) * ((double)hi[1] - lo[1]) / res,
                               lo[2] + (k + 0.5) * ((double)hi[2] - lo[2]) / res};
                out[(k * res + j) * res + i] = or_fp16_rtz(or_scene_sdf(sc, p));
            }
}

/* Radius of a sphere around p that lies inside the body.  Without a grid:
 * the union distance min_i sdf_i, which bounds the interior distance from
 * below, shrunk by 0.1 % so the sphere never touches the surface.  With a
 * grid: the nearest voxel's stored value minus the half voxel diagonal
 * (signed distances are 1-Lipschitz). */
double or_conservative_radius(const or_scene* sc, const double p[3]) {
    if (sc->sdf_fp16 && sc->res > 0) {
        int idx[3];
        double hmax = 0.0;
        for (int a = 0; a < 3; ++a) {
            double h = ((double)sc->hi[a] - sc->lo[a]) / sc->res;
            hmax = fmax(hmax, h);
            double f = (p[a] - sc->lo[a]) / h;
            if (!(f >= 0.0) || f >= sc->res) return 0.0;
            idx[a] = (int)floor(f);
        }
        double s = or_fp16_value(sc->sdf_fp16[((int64_t)idx[2] * sc->res + idx[1]) * sc->res + idx[0]]);
        double r = -s - 0.5 * sqrt(3.0) * hmax;
        return r > 0.0 ? r : 0.0;
    }
    double s = or_scene_sdf(sc, p);
    return s < 0.0 ? -0.999 * s : 0.0;
}

/* In-medium length of the segment from p to q (the d_t of Sec. 4.3). */
static double or_medium_length(const or_scene* sc, const double p[3], const double q[3]) {
    double d[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    double len = sqrt(or_dot(d, d));
    if (len == 0.0) return 0.0;
    for (int i = 0; i < 3; ++i) d[i] /= len;
    double t0[OR_MAX_IV], t1[OR_MAX_IV];
    int m = or_ray_intervals(sc, p, d, t0, t1, OR_MAX_IV);
    double acc = 0.0;
    for (int i = 0; i < m; ++i) {
        double a = fmax(t0[i], 0.0), b = fmin(t1[i], len);
        if (b > a) acc += b - a;
    }
    return acc;
}

/* Point-light next-event estimate at x for a path arriving along d:
 * I rho_g(d . w_{x->L}) exp(-sigma_t d_t) / |x_L - x|^2 (Sec. 4.3). */
static double or_nee(const or_scene* sc, const or_light* lt, const or_medium* md, const double x[3],
                     const double d[3]) {
    double wl[3] = {lt->pos[0] - x[0], lt->pos[1] - x[1], lt->pos[2] - x[2]};
    double dist2 = or_dot(wl, wl);
    double dist = sqrt(dist2);
    for (int i = 0; i < 3; ++i) wl[i] /= dist;
    double dt = or_medium_length(sc, x, lt->pos);
    return lt->intensity * or_hg_eval(md->g, or_dot(d, wl)) * exp(-md->sigma_t * dt) / dist2;
}

/* ---------------- learned sphere step ---------------- */

/* De-standardised sample of one decoder from standard normals nrm[0..L+P). */
static void or_model_sample(const or_render_desc* rd, int model, const double* cond,
                            const double* nrm, double* y) {
    const or_cvae_shape* s = &rd->shapes[model];
    const double* st = rd->stats[model];
    double cs[16], mu[16], lv[16];
    for (int k = 0; k < s->p_in; ++k) cs[k] = (cond[k] - st[k]) / st[16 + k];
    or_cvae_decode(s, rd->params[model], rd->precision, rd->act_scales[model], nrm, cs, mu, lv);
    for (int k = 0; k < s->p_out; ++k)
        y[k] = (mu[k] + exp(0.5 * lv[k]) * nrm[s->latent + k]) * st[48 + k] + st[32 + k];
}

static void or_draw_normals(const or_render_desc* rd, uint64_t id, uint32_t* c0, int count,
                            double* nrm) {
    for (int j = 0; j * 4 < count; ++j) or_normal4(rd->seed, OR_TAG_RENDER_PATH, id, (*c0)++, nrm + 4 * j);
}

/* Sum_{i=1..N} albedo^i / albedo^N, the next-event weight of a sphere step
 * that survived its absorption test (Sec. 4.3 with the reject-first order
 * of Sec. 3.2). */
static double or_lambda_weight(double phi, double N) {
    if (phi >= 1.0) return N;
    return phi * expm1(-N * log(phi)) / (1.0 - phi);
}

typedef or_step_result or_step;

/* Learned sphere step (Sec. 3.2 with the models of Sec. 4) in the sphere of
 * radius r around p entered along d: LengthGen gives N, the chain is absorbed
 * with probability 1 - albedo^N, PathGen gives the exit, and the direct light
 * at K representative events is averaged.  Each representative event is the
 * first one (the centre, entered along w_in) with probability
 * albedo / Lambda^(N) (Sec. 4.3), taken exactly; EventGen samples the others.
 * A single event (N = 1) is one HG scatter at the centre (Sec. 3.1), sampled
 * exactly instead of asking PathGen for a point mass.  With OR_STEP_PAPER the
 * step is the paper's as printed: PathGen for every step that is lit and
 * EventGen for every representative event, whatever N and k.
 * Random numbers are drawn in a fixed order: LengthGen normals; one block
 * (absorption, psi, HG, first-event test of sample 0); PathGen normals; then
 * per sample k: a block for its first-event test (k > 0) and EventGen
 * normals.  The paper's order draws the same blocks and leaves the HG and
 * first-event uniforms unused. */
static void or_cvae_step(const or_render_desc* rd, const or_medium* md, uint64_t id, uint32_t* c0,
                         const double p[3], const double d[3], double r, or_step* out) {
    double str = md->sigma_t * r, lst = log(str), g = md->g, phi = md->albedo;
    int K = rd->nee_samples > 0 ? rd->nee_samples : 1;
    int before = (rd->flags & OR_NEE_BEFORE_ABSORPTION) != 0;
    int paper = (rd->flags & OR_STEP_PAPER) != 0;
    memset(out->first, 0, sizeof out->first);
    double nrm[16], y[8];
    /* LengthGen */
    double c_len[2] = {lst, g};
    or_draw_normals(rd, id, c0, rd->shapes[0].latent + rd->shapes[0].p_out, nrm);
    or_model_sample(rd, 0, c_len, nrm, y);
    double ey = exp(fmin(y[0], 20.0));
    double N = floor(ey + 0.5);
    if (N < 1.0) N = 1.0;
    out->N = N;
    double u[4];
    or_uniform4(rd->seed, OR_TAG_RENDER_PATH, id, (*c0)++, u);
    /* absorption along the bypassed chain: survive with probability albedo^N */
    double phiN = exp(N * log(phi));
    out->survived = u[0] <= phiN;
    int lit = before ? 1 : out->survived;
    /* With nee_chain, the step's own number of representative events: one
     * more per nee_chain events of its chain, up to nee_samples (the
     * variance of a one-event estimate grows with the square of its weight,
     * which grows with N; K follows N alone, so the estimate stays unbiased) */
    if (rd->nee_chain > 0) {
        int64_t more = ((int64_t)N - 1) / rd->nee_chain;
        if (more + 1 < K) K = (int)(more + 1);
    }
    out->n_rep = lit ? K : 0;
    /* Lambda^(N) = sum_{i=1..N} albedo^i; survivors carry Lambda / albedo^N */
    double lam = phi >= 1.0 ? N : phi * -expm1(N * log(phi)) / (1.0 - phi);
    out->nee_w = (before ? lam : or_lambda_weight(phi, N)) / K;
    if (!lit) return;
    double psi = 2.0 * OR_PI * u[1];
    out->psi = psi;
    double ct, al = 0.0, be = 0.0, ga = 1.0;
    if (N < 2.0 && !paper) {
        ct = or_hg_sample(g, u[2]);
    } else {
        /* PathGen */
        double c_path[3] = {lst, g, log(N)};
        or_draw_normals(rd, id, c0, rd->shapes[1].latent + rd->shapes[1].p_out, nrm);
        or_model_sample(rd, 1, c_path, nrm, y);
        ct = fmin(1.0, fmax(-1.0, y[0]));
        al = y[1];
        be = y[2];
        ga = sqrt(fmax(0.0, 1.0 - al * al - be * be));
        double nl = sqrt(al * al + be * be + ga * ga);
        al /= nl;
        be /= nl;
        ga /= nl;
    }
    double e1[3], e2[3];
    or_onb(d, e1, e2);
    double cp = cos(psi), sp = sin(psi);
    double p_first = phi >= 1.0 ? 1.0 / N : (1.0 - phi) / (-expm1(N * log(phi)));
    for (int k = 0; k < K; ++k) {
        double uf = u[3];
        if (k > 0) {
            double v[4];
            or_uniform4(rd->seed, OR_TAG_RENDER_PATH, id, (*c0)++, v);
            uf = v[0];
        }
        double X[3] = {0.0, 0.0, 0.0}, W[3] = {0.0, 0.0, 1.0};
        out->first[k] = 1;
        if (paper || (N >= 2.0 && !(uf <= p_first))) {
            out->first[k] = 0;
            double c_ev[7] = {lst, g, phi, ct, al, be, log(N)};
            or_draw_normals(rd, id, c0, rd->shapes[2].latent + rd->shapes[2].p_out, nrm);
            or_model_sample(rd, 2, c_ev, nrm, y);
            for (int i = 0; i < 3; ++i) {
                X[i] = y[i];
                W[i] = y[3 + i];
            }
            double xl = sqrt(or_dot(X, X));
            if (xl > 1.0)
                for (int i = 0; i < 3; ++i) X[i] /= xl;
            double wl = sqrt(or_dot(W, W));
            if (wl > 0.0) {
                for (int i = 0; i < 3; ++i) W[i] /= wl;
            } else {
                W[0] = 0.0;
                W[1] = 0.0;
                W[2] = 1.0;
            }
        }
        /* (X, W) rotated by psi about w_in, then into R = [e1 e2 d] */
        double Xt[3] = {cp * X[0] - sp * X[1], sp * X[0] + cp * X[1], X[2]};
        double Wt[3] = {cp * W[0] - sp * W[1], sp * W[0] + cp * W[1], W[2]};
        for (int i = 0; i < 3; ++i) {
            out->X[k][i] = p[i] + r * (Xt[0] * e1[i] + Xt[1] * e2[i] + Xt[2] * d[i]);
            out->W[k][i] = Wt[0] * e1[i] + Wt[1] * e2[i] + Wt[2] * d[i];
        }
        or_normalize(out->W[k]);
    }
    if (!out->survived) return;
    /* Eq. (transform): x = p + r R R_psi x~ with R = [e1 e2 d], plus the
     * exit-frame direction of Sec. 4.1. */
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double xt[3] = {st * cp, st * sp, ct};
    double w0[3] = {be * ct + ga * st, al, -be * st + ga * ct};
    double wt[3] = {cp * w0[0] - sp * w0[1], sp * w0[0] + cp * w0[1], w0[2]};
    for (int i = 0; i < 3; ++i) {
        out->x[i] = p[i] + r * (xt[0] * e1[i] + xt[1] * e2[i] + xt[2] * d[i]);
        out->w[i] = wt[0] * e1[i] + wt[1] * e2[i] + wt[2] * d[i];
    }
    or_normalize(out->w);
}

/* Reference sphere step: the actual random walk inside the sphere (the
 * process the CVAEs learn), with the representative event drawn by the
 * albedo-power reservoir and the absorption decided after the walk. */
static void or_exact_step(const or_render_desc* rd, const or_medium* md, uint64_t id, uint32_t* c0,
                          const double p[3], const double d[3], double r, or_step* out) {
    double x[3] = {p[0], p[1], p[2]}, dir[3] = {d[0], d[1], d[2]};
    double phi = md->albedo, resv = 0.0;
    uint32_t nev = 0;
    for (;;) {
        ++nev;
        double u[4];
        or_uniform4(rd->seed, OR_TAG_RENDER_PATH, id, (*c0)++, u);
        resv = (nev == 1) ? 1.0 : 1.0 + resv / phi;
        if (u[3] * resv <= 1.0) {
            memcpy(out->X[0], x, sizeof out->X[0]);
            memcpy(out->W[0], dir, sizeof out->W[0]);
        }
        double mu = or_hg_sample(md->g, u[1]);
        or_scatter_dir(dir, mu, 2.0 * OR_PI * u[2]);
        double l = -log(u[0]) / md->sigma_t;
        double q[3] = {x[0] - p[0] + l * dir[0], x[1] - p[1] + l * dir[1], x[2] - p[2] + l * dir[2]};
        if (or_dot(q, q) >= r * r) {
            double rel[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
            double b = or_dot(rel, dir), c = or_dot(rel, rel) - r * r;
            double t = -b + sqrt(fmax(0.0, b * b - c));
            for (int i = 0; i < 3; ++i) out->x[i] = x[i] + t * dir[i];
            break;
        }
        for (int i = 0; i < 3; ++i) x[i] += l * dir[i];
    }
    memcpy(out->w, dir, sizeof out->w);
    out->N = (double)nev;
    double u[4];
    or_uniform4(rd->seed, OR_TAG_RENDER_PATH, id, (*c0)++, u);
    out->survived = u[0] <= exp(out->N * log(phi));
    out->n_rep = out->survived;
    out->nee_w = or_lambda_weight(phi, out->N);
}

/* One sphere step on its own (test entry): the learned step, or the exact
 * in-sphere walk with sampler OR_SAMPLER_EXACT_WALK, for path id `id` with
 * its draw counter at c0; returns the counter after the step. */
uint32_t or_sphere_step(const or_render_desc* rd, const or_medium* md, uint64_t id, uint32_t c0,
                        const double p[3], const double d[3], double r, or_step_result* out) {
    memset(out, 0, sizeof *out);
    if (rd->sampler == OR_SAMPLER_EXACT_WALK) or_exact_step(rd, md, id, &c0, p, d, r, out);
    else or_cvae_step(rd, md, id, &c0, p, d, r, out);
    return c0;
}

/* ---------------- path ---------------- */

typedef struct {
    double value, events, steps;
} or_path_result;

static void or_camera_ray(const or_camera* cam, int64_t pixel, double jx, double jy, double o[3],
                          double d[3]) {
    double f[3] = {cam->look_at[0] - cam->eye[0], cam->look_at[1] - cam->eye[1],
                   cam->look_at[2] - cam->eye[2]};
    or_normalize(f);
    double rt[3] = {f[1] * cam->up[2] - f[2] * cam->up[1], f[2] * cam->up[0] - f[0] * cam->up[2],
                    f[0] * cam->up[1] - f[1] * cam->up[0]};
    or_normalize(rt);
    double uv[3] = {rt[1] * f[2] - rt[2] * f[1], rt[2] * f[0] - rt[0] * f[2],
                    rt[0] * f[1] - rt[1] * f[0]};
    double th = tan(0.5 * cam->vfov_deg * OR_PI / 180.0);
    double aspect = (double)cam->width / cam->height;
    int64_t px = pixel % cam->width, py = pixel / cam->width;
    double sx = (2.0 * (px + jx) / cam->width - 1.0) * th * aspect;
    double sy = (1.0 - 2.0 * (py + jy) / cam->height) * th;
    for (int i = 0; i < 3; ++i) {
        o[i] = cam->eye[i];
        d[i] = f[i] + sx * rt[i] + sy * uv[i];
    }
    or_normalize(d);
}

static or_path_result or_trace_path(const or_scene* sc, const or_camera* cam, const or_light* lt,
                                    const or_medium* md, const or_render_desc* rd, int64_t pixel,
                                    uint64_t sample) {
    or_path_result res = {0.0, 0.0, 0.0};
    const uint64_t id = (uint64_t)pixel | (sample << 32);
    double jit[4];
    or_uniform4(rd->seed, OR_TAG_RENDER_PIXEL, id, 0, jit);
    double o[3], d[3];
    or_camera_ray(cam, pixel, jit[0], jit[1], o, d);
    const double phi = md->albedo;
    const uint64_t surv_thr = (uint64_t)floor(phi * OR_U24);
    uint32_t c0 = 0;
    double t0[OR_MAX_IV], t1[OR_MAX_IV];
    int m = or_ray_intervals(sc, o, d, t0, t1, OR_MAX_IV);
    double t = 0.0;
    uint32_t iters = 0;
    for (;;) {
        /* the medium interval that the ray is in or enters next */
        int k = -1;
        for (int i = 0; i < m; ++i)
            if (t1[i] > t) {
                k = i;
                break;
            }
        if (k < 0) break; /* escapes to the black background */
        if (t0[k] > t) t = t0[k];
        uint32_t wv[4];
        or_philox_blocks(rd->seed, OR_TAG_RENDER_PATH, id, c0++, 1, wv);
        double l = -log(or_u01(wv[0])) / md->sigma_t;
        if (t + l >= t1[k]) {
            t = t1[k];
            continue;
        }
        t += l;
        double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        if (rd->max_events && ++iters > rd->max_events) break;
        if (rd->method == OR_METHOD_ST) {
            double r = fmin(or_conservative_radius(sc, p), rd->st_max / md->sigma_t);
            if (md->sigma_t * r >= rd->tau_min) {
                or_step st;
                if (rd->sampler == OR_SAMPLER_EXACT_WALK)
                    or_exact_step(rd, md, id, &c0, p, d, r, &st);
                else
                    or_cvae_step(rd, md, id, &c0, p, d, r, &st);
                res.steps += 1.0;
                for (int k = 0; k < st.n_rep; ++k) res.value += st.nee_w * or_nee(sc, lt, md, st.X[k], st.W[k]);
                if (!st.survived) break;
                memcpy(o, st.x, sizeof o);
                memcpy(d, st.w, sizeof d);
                m = or_ray_intervals(sc, o, d, t0, t1, OR_MAX_IV);
                t = 0.0;
                continue;
            }
        }
        /* plain event: NEE weighted by the albedo, roulette, HG scatter */
        res.events += 1.0;
        res.value += phi * or_nee(sc, lt, md, p, d);
        if ((uint64_t)(wv[3] >> 8) + 1u > surv_thr) break;
        double mu = or_hg_sample(md->g, or_u01(wv[1]));
        or_scatter_dir(d, mu, 2.0 * OR_PI * or_u01(wv[2]));
        memcpy(o, p, sizeof o);
        m = or_ray_intervals(sc, o, d, t0, t1, OR_MAX_IV);
        t = 0.0;
    }
    return res;
}

typedef struct {
    const or_scene* sc;
    const or_camera* cam;
    const or_light* lt;
    const or_medium* md;
    const or_render_desc* rd;
    const or_image_out* img;
    int t, nt;
} or_render_job;

static void* or_render_worker(void* arg) {
    or_render_job* j = (or_render_job*)arg;
    const or_render_desc* rd = j->rd;
    int64_t npx = rd->n_pixels > 0 ? rd->n_pixels : (int64_t)j->cam->width * j->cam->height;
    for (int64_t q = j->t; q < npx; q += j->nt) {
        int64_t pixel = rd->pixels ? rd->pixels[q] : q;
        double s = 0.0, s2 = 0.0, ev = 0.0, stp = 0.0;
        for (int32_t k = 0; k < rd->spp; ++k) {
            or_path_result r =
                or_trace_path(j->sc, j->cam, j->lt, j->md, rd, pixel, rd->sample_offset + (uint64_t)k);
            s += r.value;
            s2 += r.value * r.value;
            ev += r.events;
            stp += r.steps;
        }
        if (j->img->sum) j->img->sum[q] = s;
        if (j->img->sumsq) j->img->sumsq[q] = s2;
        if (j->img->events) j->img->events[q] = ev;
        if (j->img->steps) j->img->steps[q] = stp;
    }
    return NULL;
}

int or_render(const or_scene* sc, const or_camera* cam, const or_light* light,
              const or_medium* med, const or_render_desc* rd, const or_image_out* img) {
    if (!sc || !cam || !light || !med || !rd || !img) return -1;
    int nt = rd->n_threads > 0 ? rd->n_threads : 1;
    if (nt > 256) nt = 256;
    pthread_t th[256];
    or_render_job jobs[256];
    for (int t = 0; t < nt; ++t) {
        or_render_job jb = {sc, cam, light, med, rd, img, t, nt};
        jobs[t] = jb;
        if (nt == 1) or_render_worker(&jobs[t]);
        else pthread_create(&th[t], NULL, or_render_worker, &jobs[t]);
    }
    if (nt > 1)
        for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    return 0;
}
