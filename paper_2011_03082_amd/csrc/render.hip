// render.hip -- persistent path tracer with next-event estimation and the
// learned sphere tracer (Sec. 3 and its overview figure; Sec. 4.1 radius
// rescale and exit frame; Sec. 4.3 direct light at a representative event).
//
// One lane carries one camera path at a time.  Work units are
// (pixel, chunk of samples), taken from a per-wave ticket pool, so waves stay
// full however long individual scattering chains are.  Each iteration of the
// wave loop has two phases:
//   VALU phase -- every lane that is not waiting advances its path by one
//                 free flight (plain scattering event, boundary crossing,
//                 path start or end);
//   MFMA phase -- once enough lanes wait for a learned sphere step, their
//                 decoder inputs are compacted into 16-path tiles in LDS and
//                 LengthGen, the absorption test, PathGen and EventGen run on
//                 matrix cores for exactly those lanes.
// Per-unit results go to a partial buffer and are reduced per pixel in a
// fixed order, so images are bitwise reproducible.
#include <math.h>

#include "host.hpp"
#include "mesh.hpp"
#include "packed.hpp"

namespace msst {

constexpr int kRenderWaves = 4;

// Lane states: no path in flight (NEED: start a sample, take a work unit,
// or wait for the parked path), tracing (FLY), waiting for a learned step
// (WAIT), path finished and not yet banked (END), no work left (DONE).
enum : int { S_NEED = 0, S_FLY = 2, S_WAIT = 3, S_DONE = 4, S_END = 5 };

// Per-lane words kept in LDS ([word][thread]): the work unit's compensated
// sum, compensation, sum of squares, event and step counts, next sample,
// end of its sample range and index (U_NONE: no unit), then the lane's
// launch totals of events, learned steps and truncated paths.
enum : int {
    U_SUM = 0, U_COMP, U_SQ, U_EV, U_ST, U_NEXT, U_END, U_UNIT, T_EVENTS, T_STEPS, T_TRUNC, kLaneWords
};
constexpr uint32_t U_NONE = 0xFFFFFFFFu;

// Result of one work unit (one pixel, `chunk` consecutive samples): the
// compensated radiance sum folded to binary32, the sum of squares and the
// event / learned-step counts, written with one 16-byte store.
struct alignas(16) UnitRecord {
    float sum, sumsq;
    uint32_t events, steps;
};

struct RenderArgs {
    const float* prims;  // device [n_prims][8]
    int n_prims;
    const BvhNode* bvh;  // mesh scenes: nodes and reordered triangles
    const float* tris;
    int n_nodes, n_tris;
    const uint16_t* grid;
    int res;
    float grid_lo[3], grid_inv_h[3], grid_half_diag;
    float eye[3], fwd[3], right[3], upv[3];
    int width, height;
    int64_t npix;
    float light[3], intensity;
    float sigma_t, inv_sigma_t, g, albedo, ln_albedo;
    uint32_t surv_thr;
    int method, sampler;
    const PackedModel* pm[3];
    float tau_min, st_max, min_chain;
    int spp, chunk, n_chunks;
    int64_t n_units;                      // below 2^32
    double inv_n_chunks, inv_width;       // reciprocals for the unit -> (pixel, chunk) split
    uint64_t seed, sample_offset;
    uint32_t max_events;
    int batch_min;
    int restart_min;
    int max_wait;
    int nee_samples, nee_chain;
    int flags;
    UnitRecord* part;  // [n_units], unit = pixel * n_chunks + chunk
    unsigned long long* ticket;
    unsigned long long* counters;
};

// Primitives held in registers for the whole kernel (NP slots).
template <int NP>
struct Prims {
    float p[NP][8];
    int n;
};

struct RenderLds {
    float x[64][kTile];  // decoder input rows of the compacted lanes; outputs overwrite them
    float eps[64][6];    // decoder posterior noise of each row (at most 6 outputs)
    uint4 rid[64];       // Philox stream (id_lo, id_hi) and first block of each row's normals
};

enum : int { kModePlain = 0, kModeStExact = 1, kModeStCvae = 2 };

// Events of one exact walk inside a sphere before it is cut off (the reference
// sampler; a sphere of optical radius 200 takes about 10^5 on average).
constexpr uint32_t kInnerWalkBound = 1u << 24;

// ---------------------------------------------------------------- geometry

__device__ __forceinline__ bool prim_interval(const float* pr, V3 o, V3 d, float& t0, float& t1) {
    const V3 q = v3(o.x - pr[1], o.y - pr[2], o.z - pr[3]);
    if (pr[0] == 0.0f) {  // sphere
        // discriminant from the closest-approach vector (Haines, Guenther,
        // Akenine-Moller, "Precision Improvements for Ray/Sphere
        // Intersection", Ray Tracing Gems, 2019): r^2 - |q - (q.d) d|^2 does
        // not cancel for distant origins the way b^2 - (|q|^2 - r^2) does;
        // the roots come from the stable quadratic form.
        const float b = dot(q, d);
        const V3 h = fma3(-b, d, q);
        const float r = pr[4];
        const float hl = fast_sqrt(dot(h, h));
        const float disc = (r - hl) * (r + hl);
        if (!(disc > 0.0f)) return false;
        const float s = fast_sqrt(disc);
        const float c = dot(q, q) - r * r;
        const float qq = b > 0.0f ? -b - s : -b + s;  // same sign as -b, no cancellation
        const float ta = fast_div(c, qq), tb = qq;
        t0 = __builtin_fminf(ta, tb);
        t1 = __builtin_fmaxf(ta, tb);
        return true;
    }
    float lo = -INFINITY, hi = INFINITY;
    const float qa[3] = {q.x, q.y, q.z}, da[3] = {d.x, d.y, d.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float h = pr[4 + a];
        if (da[a] == 0.0f) {
            if (qa[a] < -h || qa[a] > h) return false;
            continue;
        }
        const float inv = fast_rcp(da[a]);
        float ta = (-h - qa[a]) * inv, tb = (h - qa[a]) * inv;
        lo = __builtin_fmaxf(lo, __builtin_fminf(ta, tb));
        hi = __builtin_fminf(hi, __builtin_fmaxf(ta, tb));
    }
    if (!(lo < hi)) return false;
    t0 = lo;
    t1 = hi;
    return true;
}

// Intervals of one ray in each primitive (unused slots: [+inf, -inf]).
template <int NP>
struct RayIv {
    float a[NP], b[NP];
};

template <int NP>
__device__ __forceinline__ void ray_intervals(const Prims<NP>& P, V3 o, V3 d, RayIv<NP>& iv) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        iv.a[i] = INFINITY;
        iv.b[i] = -INFINITY;
        float t0, t1;
        if (i < P.n && prim_interval(P.p[i], o, d, t0, t1)) {
            iv.a[i] = t0;
            iv.b[i] = t1;
        }
    }
}

// The connected piece [s, e] of the union of primitive intervals that
// contains t or starts first after it; false if the ray leaves for good.
template <int NP>
__device__ __forceinline__ bool union_piece(const RayIv<NP>& iv, float t, float& s, float& e) {
    s = INFINITY;
#pragma unroll
    for (int i = 0; i < NP; ++i)
        if (iv.b[i] > t) s = __builtin_fminf(s, __builtin_fmaxf(iv.a[i], t));
    if (s == INFINITY) return false;
    e = s;
#pragma unroll
    for (int pass = 0; pass < NP; ++pass)
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (iv.a[i] <= e && iv.b[i] > e) e = iv.b[i];
    return true;
}

// Signed distance of one primitive where it is negative (p inside); outside
// only its sign is kept (a box returns its largest axis excess, a lower
// bound of the distance).  The union radius only reads the most negative
// value, so it equals the one from the exact distances.
__device__ __forceinline__ float prim_depth(const float* pr, V3 p) {
    const V3 q = v3(p.x - pr[1], p.y - pr[2], p.z - pr[3]);
    if (pr[0] == 0.0f) return fast_sqrt(dot(q, q)) - pr[4];
    const float ex = __builtin_fabsf(q.x) - pr[4], ey = __builtin_fabsf(q.y) - pr[5], ez = __builtin_fabsf(q.z) - pr[6];
    return __builtin_fmaxf(ex, __builtin_fmaxf(ey, ez));
}

__device__ __forceinline__ float fp16_value(uint16_t h) {
    return (float)__builtin_bit_cast(_Float16, h);
}

// Radius of a sphere around p inside the body (see the C header): the
// nearest grid voxel's distance minus half a voxel diagonal ...
__device__ __forceinline__ float grid_radius(const RenderArgs& A, V3 p) {
    const float fx = (p.x - A.grid_lo[0]) * A.grid_inv_h[0];
    const float fy = (p.y - A.grid_lo[1]) * A.grid_inv_h[1];
    const float fz = (p.z - A.grid_lo[2]) * A.grid_inv_h[2];
    const float fr = (float)A.res;
    if (!(fx >= 0.0f && fy >= 0.0f && fz >= 0.0f && fx < fr && fy < fr && fz < fr)) return 0.0f;
    const int64_t ix = (int64_t)fx, iy = (int64_t)fy, iz = (int64_t)fz;
    const float s = fp16_value(A.grid[(iz * A.res + iy) * A.res + ix]);
    return __builtin_fmaxf(0.0f, -s - A.grid_half_diag);
}

// ... or, without a grid, the analytic union distance shrunk by 0.1 %.
__device__ __forceinline__ float union_radius(float s) { return s < 0.0f ? -0.999f * s : 0.0f; }

// Point-light next-event estimate at x for a path travelling along d:
// I rho_g(d . w_{x->L}) exp(-sigma_t d_t) / |x_L - x|^2 (Sec. 4.3).
template <int NP>
__device__ __forceinline__ float nee(const RenderArgs& A, const Prims<NP>& P, V3 x, V3 d) {
    V3 wl = v3(A.light[0] - x.x, A.light[1] - x.y, A.light[2] - x.z);
    const float dist2 = dot(wl, wl);
    const float inv_dist = fast_rsq(dist2);
    const float dist = dist2 * inv_dist;
    wl = inv_dist * wl;
    RayIv<NP> iv;
    ray_intervals(P, x, wl, iv);
    float acc = 0.0f, t = 0.0f;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        float s, e;
        if (t < dist && union_piece(iv, t, s, e) && s < dist) {
            acc += __builtin_fminf(e, dist) - s;
            t = e;
        } else {
            t = dist;
        }
    }
    return A.intensity * hg_eval(A.g, dot(d, wl)) * fast_exp(-A.sigma_t * acc) * (inv_dist * inv_dist);
}

// ---------------------------------------------------------------- geometry policies

// Few primitives (NP <= 4) in registers; the intervals of the current ray
// are computed once per ray and kept in registers.
template <int NP, bool GRID>
struct Geo {
    static constexpr bool kWaveLight = false;  // shadow rays tested per lane (few primitives)
    Prims<NP> P;
    RayIv<NP> iv;
    __device__ __forceinline__ void init(const RenderArgs& A, const float*) {
        P.n = A.n_prims;
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int k = 0; k < 8; ++k) P.p[i][k] = i < A.n_prims ? A.prims[i * 8 + k] : 0.0f;
    }
    __device__ __forceinline__ void set_ray(V3 o, V3 d) { ray_intervals(P, o, d, iv); }
    __device__ __forceinline__ void set_camera_ray(V3 o, V3 d) { ray_intervals(P, o, d, iv); }
    __device__ __forceinline__ bool piece(V3, V3, float t, float& s, float& e) const { return union_piece(iv, t, s, e); }
    __device__ __forceinline__ float radius(const RenderArgs& A, V3 p) const {
        if (GRID) return grid_radius(A, p);
        float s = INFINITY;
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (i < P.n) s = __builtin_fminf(s, prim_depth(P.p[i], p));
        return union_radius(s);
    }
    // An upper bound of radius() over the whole scene: union_radius of the
    // deepest point of the deepest primitive (a sphere's centre at depth r, a
    // box's at its smallest half size), in the same rounding; unbounded with
    // a grid.
    __device__ __forceinline__ float max_radius() const {
        if (GRID) return INFINITY;
        float m = 0.0f;
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (i < P.n)
                m = __builtin_fmaxf(m, P.p[i][0] == 0.0f ? P.p[i][4]
                                                         : __builtin_fminf(P.p[i][4], __builtin_fminf(P.p[i][5], P.p[i][6])));
        return union_radius(-m);
    }
    __device__ __forceinline__ float flight_bound(const RenderArgs&, V3) const { return 0.0f; }
    __device__ __forceinline__ float light(const RenderArgs& A, V3 x, V3 d) const { return nee(A, P, x, d); }
};

// Many primitives (up to kMaxManyPrims) staged in LDS; ray intervals are
// recomputed on demand, the hits of one query kept in registers (8 slots).
// A flight shorter than the conservative radius at its start cannot leave
// the body, so it needs no exact boundary query.
constexpr int kMaxManyPrims = 256;
constexpr int kHitSlots = 8;

template <bool GRID>
struct GeoMany {
    // shadow rays of a wave share a primitive mask (light_mask below)
    static constexpr bool kWaveLight = true;
    const float* prim;  // LDS [n][8]
    int n;
    __device__ __forceinline__ void init(const RenderArgs& A, const float* lds_prims) {
        prim = lds_prims;
        n = A.n_prims;
    }
    __device__ __forceinline__ void set_ray(V3, V3) {}
    __device__ __forceinline__ void set_camera_ray(V3, V3) {}
    __device__ __forceinline__ bool piece(V3 o, V3 d, float t, float& s, float& e) const {
        float ca[kHitSlots], cb[kHitSlots];
        int m = 0;
        bool overflow = false;
        s = INFINITY;
        for (int i = 0; i < n; ++i) {
            float a, b;
            if (prim_interval(prim + 8 * i, o, d, a, b) && b > t) {
                s = __builtin_fminf(s, __builtin_fmaxf(a, t));
#pragma unroll
                for (int j = 0; j < kHitSlots; ++j)
                    if (j == m) {
                        ca[j] = a;
                        cb[j] = b;
                    }
                if (m < kHitSlots) ++m;
                else overflow = true;
            }
        }
        if (s == INFINITY) return false;
        e = s;
        if (!overflow) {
#pragma unroll
            for (int pass = 0; pass < kHitSlots; ++pass)
#pragma unroll
                for (int j = 0; j < kHitSlots; ++j)
                    if (j < m && ca[j] <= e && cb[j] > e) e = cb[j];
        } else {
            for (int pass = 0; pass < n; ++pass) {
                bool grew = false;
                for (int i = 0; i < n; ++i) {
                    float a, b;
                    if (prim_interval(prim + 8 * i, o, d, a, b) && a <= e && b > e) {
                        e = b;
                        grew = true;
                    }
                }
                if (!grew) break;
            }
        }
        return true;
    }
    __device__ __forceinline__ float radius(const RenderArgs& A, V3 p) const {
        if (GRID) return grid_radius(A, p);
        float sd = INFINITY;
        for (int i = 0; i < n; ++i) sd = __builtin_fminf(sd, prim_depth(prim + 8 * i, p));
        return union_radius(sd);
    }
    __device__ __forceinline__ float flight_bound(const RenderArgs& A, V3 p) const { return radius(A, p); }
    __device__ __forceinline__ float max_radius() const { return INFINITY; }

    // Primitives the shadow segments of this wave can meet.  Called by every
    // lane of the wave (converged); lanes with `active` will trace a segment
    // from x to the light.  All segments lie in the union of balls around the
    // axis from the centre C of the origins' bounding box to the light with
    // radius rho (the box's half diagonal), so a primitive whose bounding
    // sphere stays farther than rho from that axis segment meets none of them
    // and is left out of the wave's mask (bit i of word i / 64); the mask
    // only drops primitives that cannot contribute, so the result is the
    // one of testing them all.
    __device__ __forceinline__ void light_mask(const RenderArgs& A, bool active, V3 x, uint64_t* mask) const {
        float lo0 = active ? x.x : INFINITY, lo1 = active ? x.y : INFINITY, lo2 = active ? x.z : INFINITY;
        float hi0 = active ? x.x : -INFINITY, hi1 = active ? x.y : -INFINITY, hi2 = active ? x.z : -INFINITY;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            lo0 = __builtin_fminf(lo0, __shfl_xor(lo0, off));
            lo1 = __builtin_fminf(lo1, __shfl_xor(lo1, off));
            lo2 = __builtin_fminf(lo2, __shfl_xor(lo2, off));
            hi0 = __builtin_fmaxf(hi0, __shfl_xor(hi0, off));
            hi1 = __builtin_fmaxf(hi1, __shfl_xor(hi1, off));
            hi2 = __builtin_fmaxf(hi2, __shfl_xor(hi2, off));
        }
        const V3 c = v3(0.5f * (lo0 + hi0), 0.5f * (lo1 + hi1), 0.5f * (lo2 + hi2));
        const V3 half = v3(0.5f * (hi0 - lo0), 0.5f * (hi1 - lo1), 0.5f * (hi2 - lo2));
        const float rho = __builtin_sqrtf(dot(half, half));
        const V3 u = v3(A.light[0] - c.x, A.light[1] - c.y, A.light[2] - c.z);
        const float uu = dot(u, u);
        const float inv_uu = uu > 0.0f ? 1.0f / uu : 0.0f;
#pragma unroll
        for (int k = 0; k < kMaxManyPrims / 64; ++k) {
            const int i = 64 * k + lane_id();
            bool keep = false;
            if (i < n) {
                const float* pr = prim + 8 * i;
                const V3 q = v3(pr[1] - c.x, pr[2] - c.y, pr[3] - c.z);
                const float tt = __builtin_fminf(1.0f, __builtin_fmaxf(0.0f, dot(q, u) * inv_uu));
                const V3 off = q - tt * u;
                const float br = pr[0] == 0.0f ? pr[4] : __builtin_sqrtf(pr[4] * pr[4] + pr[5] * pr[5] + pr[6] * pr[6]);
                // widened by a relative 1e-4 against rounding
                const float reach = (rho + br) * 1.0001f + 1e-4f * (__builtin_fabsf(tt) + 1.0f) * __builtin_sqrtf(uu);
                keep = dot(off, off) <= reach * reach;
            }
            mask[k] = ballot(keep && active_any(lo0));
        }
    }
    __device__ __forceinline__ static bool active_any(float lo0) { return lo0 != INFINITY; }

    // Shadow ray: the primitives (all of them, or those of a wave mask)
    // contribute their hit intervals clipped to [0, dist] (8 slots), a
    // sorting network orders them by entry and a sweep adds the length of
    // their union; more than 8 hits falls back to piece-by-piece queries.
    __device__ __forceinline__ float light(const RenderArgs& A, V3 x, V3 d) const { return light_masked(A, x, d, nullptr); }
    __device__ __forceinline__ float light_masked(const RenderArgs& A, V3 x, V3 d, const uint64_t* mask) const {
        V3 wl = v3(A.light[0] - x.x, A.light[1] - x.y, A.light[2] - x.z);
        const float dist2 = dot(wl, wl);
        const float inv_dist = fast_rsq(dist2);
        const float dist = dist2 * inv_dist;
        wl = inv_dist * wl;
        float ca[kHitSlots], cb[kHitSlots];
#pragma unroll
        for (int j = 0; j < kHitSlots; ++j) {
            ca[j] = INFINITY;
            cb[j] = INFINITY;
        }
        int m = 0;
        auto visit = [&](int i) {
            float a, b;
            if (prim_interval(prim + 8 * i, x, wl, a, b) && b > 0.0f && a < dist) {
                a = __builtin_fmaxf(a, 0.0f);
                b = __builtin_fminf(b, dist);
#pragma unroll
                for (int j = 0; j < kHitSlots; ++j)
                    if (j == m) {
                        ca[j] = a;
                        cb[j] = b;
                    }
                ++m;
            }
        };
        if (mask == nullptr) {
            for (int i = 0; i < n; ++i) visit(i);
        } else {
            for (int k = 0; k < kMaxManyPrims / 64; ++k)
                for (uint64_t bits = mask[k]; bits != 0; bits &= bits - 1) visit(64 * k + __builtin_ctzll(bits));
        }
        float acc = 0.0f;
        if (m <= kHitSlots) {
            // odd-even transposition sort of the (entry, exit) pairs by entry
#pragma unroll
            for (int pass = 0; pass < kHitSlots; ++pass)
#pragma unroll
                for (int j = pass & 1; j + 1 < kHitSlots; j += 2) {
                    const bool sw = ca[j + 1] < ca[j];
                    const float ta = sw ? ca[j + 1] : ca[j], tb = sw ? cb[j + 1] : cb[j];
                    const float ua = sw ? ca[j] : ca[j + 1], ub = sw ? cb[j] : cb[j + 1];
                    ca[j] = ta;
                    cb[j] = tb;
                    ca[j + 1] = ua;
                    cb[j + 1] = ub;
                }
            float s0 = ca[0], e0 = cb[0];
#pragma unroll
            for (int j = 1; j < kHitSlots; ++j) {
                if (j < m) {
                    if (ca[j] <= e0) {
                        e0 = __builtin_fmaxf(e0, cb[j]);
                    } else {
                        acc += e0 - s0;
                        s0 = ca[j];
                        e0 = cb[j];
                    }
                }
            }
            if (m > 0) acc += e0 - s0;
        } else {
            float t = 0.0f;
            for (int k = 0; k < n && t < dist; ++k) {
                float ps, pe;
                if (!piece(x, wl, t, ps, pe) || ps >= dist) break;
                acc += __builtin_fminf(pe, dist) - ps;
                t = pe;
            }
        }
        return A.intensity * hg_eval(A.g, dot(d, wl)) * fast_exp(-A.sigma_t * acc) * (inv_dist * inv_dist);
    }
};

// A closed triangle mesh: the crossings ahead of each new ray's origin (BVH
// traversal of the half-line) alternate exit / entry from a scattering
// point inside the body and entry / exit from the camera; up to four medium
// intervals are kept in registers.  Radii come from the distance grid;
// shadow rays traverse their own segment to the light.
struct GeoMesh {
    static constexpr bool kWaveLight = false;  // shadow rays traverse the BVH per lane
    const BvhNode* nodes;
    const float* tris;
    int n_nodes;
    RayIv<4> iv;
    __device__ __forceinline__ void init(const RenderArgs& A, const float*) {
        nodes = A.bvh;
        tris = A.tris;
        n_nodes = A.n_nodes;
    }
    __device__ __forceinline__ void set_ray(V3 o, V3 d) { set_ray_from(o, d, true); }
    __device__ __forceinline__ void set_camera_ray(V3 o, V3 d) { set_ray_from(o, d, false); }
    __device__ __forceinline__ void set_ray_from(V3 o, V3 d, bool inside) {
        float c[kMeshCross];
        const int m = mesh_crossings(nodes, n_nodes, tris, o, d, 0.0f, INFINITY, c);
        // inside: (-inf, c0), (c1, c2), (c3, c4), ...; outside: (c0, c1), (c2, c3), ...
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float a_in = k == 0 ? -INFINITY : c[2 * k - 1];
            const bool ok = inside ? 2 * k < m : 2 * k + 1 < m;
            iv.a[k] = ok ? (inside ? a_in : c[2 * k]) : INFINITY;
            iv.b[k] = ok ? (inside ? c[2 * k] : c[2 * k + 1]) : -INFINITY;
        }
    }
    __device__ __forceinline__ bool piece(V3, V3, float t, float& s, float& e) const { return union_piece(iv, t, s, e); }
    __device__ __forceinline__ float radius(const RenderArgs& A, V3 p) const { return grid_radius(A, p); }
    __device__ __forceinline__ float max_radius() const { return INFINITY; }
    __device__ __forceinline__ float flight_bound(const RenderArgs&, V3) const { return 0.0f; }

    __device__ __forceinline__ float light(const RenderArgs& A, V3 x, V3 d) const {
        V3 wl = v3(A.light[0] - x.x, A.light[1] - x.y, A.light[2] - x.z);
        const float dist2 = dot(wl, wl);
        const float inv_dist = fast_rsq(dist2);
        const float dist = dist2 * inv_dist;
        wl = inv_dist * wl;
        float c[kMeshCross];
        const int m = mesh_crossings(nodes, n_nodes, tris, x, wl, 0.0f, dist, c);
        // x is inside: inside until c[0], outside until c[1], ...
        float acc = 0.0f, prev = 0.0f;
#pragma unroll
        for (int k = 0; k < kMeshCross; ++k)
            if (k < m) {
                if ((k & 1) == 0) acc += c[k] - prev;
                prev = c[k];
            }
        if ((m & 1) == 0) acc += dist - prev;
        return A.intensity * hg_eval(A.g, dot(d, wl)) * fast_exp(-A.sigma_t * acc) * (inv_dist * inv_dist);
    }
};
constexpr int kGeoMesh = 8;  // render_kernel template tag of mesh scenes

// Geometry policy of a kernel instance; GRID fixes the radius source at
// compile time (a mesh always has its grid).
template <int NP, bool GRID>
struct GeoSel {
    typedef Geo<NP, GRID> type;
};
template <bool GRID>
struct GeoSel<kGeoMesh, GRID> {
    typedef GeoMesh type;
};
template <bool GRID>
struct GeoSel<0, GRID> {
    typedef GeoMany<GRID> type;
};

// ---------------------------------------------------------------- kernel

__device__ __forceinline__ void neumaier_add(float& sum, float& comp, float v) {
    const float t = sum + v;
    if (__builtin_fabsf(sum) >= __builtin_fabsf(v)) comp += (sum - t) + v;
    else comp += (v - t) + sum;
    sum = t;
}

// e^x - 1 and 1 - e^-x for x >= 0 without cancellation: below 1/64 a
// four-term Taylor series (relative truncation below x^4 / 120), above it
// the exponential.
__device__ __forceinline__ float exp_minus_one(float x) {
    if (x < 0.015625f) return x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f))));
    return fast_exp(x) - 1.0f;
}
__device__ __forceinline__ float one_minus_exp_neg(float x) {
    if (x < 0.015625f) return x * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f))));
    return 1.0f - fast_exp(-x);
}

// Lambda^(N) = Sum_{i<=N} albedo^i = albedo (1 - albedo^N) / (1 - albedo),
// bounded by albedo / (1 - albedo) for any N.
__device__ __forceinline__ float lambda_total(const RenderArgs& A, float N) {
    if (A.albedo >= 1.0f) return N;
    return fast_div(A.albedo * one_minus_exp_neg(-N * A.ln_albedo), 1.0f - A.albedo);
}

// Lambda^(N) / albedo^N = albedo (albedo^-N - 1) / (1 - albedo), the weight
// of a surviving step; it only matters while albedo^N >= 2^-24 (a survivor),
// so the exponent is capped where it would overflow.
__device__ __forceinline__ float lambda_weight(const RenderArgs& A, float N) {
    if (A.albedo >= 1.0f) return N;
    return fast_div(A.albedo * exp_minus_one(__builtin_fminf(80.0f, -N * A.ln_albedo)), 1.0f - A.albedo);
}

// Writes this lane's part of its decoder input row -- the standardised
// condition after `latent` slots, zero padding -- and the Philox stream and
// first block of its normals; advances the lane's block counter past them.
template <int PO, int PI>
__device__ __forceinline__ void stage_row(const PackedModel* pm, RenderLds& L, int slot, const Rng& rng,
                                          uint32_t& c0, const float* cond) {
    const int lat = pm->latent;
    float* row = L.x[slot];
#pragma unroll
    for (int k = 0; k < PI; ++k) row[lat + k] = (cond[k] - pm->mean_c[k]) * pm->inv_std_c[k];
    for (int q = lat + PI; q < kTile; ++q) row[q] = 0.0f;
    L.rid[slot] = make_uint4(rng.id_lo, rng.id_hi, c0, 0u);
    c0 += (uint32_t)((lat + PO + 3) >> 2);
}

// floor(n / d) for n < 2^32: the double-precision quotient through the
// rounded reciprocal is within one of it (relative error 2^-52), and one
// integer check makes it exact -- a few instructions instead of the long
// integer division sequence.
__device__ __forceinline__ uint32_t udiv_exact(uint32_t n, uint32_t d, double inv_d) {
    uint32_t q = (uint32_t)((double)n * inv_d);
    const int64_t r = (int64_t)n - (int64_t)q * (int64_t)d;
    if (r < 0) --q;
    else if (r >= (int64_t)d) ++q;
    return q;
}

// q / nb for q < 2^15 and nb in 1 .. 4.
__device__ __forceinline__ int div_small(int q, int nb) {
    return nb == 1 ? q : nb == 2 ? q >> 1 : nb == 4 ? q >> 2 : (q * 0xAAAB) >> 17;
}

// The normals of the n staged rows, drawn by the whole wave: row s needs
// blocks rid[s].z .. rid[s].z + nb - 1 of its own Philox stream; the
// (row, block) tasks are spread over the 64 lanes.  Box-Muller pairs give
// four normals per block: the first `latent` are the row's z, the next PO its
// posterior noise -- the same values, in the same order, as if each lane drew
// its own.
template <int PO>
__device__ __forceinline__ void stage_normals(const RenderArgs& A, const PackedModel* pm, RenderLds& L, int n) {
    wave_sync();
    const int lat = pm->latent, n_norm = lat + PO, nb = (n_norm + 3) >> 2;
    const int total = n * nb;
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    for (int task = lane_id(); task < total; task += 64) {
        const int slot = div_small(task, nb);
        const int j = task - slot * nb;
        const uint4 r = L.rid[slot];
        const uint4 w = philox(r.z + (uint32_t)j, r.x, r.y, MS_TAG_RENDER_PATH, k0, k1);
        float nv[4];
        box_muller(u01(w.x), u01(w.y), nv[0], nv[1]);
        box_muller(u01(w.z), u01(w.w), nv[2], nv[3]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 4 * j + q;
            if (i < lat)
                L.x[slot][i] = nv[q];
            else if (i < n_norm)
                L.eps[slot][i - lat] = nv[q];
        }
    }
}

// Runs one decoder over the first n compacted rows (16-path MFMA tiles);
// each row's (mean, log variance) outputs overwrite its inputs.
__device__ __forceinline__ void decode_tiles(const PackedModel* pm, RenderLds& L, int n) {
    wave_sync();
    const int n_tiles = (n + 15) >> 4;
    if (pm->n_linear == kDecLayers) {
        const DecoderRegs w = load_decoder(pm);
        const bool fp8 = pm->precision == MS_PREC_FP8;
        for (int t = 0; t < n_tiles; ++t) {
            const int path = 16 * t + frag_row();
            const f32x4 xin = *reinterpret_cast<const f32x4*>(&L.x[path][frag_k0()]);
            // each lane rewrites exactly the 16 bytes it read (B and D layouts coincide)
            const f32x4 o = fp8 ? decoder_tile_fp8(w, xin) : decoder_tile(w, xin);
            *reinterpret_cast<f32x4*>(&L.x[path][frag_k0()]) = o;
        }
    } else {
        for (int t = 0; t < n_tiles; ++t) {
            const int path = 16 * t + frag_row();
            const f32x4 xin = *reinterpret_cast<const f32x4*>(&L.x[path][frag_k0()]);
            *reinterpret_cast<f32x4*>(&L.x[path][frag_k0()]) = decoder_tile_layers(pm, xin);
        }
    }
    wave_sync();
}

// The de-standardised sample y[0..PO) of decoded row `slot`:
// mu + exp(log variance / 2) eps.
template <int PO>
__device__ __forceinline__ void read_row(const PackedModel* pm, const RenderLds& L, int slot, float* y) {
#pragma unroll
    for (int k = 0; k < PO; ++k) {
        const float mu = L.x[slot][k];
        const float lv = __builtin_fminf(8.0f, __builtin_fmaxf(-12.0f, L.x[slot][PO + k]));
        const float ys = __builtin_fmaf(fast_exp(0.5f * lv), L.eps[slot][k], mu);
        y[k] = __builtin_fmaf(ys, pm->std_y[k], pm->mean_y[k]);
    }
}

// decode_tiles, then the sample of row `slot` for lanes that staged one.
template <int PO>
__device__ __forceinline__ void decode_rows(const PackedModel* pm, RenderLds& L, bool mine, int slot, int n,
                                            float* y) {
    decode_tiles(pm, L, n);
    if (mine) read_row<PO>(pm, L, slot, y);
    wave_sync();
}

// Exclusive prefix sum over the wave of small per-lane counts (< 2^5) and
// their total.
__device__ __forceinline__ int wave_prefix_small(int cnt, int& total) {
    int pre = 0;
    total = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        const uint64_t m = ballot((cnt >> b) & 1);
        pre += rank_in(m) << b;
        total += __popcll(m) << b;
    }
    return pre;
}

// The persistent render loop of one kernel instance (MODE fixes the
// method); the whole body of render_kernel below.  A lane traces the
// samples of its work unit one after the other and banks them in order.
template <int MODE, int NP, bool GRID>
__device__ __forceinline__ void render_loop(const RenderArgs& A, RenderLds& L, const float* lds_prims,
                                            uint32_t (*tot)[64 * kRenderWaves]) {
    typename GeoSel<NP, GRID>::type G;
    constexpr bool kWaveLight = GeoSel<NP, GRID>::type::kWaveLight;
    G.init(A, lds_prims);

    TicketPool pool;
    pool.reset();
    int state = S_NEED;
    // current path
    Rng rng = make_rng(A.seed, MS_TAG_RENDER_PATH, 0);
    V3 o = v3(0, 0, 0), d = v3(0, 0, 1);
    float t = 0.0f, Lp = 0.0f, r_step = 0.0f;
    uint32_t c0 = 0, p_ev = 0, p_st = 0;
    // iterations for which lanes have been waiting for a restart / a learned
    // step (wave-uniform): a pass also runs once the oldest wait reaches
    // max_wait, so rare steps do not idle lanes for long
    int end_age = 0, wait_age = 0;
    // The lane's work unit (its accumulators, next sample, end of range and
    // index; U_NONE when it has none) and its totals of events, learned
    // steps and truncated paths for the launch counters live in LDS: touched
    // once per sample or per unit, they would otherwise hold registers
    // through the collision and decoder loops
    const int tid = threadIdx.x;
    for (int q = 0; q < kLaneWords; ++q) tot[q][tid] = 0;
    tot[U_UNIT][tid] = U_NONE;

    auto start_path = [&](uint32_t pixel, int q) __attribute__((always_inline)) {
        const int py = (int)udiv_exact(pixel, (uint32_t)A.width, A.inv_width);
        const int px = (int)pixel - py * A.width;
        const uint64_t sample = A.sample_offset + (uint64_t)q;
        const uint64_t id = (uint64_t)pixel | (sample << 32);
        const Rng rp = make_rng(A.seed, MS_TAG_RENDER_PIXEL, id);
        const uint4 jw = rp.block(0);
        rng = make_rng(A.seed, MS_TAG_RENDER_PATH, id);
        const float sx = 2.0f * ((float)px + u01(jw.x)) / (float)A.width - 1.0f;
        const float sy = 1.0f - 2.0f * ((float)py + u01(jw.y)) / (float)A.height;
        o = v3(A.eye[0], A.eye[1], A.eye[2]);
        d = normalize(v3(A.fwd[0] + sx * A.right[0] + sy * A.upv[0], A.fwd[1] + sx * A.right[1] + sy * A.upv[1],
                         A.fwd[2] + sx * A.right[2] + sy * A.upv[2]));
        G.set_camera_ray(o, d);
        t = 0.0f;
        Lp = 0.0f;
        c0 = 0;
        p_ev = 0;
        p_st = 0;
        state = S_FLY;
    };

    // ---- restart phase, batched: lanes whose path ended bank it, lanes out
    // of samples take a work unit, then every lane with a sample to trace
    // starts its camera ray.  It runs once restart_min lanes wait, or nothing
    // else is in flight, or the oldest wait reaches max_wait, so that its
    // code is not issued for a handful of lanes on most iterations.
    auto restart_now = [&]() __attribute__((always_inline)) -> bool {
        const uint64_t rmask = ballot(state == S_END || state == S_NEED);
        const uint64_t amask = ballot(state == S_FLY || state == S_WAIT);
        end_age = rmask != 0 ? end_age + 1 : 0;
        return rmask != 0 && (__popcll(rmask) >= A.restart_min || amask == 0 || end_age > A.max_wait);
    };
    auto restart = [&]() __attribute__((always_inline)) {
        end_age = 0;
        bool start = false;
        int s_next = 0;
        if (state == S_END) {
            float acc_sum = __uint_as_float(tot[U_SUM][tid]), acc_comp = __uint_as_float(tot[U_COMP][tid]);
            neumaier_add(acc_sum, acc_comp, Lp);
            const float acc_sq = __builtin_fmaf(Lp, Lp, __uint_as_float(tot[U_SQ][tid]));
            const uint32_t acc_ev = tot[U_EV][tid] + p_ev, acc_st = tot[U_ST][tid] + p_st;
            s_next = (int)tot[U_NEXT][tid];
            if (s_next < (int)tot[U_END][tid]) {
                tot[U_SUM][tid] = __float_as_uint(acc_sum);
                tot[U_COMP][tid] = __float_as_uint(acc_comp);
                tot[U_SQ][tid] = __float_as_uint(acc_sq);
                tot[U_EV][tid] = acc_ev;
                tot[U_ST][tid] = acc_st;
                start = true;
            } else {
                // the unit's last sample: its record
                UnitRecord rec;
                rec.sum = acc_sum + acc_comp;
                rec.sumsq = acc_sq;
                rec.events = acc_ev;
                rec.steps = acc_st;
                A.part[tot[U_UNIT][tid]] = rec;
                tot[T_EVENTS][tid] += acc_ev;
                tot[T_STEPS][tid] += acc_st;
                tot[U_UNIT][tid] = U_NONE;
            }
            state = S_NEED;
        }
        const bool need = state == S_NEED && tot[U_UNIT][tid] == U_NONE;
        const uint64_t tk = pool.take(need, A.ticket, 64);
        if (need) {
            if (tk < (uint64_t)A.n_units) {
                tot[U_UNIT][tid] = (uint32_t)tk;
                // pixel-major: a wave's block of tickets covers few pixels
                const uint32_t pixel = udiv_exact((uint32_t)tk, (uint32_t)A.n_chunks, A.inv_n_chunks);
                const int ch = (int)((uint32_t)tk - pixel * (uint32_t)A.n_chunks);
                s_next = ch * A.chunk;
                tot[U_END][tid] = (uint32_t)(s_next + A.chunk < A.spp ? s_next + A.chunk : A.spp);
                tot[U_SUM][tid] = tot[U_COMP][tid] = tot[U_SQ][tid] = 0u;
                tot[U_EV][tid] = tot[U_ST][tid] = 0u;
                start = true;
            } else {
                state = S_DONE;
            }
        }
        if (start) {
            const uint32_t unit = tot[U_UNIT][tid];
            start_path(udiv_exact(unit, (uint32_t)A.n_chunks, A.inv_n_chunks), s_next);
            tot[U_NEXT][tid] = (uint32_t)(s_next + 1);
        }
    };

    // ---- VALU phase: one flight, and at a collision a plain event or the
    // start of a learned step, for every lane in flight
    auto collide = [&](bool& path_end, bool& truncated) __attribute__((always_inline)) {
        // many primitives: a plain event's shadow ray is traced after the
        // branch, where the whole wave builds its primitive mask
        bool nee_now = false;
        V3 nee_x = v3(0, 0, 0), nee_d = v3(0, 0, 1);
        if (state == S_FLY) {
            // one Philox block per flight; the boundary query (the medium
            // piece of the ray containing or following t) is skipped when the
            // flight is shorter than the conservative radius at its start
            const uint4 w = rng.block(c0++);
            const float l = -flight_ln(u01(w.x)) * A.inv_sigma_t;
            float ps = t, pe = INFINITY;
            bool inside = l < G.flight_bound(A, fma3(t, d, o));
            if (!inside && !G.piece(o, d, t, ps, pe)) {
                path_end = true;
            } else {
                t = __builtin_fmaxf(t, ps);
                if (t + l >= pe) {
                    t = pe;
                } else {
                    t += l;
                    const V3 p = fma3(t, d, o);
                    // every collision is a plain event or a learned step, so
                    // p_ev + p_st counts the path's collisions so far
                    if (p_ev + p_st >= A.max_events) {
                        path_end = true;
                        truncated = true;
                    } else {
                        bool plain = true;
                        if (MODE != kModePlain) {
                            const float r = __builtin_fminf(G.radius(A, p), A.st_max * A.inv_sigma_t);
                            if (A.sigma_t * r >= A.tau_min) {
                                plain = false;
                                if (MODE == kModeStExact) {
                                    // the actual walk inside the sphere (reference sampler)
                                    V3 x = p, dir = d, Xk = p, Wk = d;
                                    float resv = 0.0f;
                                    const float r2 = r * r;
                                    const float inv_phi = 1.0f / A.albedo;
                                    uint32_t nev = 0;
                                    for (;;) {
                                        // the path's max_events counts the step as one collision;
                                        // the walk inside the sphere has a bound of its own, reached
                                        // only with degenerate input
                                        if (++nev > kInnerWalkBound) break;
                                        const uint4 ww = rng.block(c0++);
                                        resv = nev == 1 ? 1.0f : __builtin_fmaf(resv, inv_phi, 1.0f);
                                        if (u01(ww.w) * resv <= 1.0f) {
                                            Xk = x;
                                            Wk = dir;
                                        }
                                        const HgSample h = hg_sample(A.g, u01(ww.y));
                                        dir = scatter(dir, h.mu, h.sin_t, u01(ww.z));
                                        const float ll = -flight_ln(u01(ww.x)) * A.inv_sigma_t;
                                        const V3 rel = x - p;
                                        const V3 qn = fma3(ll, dir, rel);
                                        if (!(dot(qn, qn) < r2)) {
                                            x = fma3(sphere_exit(rel, dir, r2), dir, x);
                                            break;
                                        }
                                        x = fma3(ll, dir, x);
                                    }
                                    ++p_st;
                                    const uint4 wa = rng.block(c0++);
                                    const float N = (float)nev;
                                    if (!(u01(wa.x) <= fast_exp(N * A.ln_albedo))) {
                                        path_end = true;
                                    } else {
                                        Lp += lambda_weight(A, N) * G.light(A, Xk, Wk);
                                        o = x;
                                        d = dir;
                                        G.set_ray(o, d);
                                        t = 0.0f;
                                    }
                                } else {
                                    o = p;
                                    r_step = r;
                                    state = S_WAIT;
                                }
                            }
                        }
                        if (plain) {
                            ++p_ev;
                            if constexpr (kWaveLight) {
                                nee_now = true;
                                nee_x = p;
                                nee_d = d;
                            } else {
                                Lp += A.albedo * G.light(A, p, d);
                            }
                            if (u24(w.w) > A.surv_thr) {
                                path_end = true;
                            } else {
                                const HgSample h = hg_sample(A.g, u01(w.y));
                                d = scatter(d, h.mu, h.sin_t, u01(w.z));
                                o = p;
                                G.set_ray(o, d);
                                t = 0.0f;
                            }
                        }
                    }
                }
            }
        }

        if constexpr (kWaveLight) {
            uint64_t mk[kMaxManyPrims / 64];
            G.light_mask(A, nee_now, nee_x, mk);
            if (nee_now) Lp += A.albedo * G.light_masked(A, nee_x, nee_d, mk);
        }
    };

    // ---- MFMA phase: one learned sphere step for every lane with `mine`
    // (wmask = ballot(mine)), on the path state passed in: position po (the
    // collision, the sphere's centre), direction pd, radius pr, Philox stream
    // prng at block pc0, radiance pLp, step count pst.  Returns whether the
    // path survives the step; a survivor's po, pd become the exit point and
    // direction.
    auto learned_core = [&](uint64_t wmask, bool mine, V3& po, V3& pd, float pr, const Rng& prng, uint32_t& pc0,
                            float& pLp, uint32_t& pst) __attribute__((always_inline)) -> bool {
        const int n_wait = __popcll(wmask);
        float y[6];
        float N = 1.0f, psi = 0.0f;
        const float lst = fast_ln(A.sigma_t * pr);
        // LengthGen (sigma_t r, g) -> N
        const int slot0 = rank_in(wmask);
        if (mine) {
            const float c2[2] = {lst, A.g};
            stage_row<1, 2>(A.pm[0], L, slot0, prng, pc0, c2);
        }
        stage_normals<1>(A, A.pm[0], L, n_wait);
        decode_rows<1>(A.pm[0], L, mine, slot0, n_wait, y);
        bool alive = false;
        float u_hg = 0.5f, u_first = 1.0f, phiN = 1.0f;
        if (mine) {
            ++pst;
            N = __builtin_fmaxf(1.0f, floorf(fast_exp(__builtin_fminf(y[0], 20.0f)) + 0.5f));
            const uint4 wa = prng.block(pc0++);
            psi = u01(wa.y);
            u_hg = u01(wa.z);
            u_first = u01(wa.w);
            // absorption along the bypassed chain (Sec. 3.2)
            phiN = fast_exp(N * A.ln_albedo);
            alive = u01(wa.x) <= phiN;
        }
        // N = 1: a single HG scatter at the centre, sampled exactly;
        // N >= 2: PathGen, then each representative event is the centre
        // with probability albedo / Lambda^(N), else EventGen.  With
        // NEE before absorption the direct light of the step is
        // estimated for every step (weight Lambda) and the absorption
        // only ends the path; otherwise only surviving steps add it
        // (weight Lambda / albedo^N, the order of Sec. 3.2).  The paper's
        // step as printed (MS_RENDER_STEP_PAPER) asks PathGen and EventGen
        // in every case; the HG and first-event uniforms are then drawn and
        // left unused, so both forms keep the same draw order.
        const bool before = (A.flags & MS_RENDER_NEE_BEFORE_ABSORPTION) != 0;
        const bool paper = (A.flags & MS_RENDER_STEP_PAPER) != 0;
        const bool lit = before ? mine : alive;
        const bool use_path = lit && (N >= 2.0f || paper);
        // Lambda and Lambda / albedo^N each in a form that stays finite
        // for any N (their product form overflows once albedo^-N does)
        const float lam = lambda_total(A, N);
        // this step's representative events: nee_samples, or with nee_chain
        // one more per nee_chain events of the chain, up to nee_samples (an
        // integer rule on N, so that the draws follow N alone): event k > 0
        // exists iff N - 1 >= k nee_chain
        auto events_of = [&](float n) __attribute__((always_inline)) -> int {
            if (A.nee_chain <= 0) return A.nee_samples;
            const uint32_t more = ((uint32_t)n - 1u) / (uint32_t)A.nee_chain;
            return more + 1u < (uint32_t)A.nee_samples ? (int)more + 1 : A.nee_samples;
        };
        auto has_event = [&](int k) __attribute__((always_inline)) -> bool {
            return A.nee_chain <= 0 || k == 0 || (uint32_t)N - 1u >= (uint32_t)k * (uint32_t)A.nee_chain;
        };
        const float w_nee = (before ? lam : lambda_weight(A, N)) / (float)events_of(N);
        float ct = 0.0f, al = 0.0f, be = 0.0f, ga = 1.0f;
        if (lit && !use_path) ct = hg_sample(A.g, u_hg).mu;
        const uint64_t pmask = ballot(use_path);
        const float lnN = fast_ln(N);
        if (pmask) {
            const int row = rank_in(pmask);
            // PathGen (sigma_t r, g, N) -> (cos theta, alpha, beta)
            if (use_path) {
                const float c3[3] = {lst, A.g, lnN};
                stage_row<3, 3>(A.pm[1], L, row, prng, pc0, c3);
            }
            stage_normals<3>(A, A.pm[1], L, __popcll(pmask));
            decode_rows<3>(A.pm[1], L, use_path, row, __popcll(pmask), y);
            if (use_path) {
                ct = __builtin_fminf(1.0f, __builtin_fmaxf(-1.0f, y[0]));
                al = y[1];
                be = y[2];
                ga = fast_sqrt(__builtin_fmaxf(0.0f, 1.0f - al * al - be * be));
                const float inl = fast_rsq(al * al + be * be + ga * ga);
                al *= inl;
                be *= inl;
                ga *= inl;
            }
        }
        V3 e1 = v3(1, 0, 0), e2 = v3(0, 1, 0);
        float cp = 1.0f, sp = 0.0f;
        if (lit) {
            onb(pd, e1, e2);
            cp = cos_rev(psi);
            sp = sin_rev(psi);
        }
        // The step's representative events: event k's first-event test
        // draws a block (k > 0) and, where EventGen answers, its normals
        // follow; the EventGen rows of a group of events are decoded together
        // (a lane's rows consecutive), as many events per group as 64 rows
        // hold.  The groups run to the wave's largest event count.
        int k_all = A.nee_samples;
        if (A.nee_chain > 0) {
            float n_max = lit ? N : 1.0f;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) n_max = __builtin_fmaxf(n_max, __shfl_xor(n_max, off));
            // the same in every lane: a scalar loop bound
            k_all = __builtin_amdgcn_readfirstlane(events_of(n_max));
        }
        const int n_cand = __popcll(ballot(use_path));
        const int group = n_cand > 0 ? (64 / n_cand < 1 ? 1 : 64 / n_cand) : k_all;
        const int nb_ev = (A.pm[2]->latent + 6 + 3) >> 2;
        const float c7[7] = {lst, A.g, A.albedo, ct, al, be, lnN};
        for (int ka = 0; ka < k_all; ka += group) {
            const int kb = ka + group < k_all ? ka + group : k_all;
            // decisions and draw positions of the group's events
            // bit k - ka: event k asks EventGen; bit 16 + k - ka: event k is
            // one of this lit step's (a group holds at most 16 events)
            uint32_t evbits = 0;
            const uint32_t c0_group = pc0;
            for (int k = ka; k < kb; ++k) {
                const bool has = lit && has_event(k);
                float uf = u_first;
                if (k > 0 && has) uf = u01(prng.block(pc0++).x);
                if (has) evbits |= 1u << (16 + k - ka);
                if (use_path && has && (paper || !(uf * lam <= A.albedo))) {
                    evbits |= 1u << (k - ka);
                    pc0 += (uint32_t)nb_ev;
                }
            }
            int n_rows;
            const int base = wave_prefix_small(__popc(evbits & 0xFFFFu), n_rows);
            if (n_rows > 0) {
                // EventGen (sigma_t r, g, albedo, cos theta, alpha, beta, N) -> (X, W)
                uint32_t c = c0_group;
                int j = 0;
                for (int k = ka; k < kb; ++k) {
                    if (k > 0 && ((evbits >> (16 + k - ka)) & 1u)) ++c;
                    if ((evbits >> (k - ka)) & 1u) stage_row<6, 7>(A.pm[2], L, base + j++, prng, c, c7);
                }
                stage_normals<6>(A, A.pm[2], L, n_rows);
                decode_tiles(A.pm[2], L, n_rows);
            }
            int j = 0;
            for (int k = ka; k < kb; ++k) {
                V3 X = v3(0, 0, 0), W = v3(0, 0, 1);
                if ((evbits >> (k - ka)) & 1u) {
                    read_row<6>(A.pm[2], L, base + j++, y);
                    X = v3(y[0], y[1], y[2]);
                    W = v3(y[3], y[4], y[5]);
                    const float xl2 = dot(X, X);
                    if (xl2 > 1.0f) X = fast_rsq(xl2) * X;
                    const float wl2 = dot(W, W);
                    W = wl2 > 0.0f ? fast_rsq(wl2) * W : v3(0, 0, 1);
                }
                V3 Xw = v3(0, 0, 0), Ww = v3(0, 0, 1);
                const bool lit_k = ((evbits >> (16 + k - ka)) & 1u) != 0;
                if (lit_k) {
                    // (X, W) rotated by psi about w_in, then into R = [e1 e2 d]
                    const V3 Xt = v3(cp * X.x - sp * X.y, sp * X.x + cp * X.y, X.z);
                    const V3 Wt = v3(cp * W.x - sp * W.y, sp * W.x + cp * W.y, W.z);
                    Xw = po + pr * (Xt.x * e1 + Xt.y * e2 + Xt.z * pd);
                    Ww = normalize(Wt.x * e1 + Wt.y * e2 + Wt.z * pd);
                    if constexpr (!kWaveLight) pLp += w_nee * G.light(A, Xw, Ww);
                }
                if constexpr (kWaveLight) {
                    uint64_t mk[kMaxManyPrims / 64];
                    G.light_mask(A, lit_k, Xw, mk);
                    if (lit_k) pLp += w_nee * G.light_masked(A, Xw, Ww, mk);
                }
            }
            wave_sync();
        }
        if (alive) {
            // Eq. (transform) with R = [e1 e2 d] and the exit frame of Sec. 4.1
            const float st = fast_sqrt(__builtin_fmaxf(0.0f, (1.0f - ct) * (1.0f + ct)));
            const V3 xt = v3(st * cp, st * sp, ct);
            const V3 w0 = v3(be * ct + ga * st, al, -be * st + ga * ct);
            const V3 wt = v3(cp * w0.x - sp * w0.y, sp * w0.x + cp * w0.y, w0.z);
            po = po + pr * (xt.x * e1 + xt.y * e2 + xt.z * pd);
            pd = normalize(wt.x * e1 + wt.y * e2 + wt.z * pd);
        }
        return alive;
    };

    // learned steps of the lanes waiting for one
    auto learned_pass = [&](uint64_t wmask, bool& path_end) __attribute__((always_inline)) {
        wait_age = 0;
        const bool mine = state == S_WAIT;
        const bool alive = learned_core(wmask, mine, o, d, r_step, rng, c0, Lp, p_st);
        if (mine) {
            if (alive) {
                G.set_ray(o, d);
                t = 0.0f;
                state = S_FLY;
            } else {
                path_end = true;
            }
        }
    };
    // Collisions, and for the learned method the decoder passes, repeat in a
    // loop of their own until a restart is due, so that the restart phase's
    // working set does not weigh on them (measured 5-6 % faster for plain
    // tracing, 2-3 % for sphere tracing).  The order of the phases changes no
    // path: each draws from its own stream, and decoder rows are independent.
    bool restart_due = true;
    for (;;) {
        if (restart_due) restart();
        if (ballot(state != S_DONE) == 0) break;
        do {
            bool path_end = false, truncated = false;
            collide(path_end, truncated);
            if constexpr (MODE == kModeStCvae) {
                const uint64_t wmask = ballot(state == S_WAIT);
                const uint64_t lmask = ballot(state == S_FLY || state == S_WAIT);
                const int n_wait = __popcll(wmask);
                wait_age = n_wait > 0 ? wait_age + 1 : 0;
                if (n_wait > 0 && (n_wait >= A.batch_min || wmask == lmask || wait_age > A.max_wait))
                    learned_pass(wmask, path_end);
            }
            if (path_end) {
                if (truncated) tot[T_TRUNC][tid] += 1;
                state = S_END;
            }
            restart_due = restart_now();
        } while (!restart_due);
    }
    if (A.counters) {
        const uint64_t a1 = wave_sum_u64(tot[T_EVENTS][tid]), a2 = wave_sum_u64(tot[T_STEPS][tid]),
                       a3 = wave_sum_u64(tot[T_TRUNC][tid]);
        if (lane_id() == 0) {
            if (a1) atomicAdd(A.counters + 1, (unsigned long long)a1);
            if (a2) atomicAdd(A.counters + 2, (unsigned long long)a2);
            if (a3) atomicAdd(A.counters + 3, (unsigned long long)a3);
        }
    }
}

// Four waves per SIMD: measured faster than the unconstrained allocation
// (three waves) despite a few spilled registers.
template <int MODE, int NP, bool GRID>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void render_kernel(const RenderArgs A) {
    __shared__ RenderLds lds_all[kRenderWaves];
    __shared__ uint32_t lds_tot[kLaneWords][64 * kRenderWaves];
    // many primitives: the scene's n_prims x 8 floats in dynamic LDS, sized
    // at launch, so that the usual scenes (64 spheres: 2 KB) leave room for
    // four blocks per CU
    extern __shared__ float lds_dyn[];
    __shared__ float lds_none[8];
    float* lds_prims = NP == 0 ? lds_dyn : lds_none;
    RenderLds& L = lds_all[threadIdx.x >> 6];
    if (NP == 0) {
        for (int q = threadIdx.x; q < A.n_prims * 8; q += blockDim.x) lds_prims[q] = A.prims[q];
        __syncthreads();
    }
    if (MODE != kModePlain) {
        // No point of the scene reaches tau_min (the deepest point of the
        // deepest primitive, or the step cap, is too shallow), or the deepest
        // possible step would bypass fewer than min_chain collisions (the
        // launch's cost rule): every collision is a plain one, so the plain
        // loop runs -- the same paths and draws, without the learned step's
        // checks and register pressure.
        typename GeoSel<NP, GRID>::type G;
        G.init(A, lds_prims);
        const float t_max = A.sigma_t * __builtin_fminf(G.max_radius(), A.st_max * A.inv_sigma_t);
        const bool pays = !(A.min_chain > 0.0f) || 0.5f * t_max * t_max * (1.0f - A.g) >= A.min_chain;
        if (!(t_max >= A.tau_min) || !pays) {
            render_loop<kModePlain, NP, GRID>(A, L, lds_prims, lds_tot);
            return;
        }
    }
    render_loop<MODE, NP, GRID>(A, L, lds_prims, lds_tot);
}

// Per-pixel fixed-order reduction of the unit partials, added to the image
// with the compensation carried in the comp buffer.
// One wave per pixel: lane c adds the records of chunks c, c + 64, ... in
// order (coalesced 16-byte loads), then a fixed butterfly combines the lanes,
// so the result depends only on n_chunks.
// The launch's path count (every sample of every pixel) goes to the optional
// counters; the render kernel's waves add the other totals.
__global__ void render_reduce_kernel(int64_t npix, int n_chunks, int spp, const UnitRecord* part, float* sum,
                                     float* comp, float* sumsq, uint32_t* events, uint32_t* steps,
                                     const unsigned long long* bad_models, unsigned long long* counters) {
    const int64_t wave0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int lane = lane_id();
    if (*bad_models) {
        // invalid packed models: no path was traced; poison the image
        for (int64_t p = wave0; p < npix; p += n_waves)
            if (lane == 0) sum[p] = __builtin_nanf("");
        return;
    }
    if (counters && wave0 == 0 && lane == 0) atomicAdd(counters, (unsigned long long)(npix * spp));
    for (int64_t p = wave0; p < npix; p += n_waves) {
        const UnitRecord* r = part + p * n_chunks;
        double s = 0.0, q = 0.0;
        uint32_t ev = 0, st = 0;
        for (int c = lane; c < n_chunks; c += 64) {
            const UnitRecord u = r[c];
            s += (double)u.sum;
            q += (double)u.sumsq;
            ev += u.events;
            st += u.steps;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            s += __shfl_xor(s, off);
            q += __shfl_xor(q, off);
            ev += __shfl_xor(ev, off);
            st += __shfl_xor(st, off);
        }
        if (lane == 0) {
            s += (double)sum[p] + (comp ? (double)comp[p] : 0.0);
            if (sumsq) q += (double)sumsq[p];
            if (events) ev += events[p];
            if (steps) st += steps[p];
            const float sf = (float)s;
            sum[p] = sf;
            if (comp) comp[p] = (float)(s - (double)sf);
            if (sumsq) sumsq[p] = (float)q;
            if (events) events[p] = ev;
            if (steps) steps[p] = st;
        }
    }
}

__global__ void render_check_models(const RenderArgs A, unsigned long long* flag) {
    if (threadIdx.x != 0) return;
    const int want_in[3] = {2, 3, 7}, want_out[3] = {1, 3, 6};
    int ok = 1;
    for (int m = 0; m < 3; ++m) {
        const PackedModel* pm = A.pm[m];
        ok &= pm->magic == (int32_t)kPackedMagic && pm->model == m && pm->latent >= 1 && pm->latent <= 8 &&
              pm->latent + pm->p_in <= 16 && pm->p_in == want_in[m] && pm->p_out == want_out[m] &&
              (pm->precision == MS_PREC_BF16 || pm->precision == MS_PREC_FP8) && pm->n_linear >= 2 &&
              pm->n_linear <= kMaxLayers && pm->blocks == 1 && pm->width <= 16;
    }
    *flag = ok ? 0ull : 1ull;
}

__global__ void render_zero_kernel(unsigned long long* ticket, unsigned long long* flag) {
    if (threadIdx.x == 0) {
        ticket[0] = 0ull;
        flag[0] = 0ull;
    }
}

// With invalid models the ticket counter starts past the last unit, so the
// render kernel does no work, and the reduction poisons the image.
__global__ void render_gate_kernel(const unsigned long long* flag, unsigned long long* ticket, int64_t n_units) {
    if (threadIdx.x == 0) ticket[0] = flag[0] ? (unsigned long long)n_units : 0ull;
}

// Conservative FP16 distance grid (the voxel-grid distance pre-process of
// Sec. 3): the union distance min_i sdf_i at voxel centres lo + (i + 1/2) h,
// evaluated in FP64 and rounded toward zero to binary16, so that
// |stored| <= |exact| and the renderer's nearest-voxel radius
// max(0, -stored - half diagonal) never exceeds the true interior distance.
__device__ __forceinline__ double prim_sdf64(const float* pr, double px, double py, double pz) {
    const double qx = px - pr[1], qy = py - pr[2], qz = pz - pr[3];
    if (pr[0] == 0.0f) return sqrt(qx * qx + qy * qy + qz * qz) - (double)pr[4];
    const double ex = fabs(qx) - pr[4], ey = fabs(qy) - pr[5], ez = fabs(qz) - pr[6];
    const double ox = fmax(ex, 0.0), oy = fmax(ey, 0.0), oz = fmax(ez, 0.0);
    return sqrt(ox * ox + oy * oy + oz * oz) + fmin(fmax(ex, fmax(ey, ez)), 0.0);
}

__device__ __forceinline__ uint16_t fp16_bits_rtz(double x) {
    const uint16_t sign = x < 0.0 ? 0x8000u : 0u;
    const double a = fabs(x);
    if (a >= 65504.0) return (uint16_t)(sign | 0x7bffu);
    if (a < 0x1p-24) return sign;
    int e;
    frexp(a, &e);
    const int ex = e - 1;  // a in [2^ex, 2^(ex+1))
    if (ex < -14) return (uint16_t)(sign | (uint32_t)floor(a * 0x1p24));
    const uint32_t mant = (uint32_t)floor((ldexp(a, -ex) - 1.0) * 1024.0);
    return (uint16_t)(sign | ((uint32_t)(ex + 15) << 10) | mant);
}

__global__ void sdf_grid_kernel(const float* prims, int n_prims, int res, double lox, double loy, double loz,
                                double hx, double hy, double hz, uint16_t* out) {
    const int64_t total = (int64_t)res * res * res;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < total; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = v % res, j = (v / res) % res, k = v / ((int64_t)res * res);
        const double px = lox + (i + 0.5) * hx, py = loy + (j + 0.5) * hy, pz = loz + (k + 0.5) * hz;
        double sd = INFINITY;
        for (int q = 0; q < n_prims; ++q) sd = fmin(sd, prim_sdf64(prims + 8 * q, px, py, pz));
        out[v] = fp16_bits_rtz(sd);
    }
}

// Mesh bodies: distance to the nearest triangle, negative where the ray from
// the voxel centre along (1, 2, 3) / sqrt(14) crosses the mesh an odd number
// of times.  Every triangle is visited (a pre-process).
__global__ void sdf_grid_mesh_kernel(const float* tris, int n_tris, int res, double lox, double loy, double loz,
                                     double hx, double hy, double hz, uint16_t* out) {
    const double u[3] = {0.2672612419124244, 0.5345224838248488, 0.8017837257372732};
    const int64_t total = (int64_t)res * res * res;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < total; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = v % res, j = (v / res) % res, k = v / ((int64_t)res * res);
        const double p[3] = {lox + (i + 0.5) * hx, loy + (j + 0.5) * hy, loz + (k + 0.5) * hz};
        double dmin = INFINITY;
        int odd = 0;
        for (int q = 0; q < n_tris; ++q) {
            dmin = fmin(dmin, tri_distance64(tris + 9 * q, p));
            odd ^= (int)tri_ray_crosses64(tris + 9 * q, p, u);
        }
        out[v] = fp16_bits_rtz(odd ? -dmin : dmin);
    }
}

// Samples per work unit: small units balance the end of the persistent
// kernel (a lane's last unit is its tail), large ones bound the partial
// buffers.  About 2^24 units (64 per resident lane of a 256-CU device at
// four 256-thread blocks per CU), and at least 2 samples per unit.
// One render_kernel instance per (mode, geometry policy, radius source).
template <int NP, bool GRID>
static void launch_render(int mode, dim3 grid, dim3 block, hipStream_t hs, const RenderArgs& A) {
    const size_t lds = NP == 0 ? (size_t)A.n_prims * 8 * sizeof(float) : 0;
    if (mode == kModePlain) hipLaunchKernelGGL((render_kernel<kModePlain, NP, GRID>), grid, block, lds, hs, A);
    else if (mode == kModeStExact) hipLaunchKernelGGL((render_kernel<kModeStExact, NP, GRID>), grid, block, lds, hs, A);
    else hipLaunchKernelGGL((render_kernel<kModeStCvae, NP, GRID>), grid, block, lds, hs, A);
}

// Samples per work unit: about 2^23 units (32 per lane of a full launch,
// enough to balance it) of at most 64 samples (longer units leave a longer
// tail); a launch that would then exceed 2^24 units takes longer units to
// keep its record buffer bounded.
static int default_chunk(int64_t npix, int spp) {
    const int64_t total = npix * spp;
    int64_t c = (total + (1 << 23) - 1) >> 23;
    if (c > 64) c = 64;
    if (npix * ((spp + c - 1) / c) > (1 << 24)) c = (total + (1 << 24) - 1) >> 24;
    if (c < 2) c = 2;
    if (c > spp) c = spp;
    return (int)c;
}

}  // namespace msst

extern "C" {

ms_status sphere_trace_render_workspace_size(const ms_camera* cam, const ms_render_desc* desc, size_t* bytes) {
    using namespace msst;
    MS_REQUIRE(cam && desc && bytes, "sphere_trace_render_workspace_size: NULL argument");
    MS_REQUIRE(cam->width > 0 && cam->height > 0, "sphere_trace_render_workspace_size: empty image");
    MS_REQUIRE(desc->spp > 0, "sphere_trace_render_workspace_size: spp must be positive");
    const int chunk = desc->chunk > 0 ? (desc->chunk < desc->spp ? desc->chunk : desc->spp)
                                      : default_chunk((int64_t)cam->width * cam->height, desc->spp);
    const int64_t n_chunks = (desc->spp + chunk - 1) / chunk;
    const int64_t n_units = (int64_t)cam->width * cam->height * n_chunks;
    *bytes = 256 + align_up((size_t)n_units * sizeof(UnitRecord), 256);
    return MS_OK;
}

ms_status sphere_trace_render(const ms_scene* scene, const ms_camera* cam, const ms_light* light,
                              const ms_medium* medium, const ms_render_desc* desc, const ms_image_out* out,
                              void* workspace_dev, size_t workspace_bytes, void* stream) {
    using namespace msst;
    MS_REQUIRE(scene && cam && light && medium && desc && out, "sphere_trace_render: NULL descriptor");
    const bool mesh = scene->n_tris > 0;
    if (mesh) {
        MS_REQUIRE(scene->tris != nullptr && scene->bvh != nullptr && scene->n_nodes >= 1 &&
                       scene->n_nodes <= 2 * scene->n_tris && scene->n_tris < (1 << 26),
                   "sphere_trace_render: a mesh scene needs tris, bvh and 1 <= n_nodes <= 2 n_tris");
        MS_REQUIRE(scene->sdf_fp16 != nullptr && scene->res >= 1,
                   "sphere_trace_render: a mesh scene needs its distance grid");
        MS_REQUIRE(((uintptr_t)scene->bvh & 15u) == 0, "sphere_trace_render: bvh must be 16-byte aligned");
    } else {
        MS_REQUIRE(scene->prims != nullptr && scene->n_prims >= 1 && scene->n_prims <= kMaxManyPrims,
                   "sphere_trace_render: need 1..256 primitives");
    }
    MS_REQUIRE(cam->width > 0 && cam->height > 0 && (int64_t)cam->width * cam->height < ((int64_t)1 << 31),
               "sphere_trace_render: image size must be positive and below 2^31 pixels");
    MS_REQUIRE(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f, "sphere_trace_render: vfov must be in (0, 180)");
    MS_REQUIRE(medium->sigma_t > 0.0f && medium->g > -1.0f && medium->g < 1.0f && medium->albedo > 0.0f &&
                   medium->albedo <= 1.0f,
               "sphere_trace_render: need sigma_t > 0, |g| < 1, albedo in (0, 1]");
    MS_REQUIRE(desc->method == MS_METHOD_PLAIN_NEE || desc->method == MS_METHOD_ST,
               "sphere_trace_render: method must be PLAIN_NEE or ST");
    MS_REQUIRE(desc->sampler == MS_SAMPLER_CVAE || desc->sampler == MS_SAMPLER_EXACT_WALK,
               "sphere_trace_render: unknown sampler");
    const bool learned = desc->method == MS_METHOD_ST && desc->sampler == MS_SAMPLER_CVAE;
    MS_REQUIRE(!learned || (desc->packed[0] && desc->packed[1] && desc->packed[2]),
               "sphere_trace_render: ST with the CVAE sampler needs three packed models");
    MS_REQUIRE(desc->spp > 0 && desc->spp <= (1 << 24), "sphere_trace_render: spp must be in [1, 2^24]");
    MS_REQUIRE(desc->chunk >= 0 && desc->blocks_per_cu >= 0 && desc->blocks_per_cu <= 64 && desc->cvae_batch_min >= 0 &&
                   desc->cvae_batch_min <= 64,
               "sphere_trace_render: invalid launch parameters");
    // tau_min > 0 keeps every learned step off radius 0 (no log(0) condition)
    MS_REQUIRE(desc->tau_min > 0.0f && desc->st_max > 0.0f, "sphere_trace_render: need tau_min > 0, st_max > 0");
    MS_REQUIRE(desc->min_chain >= 0.0f, "sphere_trace_render: min_chain must be >= 0");
    MS_REQUIRE(desc->nee_chain >= 0 && desc->nee_chain <= (1 << 24), "sphere_trace_render: nee_chain must be in [0, 2^24]");
    MS_REQUIRE(desc->nee_samples >= 0 && desc->nee_samples <= 16, "sphere_trace_render: nee_samples must be in [0, 16]");
    MS_REQUIRE(desc->restart_min >= 0 && desc->restart_min <= 64, "sphere_trace_render: restart_min must be in [0, 64]");
    MS_REQUIRE(desc->max_wait >= 0, "sphere_trace_render: max_wait must be >= 0");
    MS_REQUIRE((desc->flags & ~(MS_RENDER_NEE_BEFORE_ABSORPTION | MS_RENDER_STEP_PAPER)) == 0,
               "sphere_trace_render: unknown flags");
    MS_REQUIRE(out->sum && out->sumsq, "sphere_trace_render: sum and sumsq images are required");
    MS_REQUIRE(scene->sdf_fp16 == nullptr || (scene->res > 0 && scene->res <= 4096 && scene->hi[0] > scene->lo[0] &&
                                             scene->hi[1] > scene->lo[1] && scene->hi[2] > scene->lo[2]),
               "sphere_trace_render: invalid SDF grid description");
    size_t need = 0;
    sphere_trace_render_workspace_size(cam, desc, &need);
    MS_REQUIRE(need - 256 < ((size_t)1 << 32) * sizeof(UnitRecord),
               "sphere_trace_render: more than 2^32 work units (raise chunk)");
    MS_REQUIRE(workspace_dev != nullptr, "sphere_trace_render: workspace is NULL");
    if (workspace_bytes < need)
        return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "sphere_trace_render: workspace needs %zu bytes", need);
    int cus;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;

    RenderArgs A{};
    A.prims = scene->prims;
    A.n_prims = mesh ? 0 : scene->n_prims;
    A.bvh = mesh ? reinterpret_cast<const BvhNode*>(scene->bvh) : nullptr;
    A.tris = mesh ? scene->tris : nullptr;
    A.n_nodes = mesh ? scene->n_nodes : 0;
    A.n_tris = mesh ? scene->n_tris : 0;
    A.grid = scene->sdf_fp16;
    A.res = scene->res;
    for (int k = 0; k < 3; ++k) {
        A.grid_lo[k] = scene->lo[k];
        A.grid_inv_h[k] = scene->res > 0 ? (float)(scene->res / ((double)scene->hi[k] - scene->lo[k])) : 0.0f;
    }
    double hmax = 0.0;
    for (int k = 0; k < 3; ++k)
        if (scene->res > 0) hmax = fmax(hmax, ((double)scene->hi[k] - scene->lo[k]) / scene->res);
    A.grid_half_diag = (float)(0.5 * sqrt(3.0) * hmax);
    // camera basis in double, as the pinhole definition reads
    double f[3], up[3] = {cam->up[0], cam->up[1], cam->up[2]};
    for (int k = 0; k < 3; ++k) f[k] = (double)cam->look_at[k] - cam->eye[k];
    double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int k = 0; k < 3; ++k) f[k] /= fl;
    double rt[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    double rl = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    MS_REQUIRE(rl > 0.0, "sphere_trace_render: up is parallel to the view direction");
    for (int k = 0; k < 3; ++k) rt[k] /= rl;
    double uv[3] = {rt[1] * f[2] - rt[2] * f[1], rt[2] * f[0] - rt[0] * f[2], rt[0] * f[1] - rt[1] * f[0]};
    const double th = tan(0.5 * cam->vfov_deg * M_PI / 180.0), aspect = (double)cam->width / cam->height;
    for (int k = 0; k < 3; ++k) {
        A.eye[k] = cam->eye[k];
        A.fwd[k] = (float)f[k];
        A.right[k] = (float)(rt[k] * th * aspect);
        A.upv[k] = (float)(uv[k] * th);
        A.light[k] = light->pos[k];
    }
    A.width = cam->width;
    A.height = cam->height;
    A.npix = (int64_t)cam->width * cam->height;
    A.intensity = light->intensity;
    A.sigma_t = medium->sigma_t;
    A.inv_sigma_t = 1.0f / medium->sigma_t;
    A.g = medium->g;
    A.albedo = medium->albedo;
    A.ln_albedo = (float)log((double)medium->albedo);
    A.surv_thr = (uint32_t)floor((double)medium->albedo * 16777216.0);
    A.method = desc->method;
    A.sampler = desc->sampler;
    for (int m = 0; m < 3; ++m) A.pm[m] = reinterpret_cast<const PackedModel*>(desc->packed[m]);
    A.tau_min = desc->tau_min;
    A.st_max = desc->st_max;
    A.min_chain = desc->min_chain;
    A.spp = desc->spp;
    A.chunk = desc->chunk > 0 ? (desc->chunk < desc->spp ? desc->chunk : desc->spp) : default_chunk(A.npix, desc->spp);
    A.n_chunks = (desc->spp + A.chunk - 1) / A.chunk;
    A.n_units = A.npix * A.n_chunks;
    A.inv_n_chunks = 1.0 / A.n_chunks;
    A.inv_width = 1.0 / A.width;
    A.seed = desc->seed;
    A.sample_offset = desc->sample_offset;
    A.max_events = desc->max_events ? desc->max_events : (1u << 20);
    A.batch_min = desc->cvae_batch_min ? desc->cvae_batch_min : 20;
    A.nee_samples = desc->nee_samples ? desc->nee_samples : 1;
    A.nee_chain = desc->nee_chain;
    A.restart_min = desc->restart_min ? desc->restart_min : 16;
    A.max_wait = desc->max_wait ? desc->max_wait : 10;
    A.flags = desc->flags;
    char* ws = reinterpret_cast<char*>(workspace_dev);
    A.ticket = reinterpret_cast<unsigned long long*>(ws);
    unsigned long long* flag = A.ticket + 1;
    A.part = reinterpret_cast<UnitRecord*>(ws + 256);
    A.counters = reinterpret_cast<unsigned long long*>(out->counters);

    hipStream_t hs = (hipStream_t)stream;
    if (learned) {
        hipLaunchKernelGGL(render_check_models, dim3(1), dim3(64), 0, hs, A, flag);
        hipLaunchKernelGGL(render_gate_kernel, dim3(1), dim3(64), 0, hs, flag, A.ticket, A.n_units);
    } else {
        hipLaunchKernelGGL(render_zero_kernel, dim3(1), dim3(64), 0, hs, A.ticket, flag);
    }
    MS_LAUNCHED();
    const int bpc = desc->blocks_per_cu ? desc->blocks_per_cu : 4;
    int64_t blocks = (int64_t)cus * bpc;
    const int64_t need_blocks = (A.n_units + 255) / 256;
    if (blocks > need_blocks) blocks = need_blocks;
    const int mode = desc->method == MS_METHOD_PLAIN_NEE ? kModePlain
                     : (desc->sampler == MS_SAMPLER_EXACT_WALK ? kModeStExact : kModeStCvae);
    const dim3 grid((unsigned)blocks), block(64 * kRenderWaves);
    const bool grid_r = A.grid != nullptr;
    if (mesh) launch_render<kGeoMesh, true>(mode, grid, block, hs, A);
    else if (A.n_prims <= 1) grid_r ? launch_render<1, true>(mode, grid, block, hs, A) : launch_render<1, false>(mode, grid, block, hs, A);
    else if (A.n_prims == 2) grid_r ? launch_render<2, true>(mode, grid, block, hs, A) : launch_render<2, false>(mode, grid, block, hs, A);
    else if (A.n_prims <= 4) grid_r ? launch_render<4, true>(mode, grid, block, hs, A) : launch_render<4, false>(mode, grid, block, hs, A);
    else grid_r ? launch_render<0, true>(mode, grid, block, hs, A) : launch_render<0, false>(mode, grid, block, hs, A);
    MS_LAUNCHED();
    int64_t rb = (A.npix + 3) / 4;  // four pixels (waves) per block
    if (rb > cus * 16) rb = cus * 16;
    hipLaunchKernelGGL(render_reduce_kernel, dim3((unsigned)rb), dim3(256), 0, hs, A.npix, A.n_chunks, A.spp, A.part,
                       out->sum, out->comp, out->sumsq, out->events, out->steps, flag, A.counters);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

}  // extern "C"

extern "C" ms_status ms_build_sdf_grid(const ms_scene* scene, int32_t res, uint16_t* grid_dev, void* stream) {
    using namespace msst;
    MS_REQUIRE(scene && grid_dev, "ms_build_sdf_grid: NULL argument");
    const bool mesh = scene->n_tris > 0;
    MS_REQUIRE(mesh ? scene->tris != nullptr : scene->prims != nullptr, "ms_build_sdf_grid: NULL geometry");
    MS_REQUIRE(mesh || (scene->n_prims >= 1 && scene->n_prims <= kMaxManyPrims),
               "ms_build_sdf_grid: need 1..256 primitives or a mesh");
    MS_REQUIRE(res >= 1 && res <= 4096, "ms_build_sdf_grid: res must be in [1, 4096]");
    MS_REQUIRE(scene->hi[0] > scene->lo[0] && scene->hi[1] > scene->lo[1] && scene->hi[2] > scene->lo[2],
               "ms_build_sdf_grid: empty bounds");
    int cus;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;
    const int64_t total = (int64_t)res * res * res;
    int64_t blocks = (total + 255) / 256;
    if (blocks > (int64_t)cus * 16) blocks = (int64_t)cus * 16;
    const double h[3] = {((double)scene->hi[0] - scene->lo[0]) / res, ((double)scene->hi[1] - scene->lo[1]) / res,
                         ((double)scene->hi[2] - scene->lo[2]) / res};
    if (mesh)
        hipLaunchKernelGGL(sdf_grid_mesh_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, scene->tris,
                           scene->n_tris, res, (double)scene->lo[0], (double)scene->lo[1], (double)scene->lo[2], h[0],
                           h[1], h[2], grid_dev);
    else
        hipLaunchKernelGGL(sdf_grid_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, scene->prims,
                           scene->n_prims, res, (double)scene->lo[0], (double)scene->lo[1], (double)scene->lo[2], h[0],
                           h[1], h[2], grid_dev);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}
