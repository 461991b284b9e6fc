// mesh.hpp -- closed triangle-mesh bodies: a stackless bounding-volume
// hierarchy over the triangles, line crossings (the surface of record) and,
// for the distance grid, FP64 point-triangle distances with a parity sign.
#pragma once

#include "device.hpp"

namespace msst {

// Nodes in depth-first preorder: an inner node's first child follows it, and
// `skip` is the first node after its subtree, so a traversal needs no stack
// (descend on a hit, jump to `skip` on a miss or after a leaf).
struct alignas(16) BvhNode {
    float lo[3];
    int32_t skip;
    float hi[3];
    int32_t leaf;  // (first triangle << 4) | count for a leaf, -1 for an inner node
};
static_assert(sizeof(BvhNode) == 32, "BvhNode is 32 bytes");
constexpr int kBvhLeafMax = 4;

// Does the segment o + t d, tlo <= t <= thi, meet the box?
__device__ __forceinline__ bool line_box(const BvhNode& nd, V3 o, V3 inv, float tlo, float thi) {
    const float ax = (nd.lo[0] - o.x) * inv.x, bx = (nd.hi[0] - o.x) * inv.x;
    const float ay = (nd.lo[1] - o.y) * inv.y, by = (nd.hi[1] - o.y) * inv.y;
    const float az = (nd.lo[2] - o.z) * inv.z, bz = (nd.hi[2] - o.z) * inv.z;
    const float t0 = __builtin_fmaxf(__builtin_fmaxf(__builtin_fminf(ax, bx), __builtin_fminf(ay, by)),
                                     __builtin_fminf(az, bz));
    const float t1 = __builtin_fminf(__builtin_fminf(__builtin_fmaxf(ax, bx), __builtin_fmaxf(ay, by)),
                                     __builtin_fmaxf(az, bz));
    return __builtin_fmaxf(t0, tlo) <= __builtin_fminf(t1, thi);
}

// Line parameter of the crossing with triangle tr (Moller and Trumbore,
// JGT 1997, both facings); false if the line misses it.
__device__ __forceinline__ bool tri_cross(const float* tr, V3 o, V3 d, float& t) {
    const V3 a = v3(tr[0], tr[1], tr[2]);
    const V3 e1 = v3(tr[3], tr[4], tr[5]) - a, e2 = v3(tr[6], tr[7], tr[8]) - a;
    const V3 pv = cross(d, e2);
    const float det = dot(e1, pv);
    if (det == 0.0f) return false;
    const float inv = fast_rcp(det);
    const V3 s = o - a;
    const float u = dot(s, pv) * inv;
    if (u < 0.0f || u > 1.0f) return false;
    const V3 qv = cross(s, e1);
    const float v = dot(d, qv) * inv;
    if (v < 0.0f || u + v > 1.0f) return false;
    t = dot(e2, qv) * inv;
    return true;
}

constexpr int kMeshCross = 8;  // crossings of one line kept (sorted)

// The crossings of the segment o + t d, tlo < t <= thi, with the mesh,
// sorted, in c[0 .. m) (at most kMeshCross; more are dropped from the end of
// the sorted order).  Boxes the segment misses are skipped whole.
__device__ __forceinline__ int mesh_crossings(const BvhNode* nodes, int n_nodes, const float* tris, V3 o, V3 d,
                                              float tlo, float thi, float* c) {
    const V3 inv = v3(fast_rcp(d.x), fast_rcp(d.y), fast_rcp(d.z));
#pragma unroll
    for (int j = 0; j < kMeshCross; ++j) c[j] = INFINITY;
    int m = 0;
    for (int i = 0; i < n_nodes;) {
        const BvhNode nd = nodes[i];
        const bool hit = line_box(nd, o, inv, tlo, thi);
        if (hit && nd.leaf >= 0) {
            const int first = nd.leaf >> 4, cnt = nd.leaf & 15;
            for (int k = 0; k < cnt; ++k) {
                float t;
                if (tri_cross(tris + 9 * (first + k), o, d, t) && t > tlo && t <= thi) {
                    // insertion into the sorted slots (the largest falls off)
#pragma unroll
                    for (int j = kMeshCross - 1; j >= 0; --j) {
                        const float prev = j > 0 ? c[j - 1] : -INFINITY;
                        if (t < c[j]) c[j] = t < prev ? prev : t;
                    }
                    ++m;
                }
            }
        }
        i = (hit && nd.leaf < 0) ? i + 1 : nd.skip;
    }
    return m < kMeshCross ? m : kMeshCross;
}

// ---- FP64, for the distance grid

__device__ __forceinline__ double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Distance from p to triangle tr: closest point by the Voronoi-region tests
// of Ericson, "Real-Time Collision Detection" (2005), Sec. 5.1.5.
__device__ inline double tri_distance64(const float* tr, const double* p) {
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
    const double d1 = dot3(ab, ap), d2 = dot3(ac, ap), d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    if (d1 <= 0.0 && d2 <= 0.0) {
        for (int i = 0; i < 3; ++i) q[i] = a[i];
    } else if (d3 >= 0.0 && d4 <= d3) {
        for (int i = 0; i < 3; ++i) q[i] = b[i];
    } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        const double v = d1 / (d1 - d3);
        for (int i = 0; i < 3; ++i) q[i] = a[i] + v * ab[i];
    } else if (d6 >= 0.0 && d5 <= d6) {
        for (int i = 0; i < 3; ++i) q[i] = c[i];
    } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        const double w = d2 / (d2 - d6);
        for (int i = 0; i < 3; ++i) q[i] = a[i] + w * ac[i];
    } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int i = 0; i < 3; ++i) q[i] = b[i] + w * (c[i] - b[i]);
    } else {
        const double den = 1.0 / (va + vb + vc), v = vb * den, w = vc * den;
        for (int i = 0; i < 3; ++i) q[i] = a[i] + ab[i] * v + ac[i] * w;
    }
    const double e[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    return sqrt(dot3(e, e));
}

// Does the ray p + t u, t > 0, cross triangle tr (FP64 Moller-Trumbore)?
__device__ inline bool tri_ray_crosses64(const float* tr, const double* p, const double* u) {
    double a[3], e1[3], e2[3], s[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = tr[i];
        e1[i] = (double)tr[3 + i] - a[i];
        e2[i] = (double)tr[6 + i] - a[i];
        s[i] = p[i] - a[i];
    }
    const double pv[3] = {u[1] * e2[2] - u[2] * e2[1], u[2] * e2[0] - u[0] * e2[2], u[0] * e2[1] - u[1] * e2[0]};
    const double det = dot3(e1, pv);
    if (det == 0.0) return false;
    const double inv = 1.0 / det;
    const double uu = dot3(s, pv) * inv;
    if (uu < 0.0 || uu > 1.0) return false;
    const double qv[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    const double vv = dot3(u, qv) * inv;
    if (vv < 0.0 || uu + vv > 1.0) return false;
    return dot3(e2, qv) * inv > 0.0;
}

}  // namespace msst
