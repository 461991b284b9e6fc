// mesh.hip -- host construction of the triangle BVH: binned surface-area
// heuristic splits (16 bins per axis over the centroid bounds; a median split
// where the bins cannot separate the triangles), leaves of up to four
// triangles, preorder layout with skip links for stackless traversal.
#include <algorithm>
#include <cstring>
#include <vector>

#include "host.hpp"
#include "mesh.hpp"

namespace msst {
namespace {

struct Builder {
    const float* tris;
    std::vector<int32_t> idx;
    std::vector<BvhNode> nodes;

    void bounds(int b, int e, float* lo, float* hi, bool centroids) const {
        for (int a = 0; a < 3; ++a) {
            lo[a] = INFINITY;
            hi[a] = -INFINITY;
        }
        for (int i = b; i < e; ++i) {
            const float* t = tris + 9 * (size_t)idx[i];
            for (int a = 0; a < 3; ++a) {
                if (centroids) {
                    const float c = (t[a] + t[3 + a] + t[6 + a]) / 3.0f;
                    lo[a] = std::min(lo[a], c);
                    hi[a] = std::max(hi[a], c);
                } else {
                    for (int v = 0; v < 3; ++v) {
                        lo[a] = std::min(lo[a], t[3 * v + a]);
                        hi[a] = std::max(hi[a], t[3 * v + a]);
                    }
                }
            }
        }
    }

    void build(int b, int e, int depth) {
        const int self = (int)nodes.size();
        nodes.push_back(BvhNode{});
        BvhNode nd{};
        bounds(b, e, nd.lo, nd.hi, false);
        if (e - b <= kBvhLeafMax) {
            nd.leaf = (b << 4) | (e - b);
            nd.skip = self + 1;
            nodes[self] = nd;
            return;
        }
        float clo[3], chi[3];
        bounds(b, e, clo, chi, true);
        const float* T = tris;
        auto centroid3 = [T](int32_t x, int a) {
            return T[9 * (size_t)x + a] + T[9 * (size_t)x + 3 + a] + T[9 * (size_t)x + 6 + a];
        };
        // binned SAH: cost of a split = area(left) n_left + area(right) n_right
        constexpr int kBins = 16;
        int best_axis = -1, best_bin = 0;
        double best_cost = INFINITY;
        for (int a = 0; a < 3; ++a) {
            const float ext = chi[a] - clo[a];
            if (!(ext > 0.0f)) continue;
            float blo[kBins][3], bhi[kBins][3];
            int cnt[kBins] = {0};
            for (int k = 0; k < kBins; ++k)
                for (int q = 0; q < 3; ++q) {
                    blo[k][q] = INFINITY;
                    bhi[k][q] = -INFINITY;
                }
            for (int i = b; i < e; ++i) {
                int k = (int)((centroid3(idx[i], a) / 3.0f - clo[a]) / ext * kBins);
                k = std::min(kBins - 1, std::max(0, k));
                ++cnt[k];
                const float* t = tris + 9 * (size_t)idx[i];
                for (int q = 0; q < 3; ++q)
                    for (int v = 0; v < 3; ++v) {
                        blo[k][q] = std::min(blo[k][q], t[3 * v + q]);
                        bhi[k][q] = std::max(bhi[k][q], t[3 * v + q]);
                    }
            }
            auto area = [](const float* lo, const float* hi) {
                const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
                return dx < 0 ? 0.0 : dx * dy + dy * dz + dz * dx;
            };
            for (int split = 1; split < kBins; ++split) {
                float llo[3] = {INFINITY, INFINITY, INFINITY}, lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
                float rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
                int nl = 0, nr = 0;
                for (int k = 0; k < kBins; ++k) {
                    float* lo = k < split ? llo : rlo;
                    float* hi = k < split ? lhi : rhi;
                    (k < split ? nl : nr) += cnt[k];
                    for (int q = 0; q < 3; ++q) {
                        lo[q] = std::min(lo[q], blo[k][q]);
                        hi[q] = std::max(hi[q], bhi[k][q]);
                    }
                }
                if (nl == 0 || nr == 0) continue;
                const double cost = area(llo, lhi) * nl + area(rlo, rhi) * nr;
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_bin = split;
                }
            }
        }
        int mid;
        if (best_axis >= 0 && depth < 48) {
            const int a = best_axis;
            const float ext = chi[a] - clo[a];
            auto left = [&](int32_t x) {
                int k = (int)((centroid3(x, a) / 3.0f - clo[a]) / ext * kBins);
                return std::min(kBins - 1, std::max(0, k)) < best_bin;
            };
            mid = (int)(std::stable_partition(idx.begin() + b, idx.begin() + e, left) - idx.begin());
        } else {
            // no separating bin (or a deep, lopsided branch): split the index
            // range at its median along the longest centroid axis
            int axis = 0;
            for (int a = 1; a < 3; ++a)
                if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
            mid = b + (e - b) / 2;
            std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](int32_t x, int32_t y) {
                const float cx = centroid3(x, axis), cy = centroid3(y, axis);
                return cx < cy || (cx == cy && x < y);
            });
        }
        build(b, mid, depth + 1);
        build(mid, e, depth + 1);
        nd.leaf = -1;
        nd.skip = (int)nodes.size();
        nodes[self] = nd;
    }
};

}  // namespace
}  // namespace msst

extern "C" {

ms_status ms_mesh_bvh_size(int32_t n_tris, size_t* node_bytes) {
    MS_REQUIRE(node_bytes != nullptr, "ms_mesh_bvh_size: node_bytes is NULL");
    MS_REQUIRE(n_tris >= 1 && n_tris < (1 << 26), "ms_mesh_bvh_size: n_tris must be in [1, 2^26)");
    *node_bytes = (size_t)(2 * n_tris) * sizeof(msst::BvhNode);
    return MS_OK;
}

ms_status ms_build_mesh_bvh(const float* tris_host, int32_t n_tris, void* nodes_host, size_t node_bytes,
                            float* tris_sorted_host, int32_t* n_nodes) {
    using namespace msst;
    MS_REQUIRE(tris_host && nodes_host && tris_sorted_host && n_nodes, "ms_build_mesh_bvh: NULL argument");
    MS_REQUIRE(n_tris >= 1 && n_tris < (1 << 26), "ms_build_mesh_bvh: n_tris must be in [1, 2^26)");
    for (int64_t i = 0; i < 9 * (int64_t)n_tris; ++i)
        MS_REQUIRE(std::isfinite(tris_host[i]), "ms_build_mesh_bvh: vertex coordinates must be finite");
    size_t need = 0;
    ms_mesh_bvh_size(n_tris, &need);
    if (node_bytes < need) return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "ms_build_mesh_bvh: nodes need %zu bytes", need);
    Builder bld;
    bld.tris = tris_host;
    bld.idx.resize(n_tris);
    for (int i = 0; i < n_tris; ++i) bld.idx[i] = i;
    bld.nodes.reserve(2 * (size_t)n_tris);
    bld.build(0, n_tris, 0);
    std::memcpy(nodes_host, bld.nodes.data(), bld.nodes.size() * sizeof(BvhNode));
    for (int i = 0; i < n_tris; ++i)
        std::memcpy(tris_sorted_host + 9 * (size_t)i, tris_host + 9 * (size_t)bld.idx[i], 9 * sizeof(float));
    *n_nodes = (int32_t)bld.nodes.size();
    clear_error();
    return MS_OK;
}

}  // extern "C"
