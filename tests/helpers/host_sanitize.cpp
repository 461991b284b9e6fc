// host_sanitize.cpp -- drives the host side of libmsst (argument
// validation of every entry point, size queries, the host-built mesh BVH)
// in a build with AddressSanitizer and UndefinedBehaviorSanitizer on the
// host code (tests/test_host_sanitizers.py).  No device is touched: every
// call here either returns before its first HIP call or is host-only.
// Device pointers are placeholders that validation never dereferences.
// Exits 0 when every call returns the expected status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "msst.h"

static int failures = 0;

static void expect(const char* what, ms_status got, ms_status want) {
    if (got != want) {
        std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, ms_last_error());
        ++failures;
    } else if (want != MS_OK && std::strlen(ms_last_error()) == 0) {
        std::fprintf(stderr, "%s: no error message\n", what);
        ++failures;
    }
}

static void* fake() { return reinterpret_cast<void*>(uintptr_t(0x10000)); }

static void mesh_bvh() {
    std::mt19937 rng(7);
    std::uniform_real_distribution<float> u(-1.0f, 1.0f);
    for (int n : {1, 2, 5, 64, 3000}) {
        std::vector<float> tris(9 * n);
        for (auto& v : tris) v = u(rng);
        if (n > 4)  // a degenerate triangle and two identical ones
            for (int k = 0; k < 9; ++k) tris[9 + k] = tris[k] = k < 3 ? 0.5f : tris[k];
        size_t bytes = 0;
        expect("ms_mesh_bvh_size", ms_mesh_bvh_size(n, &bytes), MS_OK);
        std::vector<unsigned char> nodes(bytes);
        std::vector<float> sorted(9 * n);
        int32_t n_nodes = 0;
        expect("ms_build_mesh_bvh", ms_build_mesh_bvh(tris.data(), n, nodes.data(), bytes, sorted.data(), &n_nodes),
               MS_OK);
        if (n_nodes < 1 || n_nodes > 2 * n) {
            std::fprintf(stderr, "mesh bvh: %d nodes for %d triangles\n", n_nodes, n);
            ++failures;
        }
        if (n > 1)
            expect("ms_build_mesh_bvh small buffer",
                   ms_build_mesh_bvh(tris.data(), n, nodes.data(), 32, sorted.data(), &n_nodes),
                   MS_ERR_WORKSPACE_TOO_SMALL);
        tris[4] = NAN;
        expect("ms_build_mesh_bvh NaN", ms_build_mesh_bvh(tris.data(), n, nodes.data(), bytes, sorted.data(), &n_nodes),
               MS_ERR_INVALID_ARGUMENT);
    }
    size_t bytes = 0;
    expect("ms_mesh_bvh_size 0", ms_mesh_bvh_size(0, &bytes), MS_ERR_INVALID_ARGUMENT);
}

static void cvae_queries() {
    const ms_cvae_shape ok[] = {{0, 2, 1, 4, 16, 3}, {1, 3, 3, 9, 8, 2}, {2, 7, 6, 9, 20, 4}, {2, 7, 6, 5, 12, 2}};
    for (const auto& s : ok) {
        size_t n = 0, ws = 0;
        expect("cvae_param_count", cvae_param_count(&s, &n), MS_OK);
        expect("cvae_workspace_size", cvae_workspace_size(&s, 4096, &ws), MS_OK);
        expect("cvae_workspace_size batch", cvae_workspace_size(&s, 17, &ws), MS_ERR_INVALID_ARGUMENT);
    }
    const ms_cvae_shape bad[] = {{0, 2, 1, 4, 33, 3}, {0, 2, 1, 4, 16, 5}, {2, 7, 6, 17, 16, 3}, {3, 2, 1, 4, 16, 3},
                                 {0, 0, 1, 4, 16, 3}};
    for (const auto& s : bad) {
        size_t n = 0;
        const ms_status st = cvae_param_count(&s, &n);
        if (st == MS_OK) {
            std::fprintf(stderr, "cvae_param_count accepted an invalid shape\n");
            ++failures;
        }
    }
    const ms_cvae_shape s = ok[0];
    float* f = static_cast<float*>(fake());
    ms_adam adam{1e-3, 0.9, 0.999, 1e-8, 0.0, 1};
    expect("cvae_train_step NULL", cvae_train_step(&s, nullptr, f, f, &adam, f, f, 64, 64, 0, 0, 1, 0, 1.0, fake(),
                                                   1 << 20, nullptr, nullptr, nullptr),
           MS_ERR_INVALID_ARGUMENT);
    expect("cvae_train_step batch", cvae_train_step(&s, f, f, f, &adam, f, f, 64, 65, 0, 0, 1, 0, 1.0, fake(),
                                                    1 << 20, nullptr, nullptr, nullptr),
           MS_ERR_INVALID_ARGUMENT);
    expect("cvae_train_step_noalloc batch", cvae_train_step_noalloc(&s, f, f, f, &adam, f, f, 1 << 22, 1 << 21, 1, 0,
                                                                    1, 0, 1.0, nullptr, nullptr, nullptr),
           MS_ERR_INVALID_ARGUMENT);
    expect("cvae_pack precision", cvae_pack(&s, f, static_cast<double*>(fake()), 3, nullptr, 0, fake(),
                                            cvae_packed_bytes(), nullptr),
           MS_ERR_INVALID_ARGUMENT);
    expect("cvae_pack small", cvae_pack(&s, f, static_cast<double*>(fake()), 1, nullptr, 0, fake(), 16, nullptr),
           MS_ERR_WORKSPACE_TOO_SMALL);
    expect("cvae_sample NULL", cvae_sample(nullptr, f, 10, 0, 0, f, nullptr), MS_ERR_INVALID_ARGUMENT);
}

static void walk_queries() {
    ms_walk_desc d{};
    d.n_photons = 1000;
    d.mode = MS_WALK_ANALOG;
    d.sigma_t = 10.0, d.g = 0.8, d.albedo = 0.99, d.radius = 1.0;
    size_t ws = 0;
    expect("ms_random_walk_workspace_size", ms_random_walk_workspace_size(&d, &ws), MS_OK);
    ms_walk_out o{};
    for (int c = 0; c < 5; ++c) {
        ms_walk_desc b = d;
        if (c == 0) b.n_photons = 0;
        if (c == 1) b.sigma_t = -1.0;
        if (c == 2) b.g = 1.0;
        if (c == 3) b.albedo = 1.5;
        if (c == 4) b.radius = 0.0;
        expect("ms_random_walk invalid", ms_random_walk(&b, &o, fake(), 1 << 20, nullptr), MS_ERR_INVALID_ARGUMENT);
    }
    d.mode = MS_WALK_TRAINING;
    d.st_range[0] = 0.0, d.st_range[1] = 200.0;
    expect("ms_random_walk st_range", ms_random_walk(&d, &o, fake(), 1 << 20, nullptr), MS_ERR_INVALID_ARGUMENT);
    expect("ms_philox_fill", ms_philox_fill(0, 0, 0, 0, 0, 1, static_cast<uint32_t*>(fake()), nullptr),
           MS_ERR_INVALID_ARGUMENT);
    expect("ms_select_rows_workspace_size", ms_select_rows_workspace_size(1000, &ws), MS_OK);
    expect("ms_column_moments_workspace_size", ms_column_moments_workspace_size(1000, 3, &ws), MS_OK);
    expect("ms_column_moments dim", ms_column_moments(static_cast<float*>(fake()), 1000, 17,
                                                      static_cast<double*>(fake()), fake(), 1 << 20, nullptr),
           MS_ERR_INVALID_ARGUMENT);
    expect("ms_image_stats_workspace_size", ms_image_stats_workspace_size(4096, &ws), MS_OK);
}

static void render_queries() {
    const float prims_host[16] = {0};
    (void)prims_host;
    ms_scene sc{};
    sc.prims = static_cast<const float*>(fake());
    sc.n_prims = 2;
    ms_camera cam{{0, 0, 4}, {0, 0, 0}, {0, 1, 0}, 40.0f, 16, 16};
    ms_light light{{2, 2, 2}, 10.0f};
    ms_medium med{10.0f, 0.8f, 0.99f};
    ms_render_desc d{};
    d.method = MS_METHOD_PLAIN_NEE;
    d.spp = 4;
    d.tau_min = 1.0f;
    d.st_max = 200.0f;
    size_t ws = 0;
    expect("sphere_trace_render_workspace_size", sphere_trace_render_workspace_size(&cam, &d, &ws), MS_OK);
    ms_image_out img{static_cast<float*>(fake()), static_cast<float*>(fake()), static_cast<float*>(fake()),
                     static_cast<uint32_t*>(fake()), static_cast<uint32_t*>(fake()), nullptr};
    for (int c = 0; c < 12; ++c) {
        ms_render_desc b = d;
        ms_scene s2 = sc;
        ms_camera c2 = cam;
        ms_medium m2 = med;
        if (c == 0) b.method = 7;
        if (c == 1) b.spp = 0;
        if (c == 2) b.flags = 8;
        if (c == 3) b.tau_min = 0.0f;
        if (c == 4) b.min_chain = -1.0f;
        if (c == 5) s2.n_prims = 257;
        if (c == 6) c2.width = 0;
        if (c == 7) c2.vfov_deg = 180.0f;
        if (c == 8) m2.sigma_t = 0.0f;
        if (c == 9) m2.g = 1.0f;
        if (c == 10) b.method = MS_METHOD_ST, b.sampler = MS_SAMPLER_CVAE;  // no models
        if (c == 11) b.nee_samples = 17;
        expect("sphere_trace_render invalid",
               sphere_trace_render(&s2, &c2, &light, &m2, &b, &img, fake(), size_t(1) << 30, nullptr),
               MS_ERR_INVALID_ARGUMENT);
    }
    expect("sphere_trace_render workspace", sphere_trace_render(&sc, &cam, &light, &med, &d, &img, fake(), 16, nullptr),
           MS_ERR_WORKSPACE_TOO_SMALL);
    expect("ms_build_sdf_grid res", ms_build_sdf_grid(&sc, 0, static_cast<uint16_t*>(fake()), nullptr),
           MS_ERR_INVALID_ARGUMENT);
}

int main() {
    if (ms_abi_version() <= 0) ++failures;
    mesh_bvh();
    cvae_queries();
    walk_queries();
    render_queries();
    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("host sanitizer run ok\n");
    return 0;
}
