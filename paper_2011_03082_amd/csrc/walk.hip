// walk.hip -- persistent random-walk kernel in a homogeneous sphere
// (training-data process of Sec. 3.1; exit parameterisation of Sec. 4.1;
// representative event of Sec. 4.3).
//
// One photon per lane at a time.  Scattering-chain lengths are heavy tailed
// (1 to ~10^5 events), so lanes take new photons from a per-wave ticket pool
// as soon as theirs leaves the sphere: waves stay full until the global
// ticket counter runs past n_photons, and every wave then exits.  With a few
// photons per lane the end of the run is the last long chains on nearly empty
// waves, so training walks are handed out longest expected chain first (a
// counting sort of the photon ids by a bucket of sigma_t r and g); each
// photon's result depends only on its id, so the order changes no output.
#include "device.hpp"
#include "host.hpp"

namespace msst {

struct WalkArgs {
    uint64_t seed, photon_offset, n;
    float sigma_t, g, albedo, radius, r2, st_report;
    uint32_t surv_thr;  // survive iff u24 <= floor(albedo 2^24)
    float st_lo, st_log2_ratio, g_lo, g_span, a_lo, a_span;
    uint32_t focus_thr;  // focus iff u24 <= floor(focus_fraction 2^24); 0 = never
    float fst_lo, fst_log2_ratio, fg_lo, fg_span;
    int32_t weighting;
    uint32_t max_events;
    float* params;
    uint32_t* n_scatter;
    uint32_t* event_index;
    uint8_t* absorbed;
    uint8_t* truncated;
    float* exit_pos;
    float* exit_dir;
    float* exit_param;
    float* event_pos;
    float* event_dir;
    unsigned long long* counters;
    unsigned long long* ticket;
    const uint32_t* order;  // ticket -> photon index (TRAINING), or null
};

// Order buckets: more expected events first.
constexpr int kOrderBuckets = 128;
constexpr int kOrderChunk = 4096;  // photons per block of the sort kernels

// Parameters of training photon id (the walk kernel draws the same block).
__device__ __forceinline__ void training_params(const WalkArgs& a, uint64_t id, float& st, float& g, float& phi) {
    const uint4 pw = philox(0u, (uint32_t)id, (uint32_t)(id >> 32), MS_TAG_WALK_PARAM, (uint32_t)a.seed,
                            (uint32_t)(a.seed >> 32));
    const bool focus = u24(pw.w) <= a.focus_thr;
    st = (focus ? a.fst_lo : a.st_lo) * __builtin_amdgcn_exp2f(u01(pw.x) * (focus ? a.fst_log2_ratio : a.st_log2_ratio));
    g = __builtin_fmaf(focus ? a.fg_span : a.g_span, u01(pw.y), focus ? a.fg_lo : a.g_lo);
    phi = __builtin_fmaf(a.a_span, u01(pw.z), a.a_lo);
}

// Bucket of the expected chain length, about 1 + tau + tau^2 (1 - g) / 3
// events for optical radius tau (a diffusion estimate; only its order matters),
// reversed so that bucket 0 holds the longest chains.
__device__ __forceinline__ int order_bucket(float st, float g) {
    const float cost = 1.0f + st + 0.35f * st * st * (1.0f - g);
    const int b = (int)(8.0f * __builtin_amdgcn_logf(cost));
    return kOrderBuckets - 1 - (b < 0 ? 0 : b > kOrderBuckets - 1 ? kOrderBuckets - 1 : b);
}

__global__ __launch_bounds__(256) void walk_order_count(const WalkArgs a, uint32_t* counts) {
    __shared__ uint32_t h[kOrderBuckets];
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * kOrderChunk;
    for (uint64_t i = lo + threadIdx.x; i < a.n && i < lo + kOrderChunk; i += blockDim.x) {
        float st, g, phi;
        training_params(a, a.photon_offset + i, st, g, phi);
        atomicAdd(&h[order_bucket(st, g)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x)
        if (h[b]) atomicAdd(&counts[b], h[b]);
}

// Exclusive prefix of the bucket counts (one wave, bucket order).
__global__ void walk_order_scan(const uint32_t* counts, uint32_t* cursor) {
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int b = 0; b < kOrderBuckets; ++b) {
        cursor[b] = acc;
        acc += counts[b];
    }
}

__global__ __launch_bounds__(256) void walk_order_scatter(const WalkArgs a, uint32_t* cursor, uint32_t* order) {
    __shared__ uint32_t h[kOrderBuckets], base[kOrderBuckets];
    __shared__ uint8_t key[kOrderChunk];
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * kOrderChunk;
    for (uint64_t i = lo + threadIdx.x; i < a.n && i < lo + kOrderChunk; i += blockDim.x) {
        float st, g, phi;
        training_params(a, a.photon_offset + i, st, g, phi);
        const int b = order_bucket(st, g);
        key[i - lo] = (uint8_t)b;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) {
        base[b] = h[b] ? atomicAdd(&cursor[b], h[b]) : 0u;
        h[b] = 0u;
    }
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < a.n && i < lo + kOrderChunk; i += blockDim.x) {
        const int b = key[i - lo];
        order[base[b] + atomicAdd(&h[b], 1u)] = (uint32_t)i;
    }
}

__device__ __forceinline__ void put3(float* base, uint64_t n, uint64_t i, V3 v) {
    if (!base) return;
    base[i] = v.x;
    base[n + i] = v.y;
    base[2 * n + i] = v.z;
}

// A photon's end (writing its record) and the start of the next one run in
// one pass per wave once this many lanes wait, or when no lane is walking, so
// that the code is not issued every iteration for a few lanes.
constexpr int kWalkRestartMin = 16;

template <int MODE>
__global__ __launch_bounds__(256) void walk_kernel(const WalkArgs a) {
    TicketPool pool;
    pool.reset();
    // lane state: walking, ended (record not yet written), idle, done
    bool active = false, ended = false, done = false;
    bool absorbed = false, truncated = false;
    uint64_t i = 0;
    Rng rng = make_rng(a.seed, MS_TAG_WALK_EVENT, 0);
    V3 x = v3(0, 0, 0), d = v3(0, 0, 1), xk = v3(0, 0, 0), wk = v3(0, 0, 1);
    uint32_t nev = 0, c0 = 0, k = 1;
    float st = a.sigma_t, inv_st = 1.0f / a.sigma_t, g = a.g, phi = a.albedo, inv_phi = 1.0f, resv = 0.0f;
    const float r = MODE == MS_WALK_ANALOG ? a.radius : 1.0f;
    const float r2 = MODE == MS_WALK_ANALOG ? a.r2 : 1.0f;
    uint64_t n_events = 0, n_abs = 0, n_trunc = 0, n_max = 0;

    for (;;) {
        const uint64_t rmask = ballot(!active && !done);
        if (rmask != 0 && (__popcll(rmask) >= kWalkRestartMin || ballot(active) == 0)) {
            if (ended) {
                // the record of the finished photon; x holds its exit point
                ended = false;
                n_events += nev;
                n_abs += absorbed;
                n_trunc += truncated;
                n_max = nev > n_max ? nev : n_max;
                const uint64_t n = a.n;
                if (a.params) {
                    put3(a.params, n, i, v3(MODE == MS_WALK_ANALOG ? a.st_report : st, g, phi));
                }
                if (a.n_scatter) a.n_scatter[i] = nev;
                if (a.absorbed) a.absorbed[i] = (uint8_t)absorbed;
                if (a.truncated) a.truncated[i] = (uint8_t)truncated;
                put3(a.exit_pos, n, i, x);
                put3(a.exit_dir, n, i, d);
                // exit frame of Sec. 4.1 after rotating by -psi about w_in = z
                const float ir = 1.0f / r;
                const V3 xh = ir * x;
                const float sin_t = __builtin_sqrtf(xh.x * xh.x + xh.y * xh.y);
                float cp = 1.0f, sp = 0.0f;
                if (sin_t > 0.0f) {
                    cp = xh.x / sin_t;
                    sp = xh.y / sin_t;
                }
                if (a.exit_param) {
                    const V3 wp = v3(cp * d.x + sp * d.y, -sp * d.x + cp * d.y, d.z);
                    put3(a.exit_param, n, i, v3(xh.z, wp.y, wp.x * xh.z - wp.z * sin_t));
                }
                if (MODE == MS_WALK_TRAINING) {
                    if (a.event_index) a.event_index[i] = k;
                    const V3 xs = ir * xk;
                    put3(a.event_pos, n, i, v3(cp * xs.x + sp * xs.y, -sp * xs.x + cp * xs.y, xs.z));
                    put3(a.event_dir, n, i, v3(cp * wk.x + sp * wk.y, -sp * wk.x + cp * wk.y, wk.z));
                }
            }
            const bool need = !active && !done;
            const uint64_t t = pool.take(need, a.ticket, 64);
            if (need) {
                if (t < a.n) {
                    i = a.order ? a.order[t] : t;
                    active = true;
                    const uint64_t id = a.photon_offset + i;
                    rng = make_rng(a.seed, MS_TAG_WALK_EVENT, id);
                    if (MODE == MS_WALK_TRAINING) {
                        training_params(a, id, st, g, phi);
                        inv_st = 1.0f / st;
                        inv_phi = 1.0f / phi;
                    }
                    x = v3(0, 0, 0);
                    d = v3(0, 0, 1);
                    xk = x;
                    wk = d;
                    nev = 0;
                    c0 = 0;
                    k = 1;
                    resv = 0.0f;
                } else {
                    done = true;
                }
            }
        }
        if (ballot(!done) == 0) break;
        if (!active) continue;

        ++nev;
        const uint4 w = rng.block(c0++);
        bool stop = false;
        absorbed = false;
        truncated = false;
        V3 xe = x;
        if (MODE == MS_WALK_ANALOG) {
            if (u24(w.w) > a.surv_thr) {
                absorbed = true;
                stop = true;
            }
        } else {
            bool keep;
            if (a.weighting == MS_EVENT_UNIFORM) {
                keep = (uint64_t)u24(w.w) * nev <= (1ull << 24);
            } else {
                resv = nev == 1 ? 1.0f : __builtin_fmaf(resv, inv_phi, 1.0f);
                keep = u01(w.w) * resv <= 1.0f;
            }
            if (keep) {
                xk = x;
                wk = d;
                k = nev;
            }
        }
        if (!stop) {
            const HgSample h = hg_sample(g, u01(w.y));
            d = scatter(d, h.mu, h.sin_t, u01(w.z));
            const float l = -flight_ln(u01(w.x)) * inv_st;
            const V3 xn = fma3(l, d, x);
            if (!(dot(xn, xn) < r2)) {
                xe = fma3(sphere_exit(x, d, r2), d, x);
                stop = true;
            } else {
                x = xn;
                if (nev >= a.max_events) {
                    truncated = true;
                    xe = x;
                    stop = true;
                }
            }
        }
        if (stop) {
            active = false;
            ended = true;
            x = xe;
        }
    }
    if (a.counters) {
        const uint64_t se = wave_sum_u64(n_events), sa = wave_sum_u64(n_abs), stc = wave_sum_u64(n_trunc);
        const uint64_t mx = wave_max_u64(n_max);
        if (lane_id() == 0) {
            atomicAdd(a.counters + 0, (unsigned long long)se);
            atomicAdd(a.counters + 1, (unsigned long long)sa);
            atomicAdd(a.counters + 2, (unsigned long long)stc);
            atomicMax(a.counters + 3, (unsigned long long)mx);
        }
    }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    const int t = threadIdx.x;
    if (t < n) p[t] = 0ull;
}

}  // namespace msst

extern "C" {

ms_status ms_random_walk_workspace_size(const ms_walk_desc* desc, size_t* bytes) {
    MS_REQUIRE(desc != nullptr && bytes != nullptr, "ms_random_walk_workspace_size: NULL argument");
    // ticket counter; for training walks of fewer than 2^32 photons also the
    // order buckets and the photon order (4 bytes per photon)
    *bytes = 256;
    if (desc->mode == MS_WALK_TRAINING && desc->n_photons < (1ull << 32))
        *bytes = 2048 + msst::align_up((size_t)desc->n_photons * 4, 256);
    return MS_OK;
}

ms_status ms_random_walk(const ms_walk_desc* desc, const ms_walk_out* out, void* workspace_dev,
                         size_t workspace_bytes, void* stream) {
    using namespace msst;
    MS_REQUIRE(desc != nullptr && out != nullptr, "ms_random_walk: NULL descriptor");
    const ms_walk_desc& d = *desc;
    MS_REQUIRE(d.n_photons > 0 && d.n_photons < (1ull << 40), "ms_random_walk: n_photons must be in [1, 2^40)");
    MS_REQUIRE(d.mode == MS_WALK_ANALOG || d.mode == MS_WALK_TRAINING, "ms_random_walk: unknown mode %d", d.mode);
    MS_REQUIRE(d.blocks_per_cu >= 0 && d.blocks_per_cu <= 64, "ms_random_walk: blocks_per_cu must be in [0, 64]");
    if (d.mode == MS_WALK_ANALOG) {
        MS_REQUIRE(d.sigma_t > 0.0 && d.sigma_t < 1e30, "ms_random_walk: sigma_t must be positive and finite");
        MS_REQUIRE(d.g > -1.0 && d.g < 1.0, "ms_random_walk: |g| must be < 1");
        MS_REQUIRE(d.albedo >= 0.0 && d.albedo <= 1.0, "ms_random_walk: albedo must be in [0, 1]");
        MS_REQUIRE(d.radius > 0.0 && d.radius < 1e30, "ms_random_walk: radius must be positive and finite");
    } else {
        MS_REQUIRE(d.event_weighting == MS_EVENT_ALBEDO_POWER || d.event_weighting == MS_EVENT_UNIFORM,
                   "ms_random_walk: unknown event weighting %d", d.event_weighting);
        MS_REQUIRE(d.st_range[0] > 0.0 && d.st_range[1] >= d.st_range[0] && d.st_range[1] < 1e30,
                   "ms_random_walk: st_range must satisfy 0 < lo <= hi");
        MS_REQUIRE(d.g_range[0] > -1.0 && d.g_range[1] >= d.g_range[0] && d.g_range[1] < 1.0,
                   "ms_random_walk: g_range must satisfy -1 < lo <= hi < 1");
        MS_REQUIRE(d.albedo_range[0] > 0.0 && d.albedo_range[1] >= d.albedo_range[0] && d.albedo_range[1] <= 1.0,
                   "ms_random_walk: albedo_range must satisfy 0 < lo <= hi <= 1");
        MS_REQUIRE(d.focus_fraction >= 0.0 && d.focus_fraction <= 1.0, "ms_random_walk: focus_fraction must be in [0, 1]");
        if (d.focus_fraction > 0.0) {
            MS_REQUIRE(d.focus_st_range[0] > 0.0 && d.focus_st_range[1] >= d.focus_st_range[0] &&
                           d.focus_st_range[1] < 1e30,
                       "ms_random_walk: focus_st_range must satisfy 0 < lo <= hi");
            MS_REQUIRE(d.focus_g_range[0] > -1.0 && d.focus_g_range[1] >= d.focus_g_range[0] && d.focus_g_range[1] < 1.0,
                       "ms_random_walk: focus_g_range must satisfy -1 < lo <= hi < 1");
        }
    }
    size_t ws_need = 0;
    ms_random_walk_workspace_size(desc, &ws_need);
    MS_REQUIRE(workspace_dev != nullptr, "ms_random_walk: workspace is NULL");
    if (workspace_bytes < ws_need)
        return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "ms_random_walk: workspace needs %zu bytes", ws_need);
    MS_REQUIRE(((uintptr_t)workspace_dev & 7u) == 0, "ms_random_walk: workspace must be 8-byte aligned");

    int cus = 0;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;

    WalkArgs a{};
    a.seed = d.seed;
    a.photon_offset = d.photon_offset;
    a.n = d.n_photons;
    a.sigma_t = (float)d.sigma_t;
    a.g = (float)d.g;
    a.albedo = (float)d.albedo;
    a.radius = (float)d.radius;
    a.r2 = (float)d.radius * (float)d.radius;
    a.st_report = (float)(d.sigma_t * d.radius);
    a.surv_thr = (uint32_t)floor(d.albedo * 16777216.0);
    a.st_lo = (float)d.st_range[0];
    a.st_log2_ratio = (float)log2(d.st_range[1] / d.st_range[0]);
    a.g_lo = (float)d.g_range[0];
    a.g_span = (float)(d.g_range[1] - d.g_range[0]);
    a.a_lo = (float)d.albedo_range[0];
    a.a_span = (float)(d.albedo_range[1] - d.albedo_range[0]);
    a.focus_thr = (uint32_t)floor(d.focus_fraction * 16777216.0);
    if (d.focus_fraction > 0.0) {
        a.fst_lo = (float)d.focus_st_range[0];
        a.fst_log2_ratio = (float)log2(d.focus_st_range[1] / d.focus_st_range[0]);
        a.fg_lo = (float)d.focus_g_range[0];
        a.fg_span = (float)(d.focus_g_range[1] - d.focus_g_range[0]);
    }
    a.weighting = d.event_weighting;
    a.max_events = d.max_events ? d.max_events : (1u << 20);
    a.params = out->params;
    a.n_scatter = out->n_scatter;
    a.event_index = out->event_index;
    a.absorbed = out->absorbed;
    a.truncated = out->truncated;
    a.exit_pos = out->exit_pos;
    a.exit_dir = out->exit_dir;
    a.exit_param = out->exit_param;
    a.event_pos = out->event_pos;
    a.event_dir = out->event_dir;
    a.counters = reinterpret_cast<unsigned long long*>(out->counters);
    a.ticket = reinterpret_cast<unsigned long long*>(workspace_dev);

    hipStream_t s = (hipStream_t)stream;
    if (ws_need > 256) {
        // longest expected chains first: counts, prefix, scatter of the ids
        uint32_t* counts = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(workspace_dev) + 1024);
        uint32_t* cursor = counts + kOrderBuckets;
        uint32_t* order = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(workspace_dev) + 2048);
        const unsigned ob = (unsigned)((d.n_photons + kOrderChunk - 1) / kOrderChunk);
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long*>(counts),
                           kOrderBuckets / 2);
        hipLaunchKernelGGL(walk_order_count, dim3(ob), dim3(256), 0, s, a, counts);
        hipLaunchKernelGGL(walk_order_scan, dim3(1), dim3(64), 0, s, counts, cursor);
        hipLaunchKernelGGL(walk_order_scatter, dim3(ob), dim3(256), 0, s, a, cursor, order);
        a.order = order;
    }
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, a.ticket, 1);
    MS_LAUNCHED();
    const int bpc = d.blocks_per_cu ? d.blocks_per_cu : 2;
    uint64_t blocks = (uint64_t)cus * bpc;
    const uint64_t need = (d.n_photons + 255) / 256;
    if (blocks > need) blocks = need;
    if (d.mode == MS_WALK_ANALOG)
        hipLaunchKernelGGL(walk_kernel<MS_WALK_ANALOG>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(walk_kernel<MS_WALK_TRAINING>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

}  // extern "C"
