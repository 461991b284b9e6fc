// device.hpp -- gfx950 device primitives of libmsst: counter-based RNG,
// scattering sampling, frames, wave-level helpers and bfloat16 / FP8 packing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msst {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products; the key advances by the Weyl increments between
// rounds.  Counter = (draw index, id low, id high, stream tag).
__device__ __forceinline__ uint4 philox(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x0 = y0;
        x1 = (uint32_t)p1;
        x2 = y2;
        x3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(x0, x1, x2, x3);
}

struct Rng {
    uint32_t k0, k1, id_lo, id_hi, tag;
    __device__ __forceinline__ uint4 block(uint32_t c0) const { return philox(c0, id_lo, id_hi, tag, k0, k1); }
};

__device__ __forceinline__ Rng make_rng(uint64_t seed, uint32_t tag, uint64_t id) {
    Rng r;
    r.k0 = (uint32_t)seed;
    r.k1 = (uint32_t)(seed >> 32);
    r.id_lo = (uint32_t)id;
    r.id_hi = (uint32_t)(id >> 32);
    r.tag = tag;
    return r;
}

// Uniform on (0, 1]: ((w >> 8) + 1) 2^-24, exact in binary32.
__device__ __forceinline__ float u01(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }
// 24-bit integer form k = (w >> 8) + 1 of the same uniform, for exact
// integer decisions (u <= p  <=>  k <= floor(p 2^24)).
__device__ __forceinline__ uint32_t u24(uint32_t w) { return (w >> 8) + 1u; }

// Hardware transcendentals: v_log_f32 / v_exp_f32 work in base 2,
// v_sin_f32 / v_cos_f32 take revolutions.
__device__ __forceinline__ float fast_ln(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// Hardware square root and quotient through the reciprocal (1 ulp each)
// where a correctly rounded result buys nothing: the IEEE sequences cost
// about ten instructions apiece.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Natural log for free-flight lengths -log(u) / sigma_t: the library logf
// (about 1 ulp relative over (0, 1]).
__device__ __forceinline__ float flight_ln(float u) { return logf(u); }

// Box-Muller pair from two uniforms.
__device__ __forceinline__ void box_muller(float ua, float ub, float& n0, float& n1) {
    const float r = fast_sqrt(-2.0f * fast_ln(ua));
    n0 = r * cos_rev(ub);
    n1 = r * sin_rev(ub);
}

// Henyey-Greenstein sample for uniform xi (Eq. 1 importance sampling),
// returned as (mu, sin theta).  The inverse CDF mu(xi) is evaluated through
//   1 - mu = 2 (1 - g)^2 (1 - xi)(1 + g xi) / q^2,
//   1 + mu = 2 (1 + g)^2 xi (1 - g + g xi) / q^2,    q = 1 + g (2 xi - 1),
// which carry no cancellation for any g (including 0) or xi, so that both
// mu and sin(theta) = sqrt((1 - mu)(1 + mu)) keep full relative precision
// in the strongly forward and backward tails.
struct HgSample {
    float mu, sin_t;
};
__device__ __forceinline__ HgSample hg_sample(float g, float xi) {
    const float q = __builtin_fmaf(g, 2.0f * xi - 1.0f, 1.0f);
    const float iq2 = fast_rcp(q * q);
    const float omg = 1.0f - g, opg = 1.0f + g;
    const float om = 2.0f * omg * omg * (1.0f - xi) * __builtin_fmaf(g, xi, 1.0f) * iq2;
    const float op = 2.0f * opg * opg * xi * __builtin_fmaf(g, xi, omg) * iq2;
    HgSample h;
    h.mu = __builtin_fminf(1.0f, __builtin_fmaxf(-1.0f, 0.5f * (op - om)));
    h.sin_t = fast_sqrt(__builtin_fminf(1.0f, om * op));
    return h;
}

// HG phase function value (Eq. 1).
__device__ __forceinline__ float hg_eval(float g, float cos_t) {
    const float den = __builtin_fmaf(-2.0f * g, cos_t, 1.0f + g * g);
    return 0.0795774715459476679f * (1.0f - g * g) * fast_rsq(den) * fast_rcp(den);
}

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 fma3(float s, V3 a, V3 b) {
    return v3(__builtin_fmaf(s, a.x, b.x), __builtin_fmaf(s, a.y, b.y), __builtin_fmaf(s, a.z, b.z));
}
__device__ __forceinline__ V3 normalize(V3 a) { return fast_rsq(dot(a, a)) * a; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Right-handed orthonormal basis (b1, b2, n) of Duff et al., "Building an
// Orthonormal Basis, Revisited", JCGT 2017.
__device__ __forceinline__ void onb(V3 n, V3& b1, V3& b2) {
    const float sign = __builtin_copysignf(1.0f, n.z);
    const float a = -fast_rcp(sign + n.z);
    const float b = n.x * n.y * a;
    b1 = v3(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
    b2 = v3(b, sign + n.y * n.y * a, -n.y);
}

// Direction with polar cosine mu (sine s) and azimuth (revolutions) about d.
__device__ __forceinline__ V3 scatter(V3 d, float mu, float s, float az_rev) {
    V3 b1, b2;
    onb(d, b1, b2);
    const float ca = cos_rev(az_rev), sa = sin_rev(az_rev);
    V3 nd = mu * d + s * (ca * b1 + sa * b2);
    return normalize(nd);
}

// Distance from x (inside) along unit d to the sphere |y|^2 = r2 about the
// origin: the positive root of t^2 + 2 b t - delta = 0, delta = r2 - |x|^2,
// taken in the form without cancellation.
__device__ __forceinline__ float sphere_exit(V3 x, V3 d, float r2) {
    const float b = dot(x, d);
    const float delta = __builtin_fmaxf(0.0f, r2 - dot(x, x));
    const float root = fast_sqrt(__builtin_fmaf(b, b, delta));
    return b >= 0.0f ? fast_div(delta, b + root) : root - b;
}

// Softplus log(1 + e^x) = max(x, 0) + log(1 + e^-|x|) and its derivative.
__device__ __forceinline__ float softplus(float x) {
    return __builtin_fmaxf(x, 0.0f) + fast_ln(1.0f + fast_exp(-__builtin_fabsf(x)));
}
__device__ __forceinline__ float sigmoid(float x) { return fast_rcp(1.0f + fast_exp(-x)); }

// ---------------------------------------------------------------------------
// Wave helpers (64 lanes).
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Per-wave ticket pool over a global 64-bit counter: lanes that need work
// take consecutive tickets from the wave's private range and the wave
// refills it with one atomic per `chunk` tickets.
struct TicketPool {
    uint64_t next, end;
    __device__ __forceinline__ void reset() {
        next = 0;
        end = 0;
    }
    // Returns this lane's ticket (meaningful where `need`).
    __device__ __forceinline__ uint64_t take(bool need, unsigned long long* counter, uint32_t chunk) {
        const uint64_t mask = ballot(need);
        if (mask == 0) return 0;
        const uint32_t n_need = (uint32_t)__popcll(mask);
        const uint32_t rank = (uint32_t)rank_in(mask);
        const uint64_t avail = end - next;
        uint64_t mine;
        if (avail >= n_need) {
            mine = next + rank;
            next += n_need;
        } else {
            const int leader = __ffsll((long long)mask) - 1;
            unsigned long long base = 0;
            if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)chunk);
            base = __shfl(base, leader);
            mine = rank < avail ? next + rank : base + (rank - avail);
            next = base + (n_need - avail);
            end = base + chunk;
        }
        return mine;
    }
};

// Wave-wide sum of a 64-bit counter (result valid in every lane).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// ---------------------------------------------------------------------------
// bfloat16 (round to nearest even) and FP8 E4M3 (OCP) conversions.
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace msst
