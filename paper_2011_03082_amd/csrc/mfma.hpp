// mfma.hpp -- 16x16 CVAE layers on gfx950 matrix cores.
//
// Activations are kept feature-major: one 16 x 16 tile holds 16 features
// (rows) of 16 samples (columns).  For v_mfma_f32_16x16x16_bf16 the B
// operand and the D result of lane l both cover rows 4 (l / 16) + j,
// j = 0..3, of column l % 16, so the output of one layer, after its
// activation, is already the next layer's B operand: a whole MLP chains
// through registers with no data movement.  The A operand (the weights)
// covers row l % 16, columns 4 (l / 16) + j.
#pragma once

#include "device.hpp"

namespace msst {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 16;
constexpr int kLayerFloats = kTile * kTile + kTile;

__device__ __forceinline__ f32x4 mfma_bf16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int frag_row() { return lane_id() & 15; }  // A row / B, D column
__device__ __forceinline__ int frag_k0() { return (lane_id() >> 4) * 4; } // first of 4 K (or D) rows

__device__ __forceinline__ bf16x4 to_bf16x4(float a, float b, float c, float d) {
    bf16x4 r;
    r[0] = (__bf16)a;
    r[1] = (__bf16)b;
    r[2] = (__bf16)c;
    r[3] = (__bf16)d;
    return r;
}
__device__ __forceinline__ bf16x4 to_bf16x4(f32x4 v) { return to_bf16x4(v[0], v[1], v[2], v[3]); }
__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

// Intra-wave ordering of LDS traffic between lanes of the same wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile in LDS, row-major [row][col], 16 x 16 floats.
// D / B positions of this lane: rows k0..k0+3, column c.
__device__ __forceinline__ void tile_store_d(float* t, f32x4 v) {
    const int c = frag_row(), k0 = frag_k0();
#pragma unroll
    for (int j = 0; j < 4; ++j) t[(k0 + j) * kTile + c] = v[j];
}
__device__ __forceinline__ f32x4 tile_load_d(const float* t) {
    const int c = frag_row(), k0 = frag_k0();
    f32x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = t[(k0 + j) * kTile + c];
    return v;
}
// Transposed read: row c, columns k0..k0+3 (the A operand of a tile, or the
// B operand of its transpose).
__device__ __forceinline__ f32x4 tile_load_t(const float* t) {
    const int r = frag_row(), k0 = frag_k0();
    return *reinterpret_cast<const f32x4*>(t + r * kTile + k0);
}

}  // namespace msst
