// packed.hpp -- inference copy of one CVAE decoder and its wave-level
// evaluation on MFMA (Sec. 3.2: only the decoder is used at render time).
#pragma once

#include "mfma.hpp"

namespace msst {

constexpr uint32_t kPackedMagic = 0x5453534Du;  // "MSST"
constexpr int kMaxLayers = 4;

// Device-side layout; 16-byte aligned, fixed size (cvae_packed_bytes).
struct PackedModel {
    int32_t magic, model, p_in, p_out, latent, width, n_linear, precision;
    float mean_c[16], inv_std_c[16], mean_y[16], std_y[16];
    float w_scale[kMaxLayers];     // per-layer weight scale (FP8), 1 for BF16
    float reserved[kMaxLayers];
    float bias[kMaxLayers][16];
    // A-operand fragments per decoder layer and lane: 4 bfloat16 (BF16) or
    // 8 FP8 E4M3 values of weight row l % 16 (FP8 uses K = 32, upper half 0).
    uint32_t frag[kMaxLayers][64][2];
};
static_assert(sizeof(PackedModel) % 16 == 0, "PackedModel must stay 16-byte sized");

__device__ __forceinline__ bf16x4 load_frag_bf16(const PackedModel* pm, int layer) {
    const uint2 u = *reinterpret_cast<const uint2*>(pm->frag[layer][lane_id()]);
    return __builtin_bit_cast(bf16x4, u);
}

// Runs the decoder MLP on one 16-path tile whose inputs (z, standardised
// condition; feature-major B operand) are `x`.  Returns the output layer in
// D layout: rows k0..k0+3 of path column frag_row().
__device__ __forceinline__ f32x4 decoder_tile(const PackedModel* pm, bf16x4 x) {
    const int nl = pm->n_linear;
    const int k0 = frag_k0();
    f32x4 acc;
    for (int j = 0; j < nl; ++j) {
        const float* b = pm->bias[j];
        acc = f32x4{b[k0], b[k0 + 1], b[k0 + 2], b[k0 + 3]};
        acc = mfma_bf16(load_frag_bf16(pm, j), x, acc);
        if (j < nl - 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = softplus(acc[q]);
            x = to_bf16x4(acc);
        }
    }
    return acc;
}

}  // namespace msst
