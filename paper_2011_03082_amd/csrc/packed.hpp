// packed.hpp -- inference copy of one CVAE decoder and its wave-level
// evaluation on MFMA (Sec. 3.2: only the decoder is used at render time).
#pragma once

#include "mfma.hpp"
#include "msst.h"

namespace msst {

constexpr uint32_t kPackedMagic = 0x5453534Du;  // "MSST"
constexpr int kMaxLayers = 4;

// Device-side layout; 16-byte aligned, fixed size (cvae_packed_bytes).
struct PackedModel {
    int32_t magic, model, p_in, p_out, latent, width, n_linear, precision;
    float mean_c[16], inv_std_c[16], mean_y[16], std_y[16];
    // FP8: products of layer j are rescaled by out_scale[j] = s_w s_a (weight
    // scale max|W| / 448 times the activation scale s_a, a power of two) and
    // its inputs enter E4M3 multiplied by in_scale[j] = 1 / s_a; both 1 for
    // BF16 (and in_scale 1 without calibration rows)
    float out_scale[kMaxLayers];
    float in_scale[kMaxLayers];
    float bias[kMaxLayers][16];
    // A-operand fragments per decoder layer and lane: 4 bfloat16 (BF16) or
    // 8 FP8 E4M3 values of weight row l % 16 (FP8 uses K = 32, upper half 0
    // for one-block layers).
    uint32_t frag[kMaxLayers][64][2];
    // Two-block layers only (32 features in two 16-row blocks): biases of
    // output rows 16..31 and the other tiles.  BF16 tile t = 2 o + k (t = 0
    // in frag, t = 1..3 in frag_hi[t - 1]) is the weight block of output
    // block o and input block k; FP8 tile o (frag, frag_hi[0]) is output
    // block o, its K = 32 covering both input blocks (bytes 0..3 block 0,
    // bytes 4..7 block 1).
    float bias_hi[kMaxLayers][16];
    uint32_t frag_hi[kMaxLayers][3][64][2];
    int32_t blocks;  // 16 x 16 tiles per layer dimension, 1 or 2
    int32_t pad_[3];
};

__device__ __forceinline__ const uint32_t* frag_tile(const PackedModel* pm, int layer, int t) {
    return t == 0 ? pm->frag[layer][lane_id()] : pm->frag_hi[layer][t - 1][lane_id()];
}
static_assert(sizeof(PackedModel) % 16 == 0, "PackedModel must stay 16-byte sized");

__device__ __forceinline__ bf16x4 load_frag_bf16(const PackedModel* pm, int layer) {
    const uint2 u = *reinterpret_cast<const uint2*>(pm->frag[layer][lane_id()]);
    return __builtin_bit_cast(bf16x4, u);
}

// FP8 E4M3 products on v_mfma_f32_16x16x32_fp8_fp8.  The contraction index
// is permuted so that no data moves between layers: lane group q (lanes
// 16q .. 16q+15) feeds K slots 8q .. 8q+3 with the four D rows 4q .. 4q+3 it
// already holds and zeros in K slots 8q+4 .. 8q+7; the packed weights use
// the same K order (half of K = 32 is padding, as for any 16-wide layer).
typedef long fp8x8;

__device__ __forceinline__ f32x4 mfma_fp8(fp8x8 a, fp8x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ fp8x8 to_fp8x4_lo(f32x4 v) {
    // v_cvt_pk_fp8_f32: two floats to OCP E4M3, round to nearest even;
    // clamped to the largest finite E4M3 value first
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = __builtin_fminf(448.0f, __builtin_fmaxf(-448.0f, v[q]));
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
    return (fp8x8)(uint32_t)w;
}

// Decoder weights of one model held in registers for a pass over several
// tiles: per layer the lane's A fragment (2 dwords: 4 BF16 or 8 FP8 values)
// and the four biases of the output rows k0 .. k0+3 it produces.
constexpr int kDecLayers = 3;

struct DecoderRegs {
    uint2 a[kDecLayers];
    f32x4 b[kDecLayers];
    float sc[kDecLayers];   // out_scale
    float isc[kDecLayers];  // in_scale
};

__device__ __forceinline__ DecoderRegs load_decoder(const PackedModel* pm) {
    DecoderRegs w;
    const int k0 = frag_k0();
#pragma unroll
    for (int j = 0; j < kDecLayers; ++j) {
        w.a[j] = *reinterpret_cast<const uint2*>(pm->frag[j][lane_id()]);
        w.b[j] = *reinterpret_cast<const f32x4*>(&pm->bias[j][k0]);
        w.sc[j] = pm->out_scale[j];
        w.isc[j] = pm->in_scale[j];
    }
    return w;
}

// Runs the three-layer decoder MLP on one 16-path tile whose inputs (z,
// standardised condition; feature-major B operand) are `x`.  Returns the
// output layer in D layout: rows k0..k0+3 of path column frag_row().
__device__ __forceinline__ f32x4 decoder_tile(const DecoderRegs& w, f32x4 xin) {
    bf16x4 x = to_bf16x4(xin);
    f32x4 acc;
#pragma unroll
    for (int j = 0; j < kDecLayers; ++j) {
        acc = mfma_bf16(__builtin_bit_cast(bf16x4, w.a[j]), x, w.b[j]);
        if (j < kDecLayers - 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = softplus(acc[q]);
            x = to_bf16x4(acc);
        }
    }
    return acc;
}

// Layer inputs times the activation scale's reciprocal (a power of two, so
// exact), the operand that enters E4M3.
__device__ __forceinline__ f32x4 scaled(f32x4 x, float isc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] *= isc;
    return x;
}

// The same on FP8 E4M3 weights and activations with per-layer weight and
// activation scales.
__device__ __forceinline__ f32x4 decoder_tile_fp8(const DecoderRegs& w, f32x4 x) {
    f32x4 acc;
#pragma unroll
    for (int j = 0; j < kDecLayers; ++j) {
        const fp8x8 a = (fp8x8)(((uint64_t)w.a[j].y << 32) | w.a[j].x);
        acc = mfma_fp8(a, to_fp8x4_lo(scaled(x, w.isc[j])), f32x4{0, 0, 0, 0});
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = __builtin_fmaf(acc[q], w.sc[j], w.b[j][q]);
        if (j < kDecLayers - 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = softplus(acc[q]);
        }
    }
    return acc;
}

// Any depth (2 .. kMaxLayers linear maps), weights read per layer: the
// path for architectures other than the three-layer default.
__device__ __forceinline__ f32x4 decoder_tile_layers(const PackedModel* pm, f32x4 xin) {
    const int nl = pm->n_linear;
    const int k0 = frag_k0();
    const bool fp8 = pm->precision == MS_PREC_FP8;
    f32x4 x = xin, acc;
    for (int j = 0; j < nl; ++j) {
        const uint2 u = *reinterpret_cast<const uint2*>(pm->frag[j][lane_id()]);
        const f32x4 b = *reinterpret_cast<const f32x4*>(&pm->bias[j][k0]);
        if (fp8) {
            const fp8x8 a = (fp8x8)(((uint64_t)u.y << 32) | u.x);
            acc = mfma_fp8(a, to_fp8x4_lo(scaled(x, pm->in_scale[j])), f32x4{0, 0, 0, 0});
            const float sc = pm->out_scale[j];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_fmaf(acc[q], sc, b[q]);
        } else {
            acc = mfma_bf16(__builtin_bit_cast(bf16x4, u), to_bf16x4(x), b);
        }
        if (j < nl - 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = softplus(acc[q]);
        }
    }
    return acc;
}

// Two-block decoders (Table 1's widest settings), any depth: inputs and
// outputs are 32 features of one 16-path tile, xin[0] rows 0..15 and
// xin[1] rows 16..31 in D layout; weights read per layer.
__device__ __forceinline__ void decoder_tile_wide(const PackedModel* pm, const f32x4* xin, f32x4* out) {
    const int nl = pm->n_linear;
    const int k0 = frag_k0();
    const bool fp8 = pm->precision == MS_PREC_FP8;
    f32x4 x[2] = {xin[0], xin[1]};
    for (int j = 0; j < nl; ++j) {
        f32x4 acc[2];
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const f32x4 b = *reinterpret_cast<const f32x4*>(o == 0 ? &pm->bias[j][k0] : &pm->bias_hi[j][k0]);
            if (fp8) {
                const uint2 u = *reinterpret_cast<const uint2*>(frag_tile(pm, j, o));
                const fp8x8 a = (fp8x8)(((uint64_t)u.y << 32) | u.x);
                const float isc = pm->in_scale[j], sc = pm->out_scale[j];
                const uint64_t lo = (uint32_t)to_fp8x4_lo(scaled(x[0], isc));
                const uint64_t hi = (uint32_t)to_fp8x4_lo(scaled(x[1], isc));
                f32x4 r = mfma_fp8(a, (fp8x8)(lo | (hi << 32)), f32x4{0, 0, 0, 0});
#pragma unroll
                for (int q = 0; q < 4; ++q) r[q] = __builtin_fmaf(r[q], sc, b[q]);
                acc[o] = r;
            } else {
                f32x4 r = b;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const uint2 u = *reinterpret_cast<const uint2*>(frag_tile(pm, j, 2 * o + k));
                    r = mfma_bf16(__builtin_bit_cast(bf16x4, u), to_bf16x4(x[k]), r);
                }
                acc[o] = r;
            }
        }
        if (j < nl - 1) {
#pragma unroll
            for (int o = 0; o < 2; ++o) {
#pragma unroll
                for (int q = 0; q < 4; ++q) x[o][q] = softplus(acc[o][q]);
            }
        } else {
            out[0] = acc[0];
            out[1] = acc[1];
        }
    }
}

}  // namespace msst
