// cvae.hip -- conditional VAEs of Sec. 3.2 / Sec. 4.2 on gfx950: parameter
// init, training features, FP64 column moments, fused forward + backward on
// bfloat16 MFMA with FP32 master weights and AdamW, packing of the decoder
// for inference, and decoder-only sampling.
#include <math.h>

#include <mutex>

#include "host.hpp"
#include "packed.hpp"

namespace msst {

constexpr float kLvMin = -12.0f, kLvMax = 8.0f;
constexpr float kLog2Pi = 1.83787706640934548f;
constexpr int kTrainWaves = 4;  // waves per training block
constexpr int kMaxNL = 4;       // linear maps per network: 2 .. 4 (one to three hidden layers)
constexpr int kMaxDevices = 64; // devices whose noalloc scratch address is kept

struct Shape {
    int model, p_in, p_out, latent, width, n_linear;
};

__device__ __forceinline__ float clamp_lv(float x) { return __builtin_fminf(kLvMax, __builtin_fmaxf(kLvMin, x)); }
__device__ __forceinline__ float clamp_mask(float x) { return (x > kLvMin && x < kLvMax) ? 1.0f : 0.0f; }

// Normals n[4 j .. 4 j + 3] of Philox block c0 + j: Box-Muller on the word
// pairs (0, 1) and (2, 3).
__device__ __forceinline__ void normals4(const Rng& r, uint32_t c0, float* n) {
    const uint4 w = r.block(c0);
    box_muller(u01(w.x), u01(w.y), n[0], n[1]);
    box_muller(u01(w.z), u01(w.w), n[2], n[3]);
}

// ---------------------------------------------------------------------------
// init

struct LayerDims {
    int n_in, n_out;
};

// Feature blocks per layer dimension: every layer is stored and computed as
// a (16 T) x (16 T) grid of 16 x 16 MFMA tiles, T = 1 when all of the
// network's widths (hidden units, both networks' inputs and outputs) fit one
// tile and T = 2 up to 32 (Table 1's widest settings: 20 hidden units, or
// 2 x 9 encoder outputs).
__host__ __device__ inline int shape_blocks(const Shape& s) {
    int m = s.width;
    m = m > s.p_out + s.p_in ? m : s.p_out + s.p_in;
    m = m > s.latent + s.p_in ? m : s.latent + s.p_in;
    m = m > 2 * s.p_out ? m : 2 * s.p_out;
    m = m > 2 * s.latent ? m : 2 * s.latent;
    return m <= kTile ? 1 : 2;
}
// Floats of one layer: (16 T)^2 row-major weights, then 16 T biases.
__host__ __device__ inline int layer_floats(const Shape& s) {
    const int S = kTile * shape_blocks(s);
    return S * S + S;
}
constexpr int kMaxBlocks = 2;
constexpr int kMaxLayerFloats = (kTile * kMaxBlocks) * (kTile * kMaxBlocks) + kTile * kMaxBlocks;
__host__ __device__ inline LayerDims layer_dims(const Shape& s, int layer) {
    const int nl = s.n_linear;
    const bool dec = layer >= nl;
    const int j = dec ? layer - nl : layer;
    const int in0 = dec ? s.latent + s.p_in : s.p_out + s.p_in;
    const int outl = dec ? 2 * s.p_out : 2 * s.latent;
    return LayerDims{j == 0 ? in0 : s.width, j == nl - 1 ? outl : s.width};
}

__global__ void cvae_init_kernel(Shape s, uint64_t seed, float* master, int n_params) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_params) return;
    const int lf = layer_floats(s), S = kTile * shape_blocks(s);
    const int layer = p / lf, flat = p % lf;
    const LayerDims d = layer_dims(s, layer);
    int row, col;
    if (flat < S * S) {
        row = flat / S;
        col = flat % S;
    } else {
        row = flat - S * S;
        col = 0;
    }
    float v = 0.0f;
    if (row < d.n_out && col < d.n_in) {
        const Rng r = make_rng(seed, MS_TAG_CVAE_INIT, (uint64_t)s.model);
        const uint4 w = r.block((uint32_t)p >> 2);
        const uint32_t word = (p & 3) == 0 ? w.x : (p & 3) == 1 ? w.y : (p & 3) == 2 ? w.z : w.w;
        v = (2.0f * u01(word) - 1.0f) / sqrtf((float)d.n_in);
    }
    master[p] = v;
}

// ---------------------------------------------------------------------------
// features (Sec. 4.2 model inputs; LengthGen target dequantised)

__global__ void cvae_features_kernel(int model, int64_t n_out, const int64_t* rows, int64_t n, const float* params3,
                                     const uint32_t* n_scatter, const float* exit_param, const float* event_pos,
                                     const float* event_dir, uint64_t seed, uint64_t id_offset, const double* stats,
                                     float* cond, float* target) {
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n_out;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = rows ? rows[o] : o;
        const float lst = logf(params3[i]), g = params3[n + i], phi = params3[2 * n + i];
        const float N = (float)n_scatter[i];
        float c[7], y[6];
        int pc, py;
        if (model == MS_MODEL_LENGTH) {
            const Rng r = make_rng(seed, MS_TAG_DEQUANT, id_offset + (uint64_t)i);
            const float u = u01(r.block(0).x);
            c[0] = lst;
            c[1] = g;
            y[0] = logf(N + u - 0.5f);
            pc = 2;
            py = 1;
        } else if (model == MS_MODEL_PATH) {
            c[0] = lst;
            c[1] = g;
            c[2] = logf(N);
            for (int k = 0; k < 3; ++k) y[k] = exit_param[k * n + i];
            pc = 3;
            py = 3;
        } else {
            c[0] = lst;
            c[1] = g;
            c[2] = phi;
            for (int k = 0; k < 3; ++k) c[3 + k] = exit_param[k * n + i];
            c[6] = logf(N);
            for (int k = 0; k < 3; ++k) {
                y[k] = event_pos[k * n + i];
                y[3 + k] = event_dir[k * n + i];
            }
            pc = 7;
            py = 6;
        }
        if (stats) {
            for (int k = 0; k < pc; ++k) c[k] = (float)((c[k] - stats[k]) / stats[16 + k]);
            for (int k = 0; k < py; ++k) y[k] = (float)((y[k] - stats[32 + k]) / stats[48 + k]);
        }
        for (int k = 0; k < pc; ++k) cond[o * pc + k] = c[k];
        for (int k = 0; k < py; ++k) target[o * py + k] = y[k];
    }
}

// ---------------------------------------------------------------------------
// deterministic row selection (stream compaction in index order)

constexpr int kSelPerBlock = 2048;  // 256 threads x 8 consecutive rows

__device__ __forceinline__ bool row_selected(int64_t i, int64_t n, const uint32_t* ns, const uint32_t* ek,
                                             uint32_t min_n, uint32_t min_k) {
    return i < n && ns[i] >= min_n && (ek == nullptr || ek[i] >= min_k);
}

__global__ void select_count_kernel(int64_t n, const uint32_t* ns, const uint32_t* ek, uint32_t min_n,
                                    uint32_t min_k, int64_t* block_count) {
    __shared__ int red[256];
    const int64_t base = blockIdx.x * (int64_t)kSelPerBlock + threadIdx.x * 8;
    int c = 0;
    for (int j = 0; j < 8; ++j) c += row_selected(base + j, n, ns, ek, min_n, min_k);
    red[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_count[blockIdx.x] = red[0];
}

__global__ void select_scan_kernel(int64_t nb, int64_t* block_count, int64_t* total) {
    if (threadIdx.x != 0) return;
    int64_t acc = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t c = block_count[b];
        block_count[b] = acc;
        acc += c;
    }
    *total = acc;
}

__global__ void select_write_kernel(int64_t n, const uint32_t* ns, const uint32_t* ek, uint32_t min_n,
                                    uint32_t min_k, const int64_t* block_offset, int64_t* rows) {
    __shared__ int wave_sum[4];
    const int64_t base = blockIdx.x * (int64_t)kSelPerBlock + threadIdx.x * 8;
    bool f[8];
    int c = 0;
    for (int j = 0; j < 8; ++j) {
        f[j] = row_selected(base + j, n, ns, ek, min_n, min_k);
        c += f[j];
    }
    // exclusive prefix of c over the block: within the wave, then across waves
    int incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane_id() >= off) incl += v;
    }
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 63) wave_sum[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wave_sum[w];
    int64_t pos = block_offset[blockIdx.x] + before + incl - c;
    for (int j = 0; j < 8; ++j)
        if (f[j]) rows[pos++] = base + j;
}

// ---------------------------------------------------------------------------
// FP64 column moments: deterministic two-pass (mean, then centred squares).

constexpr int kMomBlocks = 256;

__global__ void moments_partial_kernel(const float* x, int64_t n, int dim, const double* mean, double* partial) {
    __shared__ double red[256][16];
    double acc[16];
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < dim; ++k) {
            double v = (double)x[i * dim + k];
            if (mean) {
                v -= mean[k];
                v *= v;
            }
            acc[k] += v;
        }
    }
    for (int k = 0; k < 16; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < dim; ++k) red[threadIdx.x][k] += red[threadIdx.x + off][k];
        __syncthreads();
    }
    if (threadIdx.x < dim) partial[blockIdx.x * 16 + threadIdx.x] = red[0][threadIdx.x];
}

__global__ void moments_final_kernel(const double* partial, int nblocks, int64_t n, int dim, double* out,
                                     int second_pass) {
    const int k = threadIdx.x;
    if (k >= dim) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[b * 16 + k];
    if (!second_pass) out[k] = s / (double)n;
    else out[16 + k] = sqrt(s / (double)n);
}

// ---------------------------------------------------------------------------
// Training: fused forward + backward of encoder and decoder on 16-sample
// tiles, one tile at a time per wave; per-block gradient partials.

struct TrainArgs {
    Shape s;
    const float* master;
    const float* cond;
    const float* target;
    int64_t n_rows;
    int batch;
    int sample_rows;
    uint64_t seed;
    int64_t step;
    uint64_t id_offset;
    float kl_weight;      // weight of the KL term in the gradient
    float* partial;       // [blocks][n_params]
    double* loss_partial; // [blocks][2]
};

// Per-wave LDS: inputs of the 2 NL layers and two work buffers, each 16 T
// feature rows (T stacked 16 x 16 tiles) of 16 samples.
template <int T>
struct WaveLds {
    float act[2 * kMaxNL][kTile * kTile * T];
    float work[2][kTile * kTile * T];
};

// Weight fragments of block (o, k) of a layer with row stride 16 T: the A
// operand of the forward product (output rows 16 o .., input columns
// 16 k ..), its transpose (for dX = W^T dPre) and the biases of output block o.
template <int T>
__device__ __forceinline__ bf16x4 w_frag(const float* layer, int o, int k) {
    constexpr int S = kTile * T;
    const f32x4 v = *reinterpret_cast<const f32x4*>(layer + (kTile * o + frag_row()) * S + kTile * k + frag_k0());
    return to_bf16x4(v);
}
template <int T>
__device__ __forceinline__ bf16x4 wt_frag(const float* layer, int o, int k) {
    constexpr int S = kTile * T;
    const float* p = layer + (kTile * o + frag_k0()) * S + kTile * k + frag_row();
    return to_bf16x4(p[0], p[S], p[2 * S], p[3 * S]);
}
template <int T>
__device__ __forceinline__ f32x4 bias_d(const float* layer, int o) {
    constexpr int S = kTile * T;
    const float* b = layer + S * S + kTile * o + frag_k0();
    return f32x4{b[0], b[1], b[2], b[3]};
}

// Forward of one net (NL layers starting at FIRST) from act[FIRST]; the last
// layer's output blocks go to `out`.  Hidden units at or beyond `width` do
// not exist: their activations are forced to 0, so their (zero-initialised)
// weights and biases receive zero gradients.
template <int FIRST, int NL, int T>
__device__ __forceinline__ void net_forward(const bf16x4 (*wf)[T][T], const f32x4 (*bs)[T], WaveLds<T>& L,
                                            f32x4 (*pre)[T], int width, f32x4* out) {
    const int k0 = frag_k0();
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const int layer = FIRST + j;
        bf16x4 x[T];
#pragma unroll
        for (int k = 0; k < T; ++k) x[k] = to_bf16x4(tile_load_d(L.act[layer] + kTile * kTile * k));
#pragma unroll
        for (int o = 0; o < T; ++o) {
            f32x4 acc = bs[layer][o];
#pragma unroll
            for (int k = 0; k < T; ++k) acc = mfma_bf16(wf[layer][o][k], x[k], acc);
            pre[layer][o] = acc;
            out[o] = acc;
        }
        if (j < NL - 1) {
#pragma unroll
            for (int o = 0; o < T; ++o) {
                f32x4 a;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    a[q] = kTile * o + k0 + q < width ? bf16_round(softplus(pre[layer][o][q])) : 0.0f;
                tile_store_d(L.act[layer + 1] + kTile * kTile * o, a);
            }
            wave_sync();
        }
    }
}

// Backward of one net given d loss / d (last linear output) in D layout.
// Accumulates dW (D layout: row = output unit, column = input unit) and db,
// and writes d loss / d (input of the first layer) in D layout to dx.
template <int FIRST, int NL, int T>
__device__ __forceinline__ void net_backward(const bf16x4 (*wt)[T][T], WaveLds<T>& L, const f32x4 (*pre)[T],
                                             f32x4* dpre, f32x4 (*dw)[T][T], f32x4 (*db)[T], f32x4* dx) {
#pragma unroll
    for (int j = NL - 1; j >= 0; --j) {
        const int layer = FIRST + j;
#pragma unroll
        for (int o = 0; o < T; ++o) {
            db[layer][o] += dpre[o];
            // dW += dPre X^T: both operands read transposed from LDS
            tile_store_d(L.work[0] + kTile * kTile * o, f32x4{bf16_round(dpre[o][0]), bf16_round(dpre[o][1]),
                                                               bf16_round(dpre[o][2]), bf16_round(dpre[o][3])});
        }
        wave_sync();
#pragma unroll
        for (int o = 0; o < T; ++o) {
            const bf16x4 a = to_bf16x4(tile_load_t(L.work[0] + kTile * kTile * o));
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const bf16x4 b = to_bf16x4(tile_load_t(L.act[layer] + kTile * kTile * k));
                dw[layer][o][k] = mfma_bf16(a, b, dw[layer][o][k]);
            }
        }
        wave_sync();
        // dX = W^T dPre
#pragma unroll
        for (int k = 0; k < T; ++k) {
            f32x4 acc = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int o = 0; o < T; ++o) acc = mfma_bf16(wt[layer][o][k], to_bf16x4(dpre[o]), acc);
            dx[k] = acc;
        }
        if (j > 0) {
#pragma unroll
            for (int k = 0; k < T; ++k) {
#pragma unroll
                for (int q = 0; q < 4; ++q) dpre[k][q] = dx[k][q] * sigmoid(pre[layer - 1][k][q]);
            }
        }
    }
}

template <int NL, int T>
__global__ __launch_bounds__(256) void cvae_train_kernel(const TrainArgs a) {
    constexpr int TT = kTile * kTile * T;  // floats of one activation buffer
    constexpr int S = kTile * T;           // row stride of a layer's weights
    constexpr int LF = S * S + S;          // floats per layer
    constexpr int kLat = 8 * T;            // latent sizes up to 8 T (2 L <= 16 T)
    __shared__ WaveLds<T> lds_all[kTrainWaves];
    const int wave = threadIdx.x >> 6;
    WaveLds<T>& L = lds_all[wave];
    const Shape s = a.s;
    constexpr int nl = NL;
    const int P = s.p_out, Lt = s.latent, C = s.p_in;
    const int lane = lane_id();
    const float inv_b = 1.0f / (float)a.batch;

    // all layers' weight fragments (both orientations) and biases of this
    // lane, loaded once: the tile loop is a chain of dependent steps
    bf16x4 wf[2 * NL][T][T], wt[2 * NL][T][T];
    f32x4 bs[2 * NL][T];
#pragma unroll
    for (int i = 0; i < 2 * NL; ++i) {
        const float* layer = a.master + i * LF;
#pragma unroll
        for (int o = 0; o < T; ++o) {
            bs[i][o] = bias_d<T>(layer, o);
#pragma unroll
            for (int k = 0; k < T; ++k) {
                wf[i][o][k] = w_frag<T>(layer, o, k);
                wt[i][o][k] = wt_frag<T>(layer, o, k);
            }
        }
    }
    f32x4 dw[2 * NL][T][T], db[2 * NL][T], pre[2 * NL][T];
#pragma unroll
    for (int i = 0; i < 2 * NL; ++i) {
#pragma unroll
        for (int o = 0; o < T; ++o) {
            db[i][o] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < T; ++k) dw[i][o][k] = f32x4{0, 0, 0, 0};
        }
    }
    double kl_acc = 0.0, nll_acc = 0.0;

    const int n_tiles = a.batch / kTile;
    const int wave_global = blockIdx.x * kTrainWaves + wave;
    const int n_waves = gridDim.x * kTrainWaves;
    for (int tile = wave_global; tile < n_tiles; tile += n_waves) {
        const int b = tile * kTile + (lane & 15);  // sample of this lane's column
        // zero the two input buffers, then gather (target, cond) rows
        for (int q = lane; q < TT; q += 64) {
            L.act[0][q] = 0.0f;
            L.act[nl][q] = 0.0f;
        }
        wave_sync();
        float mu_z[kLat], lv_z[kLat], lvr_z[kLat], eps[kLat];
        if (lane < 16) {
            int64_t row = b;
            if (a.sample_rows) {
                const Rng rb = make_rng(a.seed, MS_TAG_CVAE_BATCH, (uint64_t)b);
                row = (int64_t)(((uint64_t)rb.block((uint32_t)a.step).x * (uint64_t)a.n_rows) >> 32);
            }
            for (int k = 0; k < P; ++k) L.act[0][k * kTile + lane] = bf16_round(a.target[row * P + k]);
            for (int k = 0; k < C; ++k) {
                const float cv = bf16_round(a.cond[row * C + k]);
                L.act[0][(P + k) * kTile + lane] = cv;
                L.act[nl][(Lt + k) * kTile + lane] = cv;
            }
        }
        wave_sync();
        // encoder
        f32x4 oe[T];
        net_forward<0, NL, T>(wf, bs, L, pre, s.width, oe);
#pragma unroll
        for (int o = 0; o < T; ++o) tile_store_d(L.work[0] + kTile * kTile * o, oe[o]);
        wave_sync();
        if (lane < 16) {
            const Rng rr = make_rng(a.seed, MS_TAG_CVAE_REPARAM, a.id_offset + (uint64_t)b);
            for (int j = 0; 4 * j < Lt; ++j) normals4(rr, (uint32_t)(4 * a.step + j), eps + 4 * j);
            float kl = 0.0f;
            for (int i = 0; i < Lt; ++i) {
                mu_z[i] = L.work[0][i * kTile + lane];
                lvr_z[i] = L.work[0][(Lt + i) * kTile + lane];
                lv_z[i] = clamp_lv(lvr_z[i]);
                const float z = __builtin_fmaf(fast_exp(0.5f * lv_z[i]), eps[i], mu_z[i]);
                L.act[nl][i * kTile + lane] = bf16_round(z);
                kl += 0.5f * (mu_z[i] * mu_z[i] + fast_exp(lv_z[i]) - lv_z[i] - 1.0f);
            }
            kl_acc += (double)kl;
        }
        wave_sync();
        // decoder
        f32x4 od[T];
        net_forward<NL, NL, T>(wf, bs, L, pre, s.width, od);
#pragma unroll
        for (int o = 0; o < T; ++o) tile_store_d(L.work[0] + kTile * kTile * o, od[o]);
        for (int q = lane; q < TT; q += 64) L.work[1][q] = 0.0f;
        wave_sync();
        if (lane < 16) {
            int64_t row = b;
            if (a.sample_rows) {
                const Rng rb = make_rng(a.seed, MS_TAG_CVAE_BATCH, (uint64_t)b);
                row = (int64_t)(((uint64_t)rb.block((uint32_t)a.step).x * (uint64_t)a.n_rows) >> 32);
            }
            float nll = 0.0f;
            for (int k = 0; k < P; ++k) {
                const float mu = L.work[0][k * kTile + lane];
                const float lvr = L.work[0][(P + k) * kTile + lane];
                const float lv = clamp_lv(lvr);
                const float y = a.target[row * P + k];
                const float r = y - mu, iv = fast_exp(-lv);
                nll += 0.5f * (kLog2Pi + lv + r * r * iv);
                L.work[1][k * kTile + lane] = -r * iv * inv_b;
                L.work[1][(P + k) * kTile + lane] = 0.5f * (1.0f - r * r * iv) * clamp_mask(lvr) * inv_b;
            }
            nll_acc += (double)nll;
        }
        wave_sync();
        f32x4 dcur[T], dzc[T];
#pragma unroll
        for (int o = 0; o < T; ++o) dcur[o] = tile_load_d(L.work[1] + kTile * kTile * o);
        net_backward<NL, NL, T>(wt, L, pre, dcur, dw, db, dzc);
#pragma unroll
        for (int o = 0; o < T; ++o) tile_store_d(L.work[0] + kTile * kTile * o, dzc[o]);
        for (int q = lane; q < TT; q += 64) L.work[1][q] = 0.0f;
        wave_sync();
        if (lane < 16) {
            for (int i = 0; i < Lt; ++i) {
                const float dz = L.work[0][i * kTile + lane];
                const float sd = fast_exp(0.5f * lv_z[i]);
                L.work[1][i * kTile + lane] = dz + a.kl_weight * mu_z[i] * inv_b;
                L.work[1][(Lt + i) * kTile + lane] =
                    (0.5f * dz * eps[i] * sd + a.kl_weight * 0.5f * (fast_exp(lv_z[i]) - 1.0f) * inv_b) *
                    clamp_mask(lvr_z[i]);
            }
        }
        wave_sync();
#pragma unroll
        for (int o = 0; o < T; ++o) dcur[o] = tile_load_d(L.work[1] + kTile * kTile * o);
        net_backward<0, NL, T>(wt, L, pre, dcur, dw, db, dzc);
        wave_sync();
    }

    // bias gradients: sum over the 16 sample columns of each lane group
#pragma unroll
    for (int i = 0; i < 2 * nl; ++i) {
#pragma unroll
        for (int o = 0; o < T; ++o) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float v = db[i][o][q];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 8);
                db[i][o][q] = v;
            }
        }
    }
    // block reduction through LDS (reusing the tile space): the waves add
    // their gradients into one buffer one after the other, a fixed order
    const int n_params = 2 * nl * LF;
    float* red = reinterpret_cast<float*>(lds_all);  // [n_params]
    static_assert(sizeof(lds_all) >= sizeof(float) * 2 * kMaxNL * LF, "gradient buffer exceeds the LDS tiles");
    const int c = frag_row(), k0 = frag_k0();
    for (int w = 0; w < kTrainWaves; ++w) {
        __syncthreads();
        if (wave != w) continue;
#pragma unroll
        for (int i = 0; i < 2 * nl; ++i) {
#pragma unroll
            for (int o = 0; o < T; ++o) {
#pragma unroll
                for (int k = 0; k < T; ++k) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float& dst = red[i * LF + (kTile * o + k0 + q) * S + kTile * k + c];
                        dst = w == 0 ? dw[i][o][k][q] : dst + dw[i][o][k][q];
                    }
                }
                if (c == 0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float& dst = red[i * LF + S * S + kTile * o + k0 + q];
                        dst = w == 0 ? db[i][o][q] : dst + db[i][o][q];
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < n_params; p += blockDim.x) a.partial[(int64_t)blockIdx.x * n_params + p] = red[p];
    // loss partials: lanes 0..15 of each wave hold sums
    __syncthreads();
    double* dred = reinterpret_cast<double*>(lds_all);
    if (lane < 16) {
        dred[(wave * 16 + lane) * 2 + 0] = kl_acc;
        dred[(wave * 16 + lane) * 2 + 1] = nll_acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double k = 0.0, n = 0.0;
        for (int i = 0; i < kTrainWaves * 16; ++i) {
            k += dred[i * 2 + 0];
            n += dred[i * 2 + 1];
        }
        a.loss_partial[blockIdx.x * 2 + 0] = k;
        a.loss_partial[blockIdx.x * 2 + 1] = n;
    }
}

struct AdamArgs {
    int n_params, n_blocks, batch;
    const float* partial;
    const double* loss_partial;
    float* master;
    float* m;
    float* v;
    float* grad_out;
    double* loss_out;
    int do_update;
    float lr, beta1, beta2, one_m_beta1, one_m_beta2, eps, wd, bc1, bc2;
};

// Gradient = sum of the per-block partials, then the AdamW update.  The sum
// over blocks is latency-bound (one dependent load per block), so each block
// of this kernel takes 32 parameters x 8 groups of partial blocks: group q adds
// blocks q, q + 8, ... with its loads in flight together, and the 8 group sums
// are added in fixed order.  The loss partials are reduced by wave 0 of block 0
// with a fixed butterfly.
constexpr int kAdamParams = 32, kAdamGroups = 8;

__global__ __launch_bounds__(256) void cvae_adam_kernel(const AdamArgs a) {
    __shared__ float red[kAdamGroups][kAdamParams];
    const int pl = threadIdx.x % kAdamParams, grp = threadIdx.x / kAdamParams;
    const int p = blockIdx.x * kAdamParams + pl;
    float part = 0.0f;
    if (p < a.n_params) {
#pragma unroll 8
        for (int b = grp; b < a.n_blocks; b += kAdamGroups) part += a.partial[(int64_t)b * a.n_params + p];
    }
    red[grp][pl] = part;
    __syncthreads();
    if (grp == 0 && p < a.n_params) {
        float g = 0.0f;
#pragma unroll
        for (int q = 0; q < kAdamGroups; ++q) g += red[q][pl];
        if (a.grad_out) a.grad_out[p] = g;
        if (a.do_update) {
            const float m = a.beta1 * a.m[p] + a.one_m_beta1 * g;
            const float v = a.beta2 * a.v[p] + a.one_m_beta2 * g * g;
            a.m[p] = m;
            a.v[p] = v;
            const float mh = m / a.bc1, vh = v / a.bc2;
            const float th = a.master[p];
            a.master[p] = th - a.lr * (mh / (sqrtf(vh) + a.eps) + a.wd * th);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 64 && a.loss_out) {
        double k = 0.0, n = 0.0;
        for (int b = threadIdx.x; b < a.n_blocks; b += 64) {
            k += a.loss_partial[b * 2 + 0];
            n += a.loss_partial[b * 2 + 1];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            k += __shfl_xor(k, off);
            n += __shfl_xor(n, off);
        }
        if (threadIdx.x == 0) {
            a.loss_out[0] = (k + n) / a.batch;
            a.loss_out[1] = k / a.batch;
            a.loss_out[2] = n / a.batch;
        }
    }
}

// ---------------------------------------------------------------------------
// pack

__device__ __forceinline__ uint32_t fp8_e4m3_bits(float x) {
    // OCP E4M3: bias 7, 3 mantissa bits, max 448, round to nearest even,
    // saturating.
    const uint32_t sign = x < 0.0f ? 0x80u : 0u;
    float a = __builtin_fabsf(x);
    if (!(a == a)) return 0x7fu | sign;
    if (a >= 448.0f) return 0x7eu | sign;
    if (a < 0x1p-10f) return sign;  // rounds to zero (half of the smallest subnormal 2^-9)
    int e;
    frexpf(a, &e);
    int eu = e - 1;
    if (eu < -6) eu = -6;
    const float q = ldexpf(1.0f, eu - 3);
    float m = rintf(a / q);  // ties to even
    float v = m * q;
    if (v > 448.0f) v = 448.0f;
    // encode v
    if (v < 0x1p-6f) return sign | (uint32_t)(v / 0x1p-9f);
    int ev;
    frexpf(v, &ev);
    const int eb = ev - 1 + 7;
    const uint32_t mant = (uint32_t)((v / ldexpf(1.0f, ev - 1) - 1.0f) * 8.0f + 0.5f);
    return sign | ((uint32_t)eb << 3) | (mant & 7u);
}

// FP8 activation scales from calibration rows (one block of 256 threads):
// decoder layer j's inputs a_j, computed in FP32 from the master weights for
// every row i < n -- the standardised condition cond[i] after the latent z,
// z the first `latent` normals of the sampler's stream for seed 0 and id i
// -- give s_j, the smallest power of two with max_i |a_j| / s_j <= 448 (the
// largest E4M3 value; 1 where the maximum is 0).  Writes in_scale = 1 / s_j;
// cvae_pack_kernel then folds s_j into out_scale.
__global__ __launch_bounds__(256) void cvae_calib_kernel(Shape s, const float* master, const double* stats,
                                                         const float* cond, int64_t n, PackedModel* pm) {
    const int nl = s.n_linear, L = s.latent, C = s.p_in;
    const int S = kTile * shape_blocks(s), lf = layer_floats(s);
    float mx[kMaxLayers] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        float a[2 * kTile], nrm[2 * kTile];
        const Rng r = make_rng(0, MS_TAG_CVAE_SAMPLE, (uint64_t)i);
        for (int j = 0; 4 * j < L; ++j) normals4(r, (uint32_t)j, nrm + 4 * j);
        for (int k = 0; k < 2 * kTile; ++k) a[k] = 0.0f;
        for (int k = 0; k < L; ++k) a[k] = nrm[k];
        for (int k = 0; k < C; ++k) a[L + k] = (float)((cond[i * C + k] - stats[k]) / stats[16 + k]);
        for (int j = 0; j < nl; ++j) {
            const LayerDims d = layer_dims(s, nl + j);
            for (int k = 0; k < d.n_in; ++k) mx[j] = fmaxf(mx[j], fabsf(a[k]));
            if (j == nl - 1) break;
            const float* layer = master + (nl + j) * lf;
            float o[2 * kTile];
            for (int row = 0; row < d.n_out; ++row) {
                float acc = layer[S * S + row];
                for (int k = 0; k < d.n_in; ++k) acc = fmaf(layer[row * S + k], a[k], acc);
                o[row] = softplus(acc);
            }
            for (int k = 0; k < 2 * kTile; ++k) a[k] = k < d.n_out ? o[k] : 0.0f;
        }
    }
    __shared__ float red[kMaxLayers][256];
    for (int j = 0; j < kMaxLayers; ++j) red[j][threadIdx.x] = mx[j];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int j = 0; j < kMaxLayers; ++j) red[j][threadIdx.x] = fmaxf(red[j][threadIdx.x], red[j][threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x < kMaxLayers) {
        const float m = red[threadIdx.x][0];
        float inv = 1.0f;
        if (m > 0.0f) {
            int e;
            const float f = frexpf(m / 448.0f, &e);  // m / 448 = f 2^e, f in [0.5, 1)
            inv = ldexpf(1.0f, -(f == 0.5f ? e - 1 : e));
        }
        pm->in_scale[threadIdx.x] = inv;
    }
}

// With `calibrated`, in_scale was written by cvae_calib_kernel earlier on the
// same stream; otherwise activations enter E4M3 unscaled.
__global__ void cvae_pack_kernel(Shape s, const float* master, const double* stats, int precision, bool calibrated,
                                 PackedModel* pm) {
    const int lane = threadIdx.x;  // 64 threads
    const int nl = s.n_linear;
    const int T = shape_blocks(s), S = kTile * T, lf = layer_floats(s);
    if (lane == 0) {
        pm->magic = (int32_t)kPackedMagic;
        pm->model = s.model;
        pm->p_in = s.p_in;
        pm->p_out = s.p_out;
        pm->latent = s.latent;
        pm->width = s.width;
        pm->n_linear = nl;
        pm->precision = precision;
        pm->blocks = T;
        pm->pad_[0] = pm->pad_[1] = pm->pad_[2] = 0;
    }
    if (lane < 16) {
        pm->mean_c[lane] = stats ? (float)stats[lane] : 0.0f;
        pm->inv_std_c[lane] = stats ? (float)(1.0 / stats[16 + lane]) : 1.0f;
        pm->mean_y[lane] = stats ? (float)stats[32 + lane] : 0.0f;
        pm->std_y[lane] = stats ? (float)stats[48 + lane] : 1.0f;
    }
    __shared__ float smax[64];
    for (int j = 0; j < kMaxLayers; ++j) {
        const bool real = j < nl;
        const float* layer = master + (nl + (real ? j : 0)) * lf;
        float scale = 1.0f;
        if (precision == MS_PREC_FP8) {
            float mx = 0.0f;
            for (int q = lane; q < S * S; q += 64) mx = fmaxf(mx, real ? fabsf(layer[q]) : 0.0f);
            smax[lane] = mx;
            __syncthreads();
            for (int off = 32; off > 0; off >>= 1) {
                if (lane < off) smax[lane] = fmaxf(smax[lane], smax[lane + off]);
                __syncthreads();
            }
            scale = smax[0] > 0.0f ? smax[0] / 448.0f : 1.0f;
            __syncthreads();
        }
        if (lane == 0) {
            const float in_sc = precision == MS_PREC_FP8 && calibrated ? pm->in_scale[j] : 1.0f;
            pm->in_scale[j] = in_sc;
            pm->out_scale[j] = scale / in_sc;  // s_w s_a, exact: s_a is a power of two
        }
        if (lane < 2 * kTile) {
            const float b = real && lane < S ? layer[S * S + lane] : 0.0f;
            if (lane < kTile) pm->bias[j][lane] = b;
            else pm->bias_hi[j][lane - kTile] = b;
        }
        const int r = lane & 15, kg = lane >> 4;
        for (int ti = 0; ti < 4; ++ti) {
            uint32_t w0 = 0, w1 = 0;
            if (real && precision == MS_PREC_FP8 && ti < T) {
                // K = 32 operand in the permuted order of the FP8 decoders:
                // bytes 0..3 = columns 4 kg .. 4 kg + 3 of input block 0,
                // bytes 4..7 = the same columns of input block 1 (0 when
                // the layer has one block)
                const float* row = layer + (kTile * ti + r) * S + 4 * kg;
                uint32_t lo[4], hi[4];
                for (int q = 0; q < 4; ++q) {
                    lo[q] = fp8_e4m3_bits(row[q] / scale);
                    hi[q] = T == 2 ? fp8_e4m3_bits(row[kTile + q] / scale) : 0u;
                }
                w0 = lo[0] | (lo[1] << 8) | (lo[2] << 16) | (lo[3] << 24);
                w1 = hi[0] | (hi[1] << 8) | (hi[2] << 16) | (hi[3] << 24);
            } else if (real && precision != MS_PREC_FP8 && ti < T * T) {
                const int o = ti >> 1, k = ti & 1;
                const float* row = layer + (kTile * o + r) * S + kTile * k + 4 * kg;
                w0 = (uint32_t)bf16_bits(row[0]) | ((uint32_t)bf16_bits(row[1]) << 16);
                w1 = (uint32_t)bf16_bits(row[2]) | ((uint32_t)bf16_bits(row[3]) << 16);
            }
            uint32_t* dst = ti == 0 ? pm->frag[j][lane] : pm->frag_hi[j][ti - 1][lane];
            dst[0] = w0;
            dst[1] = w1;
        }
    }
}

// ---------------------------------------------------------------------------
// decoder-only sampling: 64 paths per wave = four 16-path MFMA tiles

constexpr int kSampleWaves = 4;

template <int T>
struct SampleLds {
    float x[64][kTile * T];
    float o[64][kTile * T];
};

// T: tiles per layer dimension of the packed model (pm->blocks).
template <int T>
__global__ __launch_bounds__(256) void cvae_sample_kernel(const PackedModel* pm, const float* cond, int64_t n,
                                                          uint64_t seed, uint64_t id_offset, float* out) {
    if ((pm->blocks == 2) != (T == 2)) return;
    __shared__ SampleLds<T> lds_all[kSampleWaves];
    SampleLds<T>& L = lds_all[threadIdx.x >> 6];
    const int lane = lane_id();
    const int P = pm->p_out, Lt = pm->latent, C = pm->p_in;
    const int64_t n_chunks = (n + 63) / 64;
    const int64_t wave_global = blockIdx.x * (int64_t)kSampleWaves + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * kSampleWaves;
    const bool three = pm->n_linear == kDecLayers;
    const DecoderRegs w = load_decoder(pm);
    const bool fp8 = pm->precision == MS_PREC_FP8;
    for (int64_t chunk = wave_global; chunk < n_chunks; chunk += n_waves) {
        const int64_t i = chunk * 64 + lane;
        const bool valid = i < n;
        float nrm[kTile * T];  // latent + p_out <= 16 T normals
        for (int q = 0; q < kTile * T; ++q) L.x[lane][q] = 0.0f;
        if (valid) {
            const Rng r = make_rng(seed, MS_TAG_CVAE_SAMPLE, id_offset + (uint64_t)i);
            for (int j = 0; 4 * j < Lt + P; ++j) normals4(r, (uint32_t)j, nrm + 4 * j);
            for (int q = 0; q < Lt; ++q) L.x[lane][q] = nrm[q];
            for (int k = 0; k < C; ++k) L.x[lane][Lt + k] = (cond[i * C + k] - pm->mean_c[k]) * pm->inv_std_c[k];
        }
        wave_sync();
        const int64_t remaining = n - chunk * 64;
        const int n_tiles = remaining >= 64 ? 4 : (int)((remaining + 15) / 16);
        for (int t = 0; t < n_tiles; ++t) {
            const int path = 16 * t + frag_row();
            if constexpr (T == 1) {
                const f32x4 xin = *reinterpret_cast<const f32x4*>(&L.x[path][frag_k0()]);
                const f32x4 o = !three ? decoder_tile_layers(pm, xin) : fp8 ? decoder_tile_fp8(w, xin)
                                                                            : decoder_tile(w, xin);
                *reinterpret_cast<f32x4*>(&L.o[path][frag_k0()]) = o;
            } else {
                const f32x4 xin[2] = {*reinterpret_cast<const f32x4*>(&L.x[path][frag_k0()]),
                                      *reinterpret_cast<const f32x4*>(&L.x[path][kTile + frag_k0()])};
                f32x4 o[2];
                decoder_tile_wide(pm, xin, o);
                *reinterpret_cast<f32x4*>(&L.o[path][frag_k0()]) = o[0];
                *reinterpret_cast<f32x4*>(&L.o[path][kTile + frag_k0()]) = o[1];
            }
        }
        wave_sync();
        if (valid) {
            for (int k = 0; k < P; ++k) {
                const float mu = L.o[lane][k];
                const float lv = clamp_lv(L.o[lane][P + k]);
                const float y = __builtin_fmaf(fast_exp(0.5f * lv), nrm[Lt + k], mu);
                out[i * P + k] = __builtin_fmaf(y, pm->std_y[k], pm->mean_y[k]);
            }
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------

static ms_status check_shape(const ms_cvae_shape* sh, Shape* out) {
    MS_REQUIRE(sh != nullptr, "CVAE shape is NULL");
    MS_REQUIRE(sh->model >= 0 && sh->model <= 2, "CVAE model must be 0, 1 or 2");
    MS_REQUIRE(sh->p_in >= 1 && sh->p_out >= 1 && sh->latent >= 1 && sh->width >= 1, "CVAE sizes must be positive");
    if (sh->width > 32 || sh->p_out + sh->p_in > 32 || sh->latent + sh->p_in > 32 || 2 * sh->p_out > 32 ||
        2 * sh->latent > 32 || sh->p_in > 16 || sh->n_linear < 2 || sh->n_linear > kMaxNL)
        return set_error(MS_ERR_UNSUPPORTED,
                         "CVAE shape unsupported: needs width <= 32, 2 <= n_linear <= 4, p_in <= 16, "
                         "p_out + p_in <= 32, latent + p_in <= 32, 2 p_out <= 32, 2 latent <= 32");
    *out = Shape{sh->model, sh->p_in, sh->p_out, sh->latent, sh->width, sh->n_linear};
    return MS_OK;
}

constexpr int kMaxTrainBatch = 1 << 20;
constexpr int kMaxTrainWaveCount = 1024;

constexpr int train_blocks(int batch) {
    return ((batch / kTile < kMaxTrainWaveCount ? batch / kTile : kMaxTrainWaveCount) + kTrainWaves - 1) /
           kTrainWaves;
}

// Scratch of one training step: per-block gradient partials [blocks][params]
// (FP32), then per-block loss partials [blocks][2] (FP64).  Every block
// writes all of its partials on every step, so nothing needs clearing.
constexpr size_t train_partial_bytes(int nb, int n_params) {
    return ((size_t)nb * n_params * sizeof(float) + 255) / 256 * 256;
}
constexpr size_t train_scratch_bytes(int nb, int n_params) {
    return train_partial_bytes(nb, n_params) + (size_t)nb * 2 * sizeof(double);
}

// Device-resident scratch of cvae_train_step_noalloc, sized for the largest
// batch and network the training kernels accept (about 8.7 MB); each device
// holds its own copy for the life of the process.  Host code must not pass
// this name to a kernel: it is a host-side stand-in, not a device address.
// Its per-device address comes from hipGetSymbolAddress (noalloc_scratch).
constexpr size_t kTrainScratchBytes = train_scratch_bytes(train_blocks(kMaxTrainBatch), 2 * kMaxNL * kMaxLayerFloats);
static __device__ __align__(256) unsigned char scratch[kTrainScratchBytes];

}  // namespace msst

extern "C" {

ms_status cvae_param_count(const ms_cvae_shape* shape, size_t* n_floats) {
    msst::Shape s;
    ms_status st = msst::check_shape(shape, &s);
    if (st != MS_OK) return st;
    MS_REQUIRE(n_floats != nullptr, "cvae_param_count: n_floats is NULL");
    *n_floats = (size_t)(2 * s.n_linear * msst::layer_floats(s));
    return MS_OK;
}

ms_status cvae_init(const ms_cvae_shape* shape, uint64_t seed, float* master_dev, void* stream) {
    using namespace msst;
    Shape s;
    ms_status st = check_shape(shape, &s);
    if (st != MS_OK) return st;
    MS_REQUIRE(master_dev != nullptr, "cvae_init: master_dev is NULL");
    int cus;
    if ((st = device_cu_count(&cus)) != MS_OK) return st;
    const int n = 2 * s.n_linear * layer_floats(s);
    hipLaunchKernelGGL(cvae_init_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, s, seed,
                       master_dev, n);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

ms_status cvae_features(int32_t model, int64_t n, const int64_t* rows_dev, int64_t n_records,
                        const float* params3_dev, const uint32_t* n_scatter_dev, const float* exit_param_dev,
                        const float* event_pos_dev, const float* event_dir_dev, uint64_t seed, uint64_t id_offset,
                        const double* stats_dev, float* cond_dev, float* target_dev, void* stream) {
    using namespace msst;
    MS_REQUIRE(model >= 0 && model <= 2, "cvae_features: model must be 0, 1 or 2");
    MS_REQUIRE(n > 0 && n_records > 0, "cvae_features: n and n_records must be positive");
    MS_REQUIRE(rows_dev != nullptr || n <= n_records, "cvae_features: n > n_records without a row list");
    MS_REQUIRE(params3_dev && n_scatter_dev && cond_dev && target_dev, "cvae_features: NULL array");
    MS_REQUIRE(model == 0 || exit_param_dev, "cvae_features: exit_param is required for PathGen and EventGen");
    MS_REQUIRE(model != 2 || (event_pos_dev && event_dir_dev), "cvae_features: event arrays required for EventGen");
    int cus;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;
    int64_t blocks = (n + 255) / 256;
    if (blocks > cus * 8) blocks = cus * 8;
    hipLaunchKernelGGL(cvae_features_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, model, n,
                       rows_dev, n_records, params3_dev, n_scatter_dev, exit_param_dev, event_pos_dev, event_dir_dev,
                       seed, id_offset, stats_dev, cond_dev, target_dev);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

ms_status ms_select_rows_workspace_size(int64_t n, size_t* bytes) {
    MS_REQUIRE(bytes != nullptr && n > 0, "ms_select_rows_workspace_size: need n > 0 and bytes");
    *bytes = (size_t)((n + msst::kSelPerBlock - 1) / msst::kSelPerBlock) * sizeof(int64_t) + 256;
    return MS_OK;
}

ms_status ms_select_rows(int64_t n, const uint32_t* n_scatter_dev, const uint32_t* event_index_dev,
                         uint32_t min_scatter, uint32_t min_event, int64_t* rows_dev, int64_t* count_dev,
                         void* workspace_dev, size_t workspace_bytes, void* stream) {
    using namespace msst;
    MS_REQUIRE(n > 0 && n < ((int64_t)1 << 40), "ms_select_rows: n must be in [1, 2^40)");
    MS_REQUIRE(n_scatter_dev && rows_dev && count_dev && workspace_dev, "ms_select_rows: NULL array");
    size_t need = 0;
    ms_select_rows_workspace_size(n, &need);
    if (workspace_bytes < need) return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "ms_select_rows: workspace needs %zu bytes", need);
    int cus;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;
    const int64_t nb = (n + kSelPerBlock - 1) / kSelPerBlock;
    int64_t* bc = reinterpret_cast<int64_t*>(workspace_dev);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(select_count_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, n_scatter_dev, event_index_dev,
                       min_scatter, min_event, bc);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(64), 0, s, nb, bc, count_dev);
    hipLaunchKernelGGL(select_write_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, n_scatter_dev, event_index_dev,
                       min_scatter, min_event, (const int64_t*)bc, rows_dev);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

ms_status ms_column_moments_workspace_size(int64_t n, int32_t dim, size_t* bytes) {
    MS_REQUIRE(bytes != nullptr, "ms_column_moments_workspace_size: bytes is NULL");
    *bytes = (size_t)msst::kMomBlocks * 16 * sizeof(double);
    return MS_OK;
}

ms_status ms_column_moments(const float* x_dev, int64_t n, int32_t dim, double* out_dev, void* workspace_dev,
                            size_t workspace_bytes, void* stream) {
    using namespace msst;
    MS_REQUIRE(x_dev && out_dev, "ms_column_moments: NULL array");
    MS_REQUIRE(n > 0 && dim >= 1 && dim <= 16, "ms_column_moments: need n > 0 and 1 <= dim <= 16");
    MS_REQUIRE(workspace_dev != nullptr, "ms_column_moments: workspace is NULL");
    if (workspace_bytes < (size_t)kMomBlocks * 16 * sizeof(double))
        return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "ms_column_moments: workspace too small");
    int cus;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    double* partial = reinterpret_cast<double*>(workspace_dev);
    hipLaunchKernelGGL(moments_partial_kernel, dim3(kMomBlocks), dim3(256), 0, s, x_dev, n, dim, (const double*)nullptr,
                       partial);
    hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(64), 0, s, partial, kMomBlocks, n, dim, out_dev, 0);
    hipLaunchKernelGGL(moments_partial_kernel, dim3(kMomBlocks), dim3(256), 0, s, x_dev, n, dim, (const double*)out_dev,
                       partial);
    hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(64), 0, s, partial, kMomBlocks, n, dim, out_dev, 1);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

ms_status cvae_workspace_size(const ms_cvae_shape* shape, int32_t batch, size_t* bytes) {
    using namespace msst;
    Shape s;
    ms_status st = check_shape(shape, &s);
    if (st != MS_OK) return st;
    MS_REQUIRE(bytes != nullptr, "cvae_workspace_size: bytes is NULL");
    MS_REQUIRE(batch > 0 && batch % 16 == 0 && batch <= kMaxTrainBatch, "cvae_workspace_size: batch must be a positive multiple of 16, <= 2^20");
    *bytes = train_scratch_bytes(train_blocks(batch), 2 * s.n_linear * layer_floats(s));
    return MS_OK;
}

}  // extern "C"

namespace msst {

// Address of this device's noalloc scratch, looked up once per device
// (hipGetSymbolAddress with the device current) and kept for the process.
static ms_status noalloc_scratch(void** out) {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = -1;
    MS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(MS_ERR_UNSUPPORTED, "device %d is beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (ptr[dev] == nullptr) {
        void* p = nullptr;
        MS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr) return set_error(MS_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the training scratch");
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return MS_OK;
}

// Validation and launches of one training step on a scratch buffer of at
// least train_scratch_bytes(train_blocks(batch), params) bytes: the caller's
// workspace (ws_dev, ws_bytes), or with `noalloc` this device's scratch
// array, looked up after the arguments have been validated.
static ms_status train_step_launch(const char* who, bool noalloc, const ms_cvae_shape* shape, float* master_dev, float* adam_m_dev,
                                   float* adam_v_dev, const ms_adam* adam, const float* cond_dev,
                                   const float* target_dev, int64_t n_rows, int32_t batch, int32_t sample_rows,
                                   uint64_t seed, int64_t step, uint64_t id_offset, double kl_weight, void* ws_dev,
                                   size_t ws_bytes, double* loss_dev, float* grad_dev, void* stream) {
    Shape s;
    ms_status st = check_shape(shape, &s);
    if (st != MS_OK) return st;
    MS_REQUIRE(master_dev && cond_dev && target_dev, "%s: NULL array", who);
    MS_REQUIRE(batch > 0 && batch % 16 == 0 && batch <= kMaxTrainBatch, "%s: batch must be a positive multiple of 16, <= 2^20", who);
    MS_REQUIRE(n_rows > 0 && n_rows < ((int64_t)1 << 32), "%s: n_rows must be in [1, 2^32)", who);
    MS_REQUIRE(sample_rows || n_rows >= batch, "%s: n_rows < batch without row sampling", who);
    MS_REQUIRE(step >= 0 && step < ((int64_t)1 << 30), "%s: step must be in [0, 2^30)", who);
    MS_REQUIRE(kl_weight >= 0.0 && kl_weight <= 1e6, "%s: kl_weight must be in [0, 1e6]", who);
    if (adam) {
        MS_REQUIRE(adam_m_dev && adam_v_dev, "%s: AdamW moments are NULL", who);
        MS_REQUIRE(adam->step >= 1, "%s: AdamW step must be >= 1", who);
        MS_REQUIRE(adam->lr > 0 && adam->beta1 >= 0 && adam->beta1 < 1 && adam->beta2 >= 0 && adam->beta2 < 1 &&
                       adam->eps > 0 && adam->weight_decay >= 0,
                   "%s: invalid AdamW hyper-parameters", who);
    }
    const int nb = train_blocks(batch);
    const int n_params = 2 * s.n_linear * layer_floats(s);
    const size_t need = train_scratch_bytes(nb, n_params);
    if (!noalloc) {
        MS_REQUIRE(ws_dev != nullptr, "%s: workspace is NULL", who);
        if (ws_bytes < need) return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "%s: workspace needs %zu bytes", who, need);
    }
    int cus;
    if ((st = device_cu_count(&cus)) != MS_OK) return st;
    if (noalloc) {
        if (need > kTrainScratchBytes)
            return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "%s: needs %zu bytes of scratch, the static maximum is %zu",
                             who, need, kTrainScratchBytes);
        if ((st = noalloc_scratch(&ws_dev)) != MS_OK) return st;
    }

    TrainArgs ta{};
    ta.s = s;
    ta.master = master_dev;
    ta.cond = cond_dev;
    ta.target = target_dev;
    ta.n_rows = n_rows;
    ta.batch = batch;
    ta.sample_rows = sample_rows;
    ta.seed = seed;
    ta.step = step;
    ta.id_offset = id_offset;
    ta.kl_weight = (float)kl_weight;
    ta.partial = reinterpret_cast<float*>(ws_dev);
    ta.loss_partial = reinterpret_cast<double*>(reinterpret_cast<char*>(ws_dev) + train_partial_bytes(nb, n_params));
    hipStream_t hs = (hipStream_t)stream;
    const dim3 grid(nb), block(64 * kTrainWaves);
    if (shape_blocks(s) == 1) {
        switch (s.n_linear) {
            case 2: hipLaunchKernelGGL((cvae_train_kernel<2, 1>), grid, block, 0, hs, ta); break;
            case 3: hipLaunchKernelGGL((cvae_train_kernel<3, 1>), grid, block, 0, hs, ta); break;
            default: hipLaunchKernelGGL((cvae_train_kernel<4, 1>), grid, block, 0, hs, ta); break;
        }
    } else {
        switch (s.n_linear) {
            case 2: hipLaunchKernelGGL((cvae_train_kernel<2, 2>), grid, block, 0, hs, ta); break;
            case 3: hipLaunchKernelGGL((cvae_train_kernel<3, 2>), grid, block, 0, hs, ta); break;
            default: hipLaunchKernelGGL((cvae_train_kernel<4, 2>), grid, block, 0, hs, ta); break;
        }
    }
    MS_LAUNCHED();
    AdamArgs aa{};
    aa.n_params = n_params;
    aa.n_blocks = nb;
    aa.batch = batch;
    aa.partial = ta.partial;
    aa.loss_partial = ta.loss_partial;
    aa.master = master_dev;
    aa.m = adam_m_dev;
    aa.v = adam_v_dev;
    aa.grad_out = grad_dev;
    aa.loss_out = loss_dev;
    aa.do_update = adam != nullptr;
    if (adam) {
        aa.lr = (float)adam->lr;
        aa.beta1 = (float)adam->beta1;
        aa.beta2 = (float)adam->beta2;
        aa.one_m_beta1 = (float)(1.0 - adam->beta1);  // 1 - beta in FP32 would lose ~1e-5 relative
        aa.one_m_beta2 = (float)(1.0 - adam->beta2);
        aa.eps = (float)adam->eps;
        aa.wd = (float)adam->weight_decay;
        aa.bc1 = (float)(1.0 - pow(adam->beta1, (double)adam->step));
        aa.bc2 = (float)(1.0 - pow(adam->beta2, (double)adam->step));
    }
    hipLaunchKernelGGL(cvae_adam_kernel, dim3((n_params + kAdamParams - 1) / kAdamParams), dim3(256), 0, hs, aa);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

}  // namespace msst

extern "C" {

ms_status cvae_train_step(const ms_cvae_shape* shape, float* master_dev, float* adam_m_dev, float* adam_v_dev,
                          const ms_adam* adam, const float* cond_dev, const float* target_dev, int64_t n_rows,
                          int32_t batch, int32_t sample_rows, uint64_t seed, int64_t step, uint64_t id_offset,
                          double kl_weight, void* workspace_dev, size_t workspace_bytes, double* loss_dev,
                          float* grad_dev, void* stream) {
    return msst::train_step_launch("cvae_train_step", false, shape, master_dev, adam_m_dev, adam_v_dev, adam, cond_dev,
                                   target_dev, n_rows, batch, sample_rows, seed, step, id_offset, kl_weight,
                                   workspace_dev, workspace_bytes, loss_dev, grad_dev, stream);
}

ms_status cvae_train_step_noalloc(const ms_cvae_shape* shape, float* master_dev, float* adam_m_dev,
                                  float* adam_v_dev, const ms_adam* adam, const float* cond_dev,
                                  const float* target_dev, int64_t n_rows, int32_t batch, int32_t sample_rows,
                                  uint64_t seed, int64_t step, uint64_t id_offset, double kl_weight,
                                  double* loss_dev, float* grad_dev, void* stream) {
    return msst::train_step_launch("cvae_train_step_noalloc", true, shape, master_dev, adam_m_dev, adam_v_dev, adam,
                                   cond_dev, target_dev, n_rows, batch, sample_rows, seed, step, id_offset, kl_weight,
                                   nullptr, 0, loss_dev, grad_dev, stream);
}

size_t cvae_packed_bytes(void) { return sizeof(msst::PackedModel); }

ms_status cvae_pack(const ms_cvae_shape* shape, const float* master_dev, const double* stats_dev, int32_t precision,
                    const float* calib_cond_dev, int64_t n_calib, void* packed_dev, size_t packed_bytes,
                    void* stream) {
    using namespace msst;
    Shape s;
    ms_status st = check_shape(shape, &s);
    if (st != MS_OK) return st;
    MS_REQUIRE(master_dev && packed_dev, "cvae_pack: NULL array");
    MS_REQUIRE(precision == MS_PREC_BF16 || precision == MS_PREC_FP8, "cvae_pack: precision must be BF16 or FP8");
    MS_REQUIRE(n_calib >= 0 && n_calib <= (1 << 20), "cvae_pack: n_calib must be in [0, 2^20]");
    MS_REQUIRE(n_calib == 0 || (calib_cond_dev && stats_dev), "cvae_pack: calibration rows need calib_cond and stats");
    MS_REQUIRE(((uintptr_t)packed_dev & 15u) == 0, "cvae_pack: packed buffer must be 16-byte aligned");
    if (packed_bytes < sizeof(PackedModel))
        return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "cvae_pack: packed buffer needs %zu bytes", sizeof(PackedModel));
    int cus;
    if ((st = device_cu_count(&cus)) != MS_OK) return st;
    const bool calib = precision == MS_PREC_FP8 && n_calib > 0;
    if (calib)
        hipLaunchKernelGGL(cvae_calib_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, s, master_dev, stats_dev,
                           calib_cond_dev, n_calib, reinterpret_cast<PackedModel*>(packed_dev));
    hipLaunchKernelGGL(cvae_pack_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, s, master_dev, stats_dev, precision,
                       calib, reinterpret_cast<PackedModel*>(packed_dev));
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

ms_status cvae_sample(const void* packed_dev, const float* cond_dev, int64_t n, uint64_t seed, uint64_t id_offset,
                      float* out_dev, void* stream) {
    using namespace msst;
    MS_REQUIRE(packed_dev && cond_dev && out_dev, "cvae_sample: NULL array");
    MS_REQUIRE(n > 0 && n < ((int64_t)1 << 40), "cvae_sample: n must be in [1, 2^40)");
    MS_REQUIRE(((uintptr_t)packed_dev & 15u) == 0, "cvae_sample: packed buffer must be 16-byte aligned");
    int cus;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;
    int64_t blocks = (n + 64 * kSampleWaves - 1) / (64 * kSampleWaves);
    if (blocks > cus * 8) blocks = cus * 8;
    // the packed model's block count is on the device: each instance returns
    // at once unless it matches
    const PackedModel* pm = reinterpret_cast<const PackedModel*>(packed_dev);
    hipLaunchKernelGGL(cvae_sample_kernel<1>, dim3((unsigned)blocks), dim3(64 * kSampleWaves), 0, (hipStream_t)stream,
                       pm, cond_dev, n, seed, id_offset, out_dev);
    hipLaunchKernelGGL(cvae_sample_kernel<2>, dim3((unsigned)blocks), dim3(64 * kSampleWaves), 0, (hipStream_t)stream,
                       pm, cond_dev, n, seed, id_offset, out_dev);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

}  // extern "C"
