/*
 * cvae.c -- oracle CVAE forward, loss, gradient, AdamW and sampling in FP64.
 * TEST INFRASTRUCTURE ONLY (see msst_oracle.h).
 *
 * Model (Sec. 3.2, Fig. 3b): encoder Enc(x, c) and decoder Dec(z, c) are MLPs
 * of n_linear linear maps with Softplus between hidden layers and linear
 * outputs (mean, log variance); both posteriors are diagonal Gaussians.  The
 * training objective is the negative ELBO: KL(q_Enc || N(0, I)) plus the
 * Gaussian negative log-likelihood of the target under the decoder, with one
 * reparameterised latent sample z = mu + exp(logvar / 2) eps.  At inference
 * the encoder is dropped, z ~ N(0, I), and x = mu_Dec + sqrt(Sigma_Dec) eps.
 * The three models and their inputs are those of Sec. 4.2:
 *   LengthGen (sigma_t r, g)                         -> N
 *   PathGen   (sigma_t r, g, N)                      -> (cos theta, alpha, beta)
 *   EventGen  (sigma_t r, g, albedo, theta, alpha, beta, N) -> (X, W)
 *
 * Parameter layout (shared interface with the GPU library, implemented
 * independently on each side): 2 * n_linear layers, encoder first; each
 * layer is an S x S row-major weight block (row = output unit, column =
 * input unit) followed by S biases; unused rows and columns are zero.
 * S = 16 when every width of the two networks (hidden units, inputs,
 * outputs) is at most 16, else 32 (Table 1's widest settings).
 */
#include "msst_oracle.h"

#include <math.h>
#include <string.h>

#define OR_LOG_2PI 1.83787706640934548356065947281123527
#define OR_LV_MIN (-12.0)
#define OR_LV_MAX (8.0)

static int or_n_linear(const or_cvae_shape* s) { return s->n_linear > 0 ? s->n_linear : 3; }

/* Row stride S of the parameter layout (see above). */
static int or_stride(const or_cvae_shape* s) {
    int m = s->width;
    if (s->p_out + s->p_in > m) m = s->p_out + s->p_in;
    if (s->latent + s->p_in > m) m = s->latent + s->p_in;
    if (2 * s->p_out > m) m = 2 * s->p_out;
    if (2 * s->latent > m) m = 2 * s->latent;
    return m <= 16 ? 16 : 32;
}

static int or_layer_floats(const or_cvae_shape* s) {
    int S = or_stride(s);
    return S * S + S;
}

int64_t or_cvae_param_count(const or_cvae_shape* s) {
    return (int64_t)(2 * or_n_linear(s)) * or_layer_floats(s);
}

double or_softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }
static double or_sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Round to binary32 (round to nearest even), then to bfloat16 (round to
 * nearest even on the upper 16 bits), as a device converting an FP32 value
 * would. */
double or_round_bf16(double x) {
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* OCP FP8 E4M3 (bias 7, max normal 448, no infinities), round to nearest
 * even, saturating at +-448. */
double or_round_fp8_e4m3(double x) {
    double a = fabs((double)(float)x);
    if (a == 0.0 || x != x) return x != x ? x : 0.0;
    if (a >= 448.0) return x < 0 ? -448.0 : 448.0;
    int e;
    frexp(a, &e); /* a = m 2^e, m in [0.5, 1) */
    int exp_unb = e - 1;                 /* a in [2^exp_unb, 2^(exp_unb+1)) */
    if (exp_unb < -6) exp_unb = -6;      /* subnormal range: spacing 2^-9 */
    double q = ldexp(1.0, exp_unb - 3);  /* 3 mantissa bits */
    double r = a / q;
    double fl = floor(r);
    double frac = r - fl;
    double m;
    if (frac > 0.5) m = fl + 1.0;
    else if (frac < 0.5) m = fl;
    else m = (fmod(fl, 2.0) == 0.0) ? fl : fl + 1.0;
    double v = m * q;
    if (v > 448.0) v = 448.0;
    return x < 0 ? -v : v;
}

typedef struct {
    int n_in[8], n_out[8];
} or_dims;

/* Real (unpadded) input / output sizes of the layers of one network. */
static void or_net_dims(const or_cvae_shape* s, int decoder, or_dims* d) {
    int nl = or_n_linear(s);
    int in0 = decoder ? s->latent + s->p_in : s->p_out + s->p_in;
    int outl = decoder ? 2 * s->p_out : 2 * s->latent;
    for (int j = 0; j < nl; ++j) {
        d->n_in[j] = j == 0 ? in0 : s->width;
        d->n_out[j] = j == nl - 1 ? outl : s->width;
    }
}

static const double* or_layer(const double* params, int layer, int lf) {
    return params + (size_t)layer * lf;
}

void or_cvae_init(const or_cvae_shape* s, uint64_t seed, double* params) {
    int nl = or_n_linear(s);
    const int S = or_stride(s), lf = or_layer_floats(s);
    memset(params, 0, sizeof(double) * (size_t)(2 * nl) * lf);
    for (int net = 0; net < 2; ++net) {
        or_dims dm;
        or_net_dims(s, net, &dm);
        for (int j = 0; j < nl; ++j) {
            int layer = net * nl + j;
            double bound = 1.0 / sqrt((double)dm.n_in[j]);
            double* w = params + (size_t)layer * lf;
            for (int r = 0; r < dm.n_out[j]; ++r) {
                for (int c = 0; c <= dm.n_in[j]; ++c) {
                    /* c == n_in stands for the bias of row r */
                    int flat = (c < dm.n_in[j]) ? r * S + c : S * S + r;
                    uint32_t p = (uint32_t)(layer * lf + flat);
                    uint32_t wd[4];
                    or_philox_blocks(seed, OR_TAG_CVAE_INIT, (uint64_t)s->model, p >> 2, 1, wd);
                    double u = or_u01(wd[p & 3u]);
                    w[flat] = (2.0 * u - 1.0) * bound;
                }
            }
        }
    }
}

/* Quantiser of one layer's operands for the precision being emulated. */
static double or_q(double x, int precision) {
    if (precision == OR_PREC_BF16) return or_round_bf16(x);
    if (precision == OR_PREC_FP8) return or_round_fp8_e4m3(x);
    return x;
}

/* One linear layer pre = W a + b, with weights and inputs quantised as the
 * emulated precision prescribes.  For FP8 the weights are divided by the
 * per-layer weight scale max|W| / 448 and the inputs by the given activation
 * scale before rounding; the product is rescaled afterwards. */
static void or_linear(const double* layer, int S, int n_in, int n_out, const double* a, int precision,
                      double act_scale, double* pre) {
    const double* W = layer;
    const double* b = layer + S * S;
    double sw = 1.0, sa = 1.0;
    if (precision == OR_PREC_FP8) {
        double mx = 0.0;
        for (int r = 0; r < S; ++r)
            for (int c = 0; c < S; ++c) mx = fmax(mx, fabs(W[r * S + c]));
        sw = mx > 0.0 ? mx / 448.0 : 1.0;
        sa = act_scale > 0.0 ? act_scale : 1.0;
    }
    for (int r = 0; r < n_out; ++r) {
        double acc = 0.0;
        for (int c = 0; c < n_in; ++c)
            acc += or_q(W[r * S + c] / sw, precision) * or_q(a[c] / sa, precision);
        pre[r] = acc * sw * sa + b[r];
    }
}

typedef struct {
    double a[9][OR_MAX_WIDTH];   /* a[j] = input of layer j; a[nl] = output */
    double pre[8][OR_MAX_WIDTH]; /* pre-activations */
} or_trace;

static void or_mlp_forward(const double* params, int S, int first_layer, int nl, const or_dims* dm,
                           int precision, const double* act_scales, or_trace* t) {
    for (int j = 0; j < nl; ++j) {
        double sa = act_scales ? act_scales[j] : 1.0;
        or_linear(or_layer(params, first_layer + j, S * S + S), S, dm->n_in[j], dm->n_out[j], t->a[j],
                  precision, sa, t->pre[j]);
        for (int r = 0; r < dm->n_out[j]; ++r)
            t->a[j + 1][r] = (j < nl - 1) ? or_softplus(t->pre[j][r]) : t->pre[j][r];
    }
}

/* Backward through an MLP given d loss / d output; accumulates parameter
 * gradients and returns d loss / d input in din. */
static void or_mlp_backward(const double* params, int S, int first_layer, int nl, const or_dims* dm,
                            const or_trace* t, const double* dout, double* grad, double* din) {
    const int lf = S * S + S;
    double dcur[OR_MAX_WIDTH];
    memcpy(dcur, dout, sizeof dcur);
    for (int j = nl - 1; j >= 0; --j) {
        double dpre[OR_MAX_WIDTH];
        for (int r = 0; r < dm->n_out[j]; ++r)
            dpre[r] = (j < nl - 1) ? dcur[r] * or_sigmoid(t->pre[j][r]) : dcur[r];
        const double* W = or_layer(params, first_layer + j, lf);
        double* gW = grad + (size_t)(first_layer + j) * lf;
        for (int r = 0; r < dm->n_out[j]; ++r) {
            for (int c = 0; c < dm->n_in[j]; ++c) gW[r * S + c] += dpre[r] * t->a[j][c];
            gW[S * S + r] += dpre[r];
        }
        double dnext[OR_MAX_WIDTH];
        for (int c = 0; c < OR_MAX_WIDTH; ++c) dnext[c] = 0.0;
        for (int c = 0; c < dm->n_in[j]; ++c) {
            double acc = 0.0;
            for (int r = 0; r < dm->n_out[j]; ++r) acc += W[r * S + c] * dpre[r];
            dnext[c] = acc;
        }
        memcpy(dcur, dnext, sizeof dcur);
    }
    if (din) memcpy(din, dcur, sizeof dcur);
}

static double or_clamp_lv(double x) { return x < OR_LV_MIN ? OR_LV_MIN : (x > OR_LV_MAX ? OR_LV_MAX : x); }
static double or_clamp_mask(double x) { return (x > OR_LV_MIN && x < OR_LV_MAX) ? 1.0 : 0.0; }

double or_cvae_loss_grad(const or_cvae_shape* s, const double* params, int32_t batch,
                         const double* cond, const double* target, uint64_t seed, int64_t step,
                         uint64_t id_offset, double kl_weight, double* grad, double* kl_out,
                         double* nll_out) {
    const int nl = or_n_linear(s);
    const int P = s->p_out, L = s->latent, C = s->p_in;
    or_dims de, dd;
    or_net_dims(s, 0, &de);
    or_net_dims(s, 1, &dd);
    const int S = or_stride(s), lf = or_layer_floats(s);
    if (grad) memset(grad, 0, sizeof(double) * (size_t)(2 * nl) * lf);
    double kl_sum = 0.0, nll_sum = 0.0;
    for (int b = 0; b < batch; ++b) {
        const double* y = target + (size_t)b * P;
        const double* c = cond + (size_t)b * C;
        /* reparameterisation noise: ceil(L / 4) blocks at c0 = 4 step + j */
        double eps[16];
        for (int j = 0; j * 4 < L; ++j)
            or_normal4(seed, OR_TAG_CVAE_REPARAM, id_offset + (uint64_t)b,
                       (uint32_t)(4 * step + j), eps + 4 * j);
        or_trace te, td;
        memset(&te, 0, sizeof te);
        memset(&td, 0, sizeof td);
        for (int i = 0; i < P; ++i) te.a[0][i] = y[i];
        for (int i = 0; i < C; ++i) te.a[0][P + i] = c[i];
        or_mlp_forward(params, S, 0, nl, &de, OR_PREC_FP64, NULL, &te);
        double muz[16], lvz_raw[16], lvz[16], z[16];
        for (int i = 0; i < L; ++i) {
            muz[i] = te.a[nl][i];
            lvz_raw[i] = te.a[nl][L + i];
            lvz[i] = or_clamp_lv(lvz_raw[i]);
            z[i] = muz[i] + exp(0.5 * lvz[i]) * eps[i];
        }
        for (int i = 0; i < L; ++i) td.a[0][i] = z[i];
        for (int i = 0; i < C; ++i) td.a[0][L + i] = c[i];
        or_mlp_forward(params, S, nl, nl, &dd, OR_PREC_FP64, NULL, &td);
        double kl = 0.0, nll = 0.0;
        for (int i = 0; i < L; ++i) kl += 0.5 * (muz[i] * muz[i] + exp(lvz[i]) - lvz[i] - 1.0);
        double dout_d[OR_MAX_WIDTH];
        for (int i = 0; i < OR_MAX_WIDTH; ++i) dout_d[i] = 0.0;
        for (int i = 0; i < P; ++i) {
            double mu = td.a[nl][i], lvr = td.a[nl][P + i], lv = or_clamp_lv(lvr);
            double r = y[i] - mu, iv = exp(-lv);
            nll += 0.5 * (OR_LOG_2PI + lv + r * r * iv);
            dout_d[i] = -r * iv;
            dout_d[P + i] = 0.5 * (1.0 - r * r * iv) * or_clamp_mask(lvr);
        }
        kl_sum += kl;
        nll_sum += nll;
        if (!grad) continue;
        double ddin[OR_MAX_WIDTH];
        or_mlp_backward(params, S, nl, nl, &dd, &td, dout_d, grad, ddin);
        double dout_e[OR_MAX_WIDTH];
        for (int i = 0; i < OR_MAX_WIDTH; ++i) dout_e[i] = 0.0;
        for (int i = 0; i < L; ++i) {
            double dz = ddin[i];
            double sd = exp(0.5 * lvz[i]);
            dout_e[i] = dz + kl_weight * muz[i];
            dout_e[L + i] = (0.5 * dz * eps[i] * sd + kl_weight * 0.5 * (exp(lvz[i]) - 1.0)) *
                            or_clamp_mask(lvz_raw[i]);
        }
        or_mlp_backward(params, S, 0, nl, &de, &te, dout_e, grad, NULL);
    }
    double inv = 1.0 / (double)batch;
    if (grad)
        for (size_t i = 0; i < (size_t)(2 * nl) * lf; ++i) grad[i] *= inv;
    if (kl_out) *kl_out = kl_sum * inv;
    if (nll_out) *nll_out = nll_sum * inv;
    return (kl_sum + nll_sum) * inv;
}

/* The gradient above is that of NLL + kl_weight * KL (kl_weight = 1 is the
 * negative ELBO); the returned loss and kl_out / nll_out are unweighted. */

/* AdamW (Loshchilov and Hutter), the optimiser named in Sec. 3.2, with bias
 * correction and decoupled weight decay applied to the pre-step value. */
void or_adamw_step(int32_t n, double* params, double* m, double* v, const double* grad,
                   double lr, double beta1, double beta2, double eps, double weight_decay,
                   int64_t step) {
    double bc1 = 1.0 - pow(beta1, (double)step);
    double bc2 = 1.0 - pow(beta2, (double)step);
    for (int32_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m[i] / bc1, vh = v[i] / bc2;
        params[i] -= lr * (mh / (sqrt(vh) + eps) + weight_decay * params[i]);
    }
}

void or_cvae_decode(const or_cvae_shape* s, const double* params, int32_t precision,
                    const double* act_scales, const double* z, const double* cond_std,
                    double* mu, double* logvar) {
    const int nl = or_n_linear(s);
    const int P = s->p_out, L = s->latent, C = s->p_in;
    or_dims dd;
    or_net_dims(s, 1, &dd);
    or_trace td;
    memset(&td, 0, sizeof td);
    for (int i = 0; i < L; ++i) td.a[0][i] = z[i];
    for (int i = 0; i < C; ++i) td.a[0][L + i] = cond_std[i];
    or_mlp_forward(params, or_stride(s), nl, nl, &dd, precision, act_scales, &td);
    for (int i = 0; i < P; ++i) {
        mu[i] = td.a[nl][i];
        logvar[i] = or_clamp_lv(td.a[nl][P + i]);
    }
}

void or_cvae_sample(const or_cvae_shape* s, const double* params, const double* stats,
                    int32_t precision, const double* act_scales, const double* cond, int64_t n,
                    uint64_t seed, uint64_t id_offset, double* out) {
    const int P = s->p_out, L = s->latent, C = s->p_in;
    for (int64_t i = 0; i < n; ++i) {
        double nrm[32];
        int nb = (L + P + 3) / 4;
        for (int j = 0; j < nb; ++j)
            or_normal4(seed, OR_TAG_CVAE_SAMPLE, id_offset + (uint64_t)i, (uint32_t)j, nrm + 4 * j);
        double cs[16], mu[16], lv[16];
        for (int k = 0; k < C; ++k) cs[k] = (cond[i * C + k] - stats[k]) / stats[16 + k];
        or_cvae_decode(s, params, precision, act_scales, nrm, cs, mu, lv);
        for (int k = 0; k < P; ++k) {
            double ys = mu[k] + exp(0.5 * lv[k]) * nrm[L + k];
            out[i * P + k] = ys * stats[48 + k] + stats[32 + k];
        }
    }
}

/* Per-layer activation scales of a decoder for FP8 inference (the per-layer
 * scaling of low-precision decoder weights and activations): for decoder
 * layer j, s_j is the smallest power of two with max |a_j| / s_j <= 448 (the
 * largest E4M3 value), where a_j is the layer's input in exact arithmetic
 * (FP64, unquantised weights), maximised over the calibration rows i < n:
 * standardised condition cond[i] and latent z the first L normals of the
 * sampler's stream for seed 0 and id i.  s_j = 1 where max |a_j| = 0.
 * Powers of two make the scaling itself exact. */
void or_cvae_act_scales(const or_cvae_shape* s, const double* params, const double* stats,
                        const double* cond, int64_t n, double* scales) {
    const int nl = or_n_linear(s);
    const int L = s->latent, C = s->p_in;
    or_dims dd;
    or_net_dims(s, 1, &dd);
    double mx[8] = {0.0};
    for (int64_t i = 0; i < n; ++i) {
        double nrm[32];
        for (int j = 0; 4 * j < L; ++j) or_normal4(0, OR_TAG_CVAE_SAMPLE, (uint64_t)i, (uint32_t)j, nrm + 4 * j);
        or_trace td;
        memset(&td, 0, sizeof td);
        for (int k = 0; k < L; ++k) td.a[0][k] = nrm[k];
        for (int k = 0; k < C; ++k) td.a[0][L + k] = (cond[i * C + k] - stats[k]) / stats[16 + k];
        or_mlp_forward(params, or_stride(s), nl, nl, &dd, OR_PREC_FP64, NULL, &td);
        for (int j = 0; j < nl; ++j)
            for (int k = 0; k < dd.n_in[j]; ++k) mx[j] = fmax(mx[j], fabs(td.a[j][k]));
    }
    for (int j = 0; j < nl; ++j) {
        scales[j] = 1.0;
        if (mx[j] > 0.0) {
            int e;
            double f = frexp(mx[j] / 448.0, &e); /* mx / 448 = f 2^e, f in [0.5, 1) */
            scales[j] = ldexp(1.0, f == 0.5 ? e - 1 : e);
        }
    }
}

/* Condition and target vectors of one model from walk tuples (Sec. 4.2):
 * sigma_t r enters as its logarithm and N as log N; LengthGen's integer
 * target N is dequantised to log(N + u - 1/2) with u uniform on (0, 1]. */
void or_cvae_features(int32_t model, int64_t n, const double* params3, const uint32_t* n_scatter,
                      const double* exit_param, const double* event_pos, const double* event_dir,
                      uint64_t seed, uint64_t id_offset, double* cond, double* target) {
    for (int64_t i = 0; i < n; ++i) {
        double lst = log(params3[i]), g = params3[n + i], phi = params3[2 * n + i];
        double N = (double)n_scatter[i];
        double ct = exit_param[i], al = exit_param[n + i], be = exit_param[2 * n + i];
        if (model == 0) {
            double u[4];
            or_uniform4(seed, OR_TAG_DEQUANT, id_offset + (uint64_t)i, 0, u);
            cond[i * 2 + 0] = lst;
            cond[i * 2 + 1] = g;
            target[i] = log(N + u[0] - 0.5);
        } else if (model == 1) {
            cond[i * 3 + 0] = lst;
            cond[i * 3 + 1] = g;
            cond[i * 3 + 2] = log(N);
            target[i * 3 + 0] = ct;
            target[i * 3 + 1] = al;
            target[i * 3 + 2] = be;
        } else {
            double* c = cond + i * 7;
            c[0] = lst;
            c[1] = g;
            c[2] = phi;
            c[3] = ct;
            c[4] = al;
            c[5] = be;
            c[6] = log(N);
            double* t = target + i * 6;
            for (int k = 0; k < 3; ++k) {
                t[k] = event_pos[(int64_t)k * n + i];
                t[3 + k] = event_dir[(int64_t)k * n + i];
            }
        }
    }
}
