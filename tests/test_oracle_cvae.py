"""Pins of the oracle CVAE (Sec. 3.2, Sec. 4.2): gradients by central finite
differences, closed forms of the ELBO terms, the AdamW update on a constant
gradient, and the bfloat16 / FP8 rounding against torch's conversions."""
import math

import numpy as np
import pytest
import torch

LOG2PI = math.log(2 * math.pi)


def layer_dims(shape):
    """(n_in, n_out) of the 2 n_linear layers, encoder first."""
    nl = shape["n_linear"]
    dims = []
    for net in range(2):
        in0 = shape["latent"] + shape["p_in"] if net else shape["p_out"] + shape["p_in"]
        outl = 2 * shape["p_out"] if net else 2 * shape["latent"]
        for j in range(nl):
            dims.append((in0 if j == 0 else shape["width"], outl if j == nl - 1 else shape["width"]))
    return dims


def stride_of(shape):
    """Row stride of the layout: 16 when every width fits one 16-wide tile."""
    widest = max(max(d) for d in layer_dims(shape))
    return 16 if widest <= 16 else 32


def real_param_mask(shape):
    """True where a parameter is a real weight or bias (not S x S padding)."""
    S = stride_of(shape)
    mask = []
    for n_in, n_out in layer_dims(shape):
        W = np.zeros((S, S), bool)
        W[:n_out, :n_in] = True
        b = np.zeros(S, bool)
        b[:n_out] = True
        mask.append(np.concatenate([W.ravel(), b]))
    return np.concatenate(mask)


def restride(p, n_layers, S_from, S_to):
    """The same weights and biases in the layout of another row stride."""
    out = np.zeros(n_layers * (S_to * S_to + S_to))
    for layer in range(n_layers):
        src = p[layer * (S_from * S_from + S_from):(layer + 1) * (S_from * S_from + S_from)]
        dst = out[layer * (S_to * S_to + S_to):(layer + 1) * (S_to * S_to + S_to)]
        m = min(S_from, S_to)
        W = dst[:S_to * S_to].reshape(S_to, S_to)
        W[:m, :m] = src[:S_from * S_from].reshape(S_from, S_from)[:m, :m]
        dst[S_to * S_to:S_to * S_to + m] = src[S_from * S_from:S_from * S_from + m]
    return out


def batch(shape, B, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(B, shape["p_in"])), rng.normal(size=(B, shape["p_out"]))


def table1_cases():
    import workloads as W
    out = {f"table1-final-{m}": W.TABLE1_SHAPES[m] for m in range(3)}
    out["table1-D1-length-W4-L6"] = W.table1_shape(0, 1, 4, 6)
    out["table1-D3-path-W12-L5"] = W.table1_shape(1, 3, 12, 5)
    out["table1-D3-event-W16-L5"] = W.table1_shape(2, 3, 16, 5)
    # two-tile layouts (row stride 32): 20 hidden units, 2 x 9 encoder outputs
    out["table1-D2-event-W20-L5"] = W.table1_shape(2, 2, 20, 5)
    out["table1-D1-path-W8-L9"] = W.table1_shape(1, 1, 8, 9)
    out["table1-D3-event-W20-L9"] = W.table1_shape(2, 3, 20, 9)
    return out


ARCH_CASES = ["length", "path", "event"] + list(table1_cases())


def arch_shape(oracle, name):
    return oracle.SHAPES[name] if name in oracle.SHAPES else table1_cases()[name]


@pytest.mark.parametrize("name", ARCH_CASES)
def test_gradient_central_differences(oracle, name):
    shape = arch_shape(oracle, name)
    p = oracle.cvae_init(shape, seed=3)
    cond, target = batch(shape, 8, 4)
    loss, kl, nll, grad = oracle.cvae_loss_grad(shape, p, cond, target, seed=9, step=2)
    assert abs(loss - (kl + nll)) < 1e-12
    idx = np.flatnonzero(real_param_mask(shape))
    rng = np.random.default_rng(0)
    for i in rng.choice(idx, 80, replace=False):
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle.cvae_loss_grad(shape, pp, cond, target, 9, 2, want_grad=False)[0]
              - oracle.cvae_loss_grad(shape, pm, cond, target, 9, 2, want_grad=False)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])) + 1e-8, (i, fd, grad[i])
    # padding never receives gradient
    assert np.all(grad[~real_param_mask(shape)] == 0)


def zero_last_layers(shape, p):
    nl = shape["n_linear"]
    p = p.copy()
    for layer in (nl - 1, 2 * nl - 1):
        p[layer * 272: (layer + 1) * 272] = 0.0
    return p


@pytest.mark.parametrize("name", ["length", "path", "event"])
def test_elbo_closed_form_at_standard_normal(oracle, name):
    """Zero output layers give mu = 0, log var = 0: KL = 0 and NLL = P/2 (log 2 pi) + |y|^2 / 2."""
    shape = oracle.SHAPES[name]
    p = zero_last_layers(shape, oracle.cvae_init(shape, seed=5))
    cond, target = batch(shape, 16, 6)
    loss, kl, nll, _ = oracle.cvae_loss_grad(shape, p, cond, target, seed=1, step=1)
    assert kl == 0.0
    exp = np.mean(0.5 * (shape["p_out"] * LOG2PI + np.sum(target**2, axis=1)))
    assert abs(nll - exp) < 1e-12


def test_softplus_identities(oracle):
    for x in np.linspace(-30, 30, 121):
        assert abs(oracle.softplus(x) - oracle.softplus(-x) - x) < 1e-12
        if abs(x) < 20:
            assert abs(oracle.softplus(x) - math.log1p(math.exp(x))) < 1e-12 * max(1, abs(x))


def test_adamw_constant_gradient_closed_form(oracle):
    n = 50
    rng = np.random.default_rng(7)
    g = rng.normal(size=n)
    p0 = rng.normal(size=n)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    lr, eps = 1e-3, 1e-8
    for t in range(1, 4):
        oracle.adamw_step(p, m, v, g, t, lr=lr, eps=eps)
        # with a constant gradient m_hat = g and v_hat = g^2 at every step
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
    # decoupled decay: zero gradient shrinks by (1 - lr wd) per step
    q, m2, v2 = p0.copy(), np.zeros(n), np.zeros(n)
    oracle.adamw_step(q, m2, v2, np.zeros(n), 1, lr=lr, weight_decay=0.1)
    np.testing.assert_allclose(q, p0 * (1 - lr * 0.1), atol=1e-15)


def test_bf16_rounding_matches_torch(oracle):
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.normal(size=3000) * 10.0 ** rng.integers(-6, 6, 3000),
                        [0.0, -0.0, 1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-9, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.round_bf16(v) for v in x])
    np.testing.assert_array_equal(got, ref)


def test_fp8_e4m3_rounding_matches_torch(oracle):
    rng = np.random.default_rng(9)
    x = rng.uniform(-448, 448, 3000) * 10.0 ** rng.integers(-4, 1, 3000)
    x = np.concatenate([x, [0.0, 448.0, -448.0, 2**-9, 2**-10, 3 * 2**-10, 0.5, 240.0, 232.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([oracle.round_fp8_e4m3(v) for v in x])
    np.testing.assert_array_equal(got, ref)
    assert oracle.round_fp8_e4m3(1000.0) == 448.0  # saturating


@pytest.mark.parametrize("name", ["length", "path", "event"])
def test_decode_of_bias_only_network(oracle, name):
    shape = oracle.SHAPES[name]
    nl = shape["n_linear"]
    p = oracle.cvae_init(shape, seed=10)
    last = 2 * nl - 1
    p[last * 272: last * 272 + 256] = 0.0
    P = shape["p_out"]
    bias = p[last * 272 + 256: last * 272 + 256 + 2 * P]
    z = np.random.default_rng(1).normal(size=shape["latent"])
    c = np.random.default_rng(2).normal(size=shape["p_in"])
    mu, lv = oracle.cvae_decode(shape, p, z, c)
    np.testing.assert_array_equal(mu, bias[:P])
    np.testing.assert_array_equal(lv, np.clip(bias[P:], -12, 8))


@pytest.mark.parametrize("name", ["length", "path", "event"])
def test_bf16_emulation_exact_on_representable_inputs(oracle, name):
    """When weights and inputs are already bfloat16 values and the hidden
    activations are not rounded differently, BF16 emulation equals FP64 on
    the first layer's pre-activations; end to end it stays within bf16 error."""
    shape = oracle.SHAPES[name]
    p = np.array([oracle.round_bf16(v) for v in oracle.cvae_init(shape, seed=11)])
    z = np.array([oracle.round_bf16(v) for v in np.random.default_rng(3).normal(size=shape["latent"])])
    c = np.array([oracle.round_bf16(v) for v in np.random.default_rng(4).normal(size=shape["p_in"])])
    mu64, lv64 = oracle.cvae_decode(shape, p, z, c, precision=oracle.PREC_FP64)
    mu16, lv16 = oracle.cvae_decode(shape, p, z, c, precision=oracle.PREC_BF16)
    np.testing.assert_allclose(mu16, mu64, atol=0.05)
    np.testing.assert_allclose(lv16, lv64, atol=0.05)


def test_sample_destandardises(oracle):
    shape = oracle.SHAPES["path"]
    p = oracle.cvae_init(shape, seed=12)
    last = 2 * shape["n_linear"] - 1
    p[last * 272: last * 272 + 256] = 0.0
    P = shape["p_out"]
    p[last * 272 + 256: last * 272 + 256 + P] = [0.5, -1.0, 2.0]
    p[last * 272 + 256 + P: last * 272 + 256 + 2 * P] = -40.0  # clamped to -12
    stats = np.zeros(64)
    stats[16:32] = 1.0
    stats[32:35] = [1.0, 2.0, 3.0]
    stats[48:51] = [2.0, 0.5, 0.1]
    cond = np.random.default_rng(5).normal(size=(1000, shape["p_in"]))
    out = oracle.cvae_sample(shape, p, stats, cond, seed=3)
    exp = np.array([0.5 * 2 + 1, -1.0 * 0.5 + 2, 2.0 * 0.1 + 3])
    sd = np.exp(-6.0) * stats[48:51]
    assert np.all(np.abs(out - exp) < 6 * sd)
    # the residual is sqrt(Sigma) eps with eps standard normal
    eps = (out - exp) / sd
    assert abs(eps.mean()) < 0.1 and abs(eps.std() - 1) < 0.1


@pytest.mark.parametrize("name", ["length", "path", "event"])
def test_init_bounds(oracle, name):
    shape = oracle.SHAPES[name]
    p = oracle.cvae_init(shape, seed=13)
    mask = real_param_mask(shape)
    assert np.all(p[~mask] == 0)
    nl = shape["n_linear"]
    for layer in range(2 * nl):
        blk = p[layer * 272:(layer + 1) * 272]
        in0 = (shape["latent"] + shape["p_in"]) if layer >= nl else (shape["p_out"] + shape["p_in"])
        fan = in0 if layer % nl == 0 else shape["width"]
        assert np.all(np.abs(blk) <= 1 / math.sqrt(fan))


def test_length_target_round_trip(oracle):
    w = oracle.random_walk(5000, seed=3, mode=oracle.WALK_TRAINING)
    cond, target = oracle.cvae_features(0, w, seed=4)
    N = np.floor(np.exp(target[:, 0]) + 0.5)
    np.testing.assert_array_equal(N, w["n_scatter"])
    np.testing.assert_allclose(cond[:, 0], np.log(w["params"][0]))
    c2, t2 = oracle.cvae_features(2, w, seed=4)
    np.testing.assert_allclose(c2[:, 6], np.log(w["n_scatter"]))
    np.testing.assert_allclose(t2[:, :3].T, w["event_pos"])


def test_training_reduces_loss(oracle):
    """Invariant of a working optimiser: 300 AdamW steps on a fixed batch lower the loss."""
    shape = oracle.SHAPES["length"]
    p = oracle.cvae_init(shape, seed=1)
    m, v = np.zeros_like(p), np.zeros_like(p)
    rng = np.random.default_rng(2)
    cond = rng.normal(size=(64, 2))
    target = (0.8 * cond[:, :1] - 0.3 * cond[:, 1:] ** 2) + 0.1 * rng.normal(size=(64, 1))
    first = oracle.cvae_loss_grad(shape, p, cond, target, 5, 1)[0]
    for t in range(1, 301):
        loss, _, _, g = oracle.cvae_loss_grad(shape, p, cond, target, 5, t)
        oracle.adamw_step(p, m, v, g, t, lr=3e-3)
    assert loss < first - 0.3


@pytest.mark.parametrize("model", [0, 1, 2])
def test_narrow_network_equals_wide_network_with_silent_units(oracle, model):
    """A width-W network is the 16-wide network whose extra hidden units have
    zero outgoing weights, whatever their incoming weights (Table 1 widths):
    same loss and the same gradient on every real parameter."""
    import workloads as W
    narrow = dict(W.TABLE1_SHAPES[model], width=8 if model else 4)
    wide = dict(narrow, width=16)
    p = oracle.cvae_init(narrow, seed=11)
    q = p.copy().reshape(2 * narrow["n_linear"], 272)
    rng = np.random.default_rng(model)
    nl, w = narrow["n_linear"], narrow["width"]
    for net in range(2):
        for j in range(nl - 1):  # hidden layers: give the extra units incoming weights and biases
            layer = q[net * nl + j]
            Wm = layer[:256].reshape(16, 16)
            n_in = (narrow["latent"] + narrow["p_in"] if net else narrow["p_out"] + narrow["p_in"]) if j == 0 else w
            Wm[w:, :n_in] = rng.normal(size=(16 - w, n_in))
            layer[256 + w:] = rng.normal(size=16 - w)
    q = q.ravel()
    cond, target = batch(narrow, 8, 3)
    ln, kln, nlln, gn = oracle.cvae_loss_grad(narrow, p, cond, target, seed=4, step=1)
    lw, klw, nllw, gw = oracle.cvae_loss_grad(wide, q, cond, target, seed=4, step=1)
    assert abs(ln - lw) < 1e-12 * max(1.0, abs(ln))
    real = real_param_mask(narrow)
    np.testing.assert_allclose(gw[real], gn[real], rtol=1e-10, atol=1e-13)


def test_twenty_units_with_four_silent_equal_sixteen_across_the_stride(oracle):
    """Table 1's W = 20 EventGen (row stride 32) with the four extra hidden
    units given incoming weights but no outgoing ones is the W = 16 network
    (row stride 16): same loss, same gradient on every real parameter of the
    narrow one, and no gradient into the silent units' incoming weights and
    biases (nothing downstream depends on them)."""
    import workloads as W
    narrow = W.table1_shape(2, 2, 16, 5)
    wide = W.table1_shape(2, 2, 20, 5)
    assert oracle.layer_stride(narrow) == 16 and oracle.layer_stride(wide) == 32
    nl = narrow["n_linear"]
    p = oracle.cvae_init(narrow, seed=13)
    q = restride(p, 2 * nl, 16, 32).reshape(2 * nl, 32 * 32 + 32)
    rng = np.random.default_rng(5)
    for layer, (n_in, n_out) in enumerate(layer_dims(wide)):
        if n_out == 20:  # hidden layers: the extra units get incoming weights and biases
            Wm = q[layer, :1024].reshape(32, 32)
            Wm[16:20, :n_in] = rng.normal(size=(4, n_in))
            q[layer, 1024 + 16:1024 + 20] = rng.normal(size=4)
    q = q.ravel()
    cond, target = batch(narrow, 8, 6)
    ln, kln, nlln, gn = oracle.cvae_loss_grad(narrow, p, cond, target, seed=4, step=1)
    lw, klw, nllw, gw = oracle.cvae_loss_grad(wide, q, cond, target, seed=4, step=1)
    assert abs(ln - lw) < 1e-12 * max(1.0, abs(ln))
    g_back = restride(gw, 2 * nl, 32, 16)
    real = real_param_mask(narrow)
    np.testing.assert_allclose(g_back[real], gn[real], rtol=1e-10, atol=1e-13)
    gw2 = gw.reshape(2 * nl, 1056)
    for layer, (n_in, n_out) in enumerate(layer_dims(wide)):
        if n_out == 20:
            assert np.all(gw2[layer, :1024].reshape(32, 32)[16:20] == 0)
            assert np.all(gw2[layer, 1024 + 16:1024 + 20] == 0)


def _normals_seed0(oracle, i, L):
    """The first L normals of the sampler's stream for seed 0, id i: Box-Muller
    on the word pairs of Philox blocks (c0, id, tag CVAE_SAMPLE = 5)."""
    out = []
    for c0 in range((L + 3) // 4):
        w = oracle.philox4x32_10([c0, i & 0xFFFFFFFF, i >> 32, 5], [0, 0])
        u = (np.asarray(w, np.float64) // 256 + 1) * 2.0**-24
        for a, b in ((u[0], u[1]), (u[2], u[3])):
            r = math.sqrt(-2.0 * math.log(a))
            out += [r * math.cos(2 * math.pi * b), r * math.sin(2 * math.pi * b)]
    return np.array(out[:L])


@pytest.mark.parametrize("name", ["length", "path", "event"])
def test_fp8_activation_scales_bound_every_layer_input(oracle, name):
    """FP8 calibration: each decoder layer's activation scale is a power of
    two and the largest calibration input of that layer divided by it lies
    in (224, 448] (so no input saturates E4M3 and the largest uses its top
    binade) -- with the layer inputs recomputed here by a numpy forward pass
    over the documented parameter layout."""
    import workloads as W
    shape = oracle.SHAPES[name]
    model = shape["model"]
    p = oracle.cvae_init(shape, seed=21)
    stats = W.random_stats(model, seed=3)
    cond = W.random_conditions(model, 300, seed=4)
    sc = oracle.cvae_act_scales(shape, p, stats, cond)
    nl, L, C = shape["n_linear"], shape["latent"], shape["p_in"]
    mx = np.zeros(nl)
    for i in range(cond.shape[0]):
        a = np.zeros(16)
        a[:L] = _normals_seed0(oracle, i, L)
        a[L:L + C] = (cond[i] - stats[:C]) / stats[16:16 + C]
        for j in range(nl):
            n_in = L + C if j == 0 else shape["width"]
            mx[j] = max(mx[j], np.abs(a[:n_in]).max())
            lay = p[(nl + j) * 272:(nl + j + 1) * 272]
            pre = lay[:256].reshape(16, 16) @ a + lay[256:]
            a = np.logaddexp(0.0, pre)
    for j in range(nl):
        m, e = np.frexp(sc[j])
        assert m == 0.5, sc  # a power of two
        assert 224.0 < mx[j] / sc[j] <= 448.0, (j, mx[j], sc[j])


def test_fp8_activation_scales_cut_the_error_of_small_activations(oracle):
    """Hidden activations far below 1 (softplus of pre-activations near -7,
    amplified by the next layer's weights) sit in E4M3's subnormal range
    unless scaled: with calibrated scales the FP8 decoder's error against
    FP64 is a fraction of the unscaled one."""
    import workloads as W
    shape = oracle.SHAPES["event"]
    p = oracle.cvae_init(shape, seed=22)
    stats = W.random_stats(2, seed=5)
    width = shape["width"]
    b0 = p[3 * 272 + 256:3 * 272 + 256 + width]
    b0[:] = -7.0  # first decoder layer: softplus outputs ~1e-3
    p[4 * 272:4 * 272 + 256] *= 300.0  # second decoder layer amplifies them
    cond = W.random_conditions(2, 400, seed=6)
    sc = oracle.cvae_act_scales(shape, p, stats, cond)
    assert sc[1] <= 2.0**-12
    e_s, e_u = [], []
    for i in range(200):
        z = _normals_seed0(oracle, 1000 + i, shape["latent"])
        cs = (cond[i] - stats[:7]) / stats[16:23]
        mu64, _ = oracle.cvae_decode(shape, p, z, cs)
        mu_s, _ = oracle.cvae_decode(shape, p, z, cs, precision=oracle.PREC_FP8, act_scales=sc)
        mu_u, _ = oracle.cvae_decode(shape, p, z, cs, precision=oracle.PREC_FP8)
        e_s.append(np.abs(mu_s - mu64).max())
        e_u.append(np.abs(mu_u - mu64).max())
    assert np.median(e_s) < 0.5 * np.median(e_u), (np.median(e_s), np.median(e_u))
