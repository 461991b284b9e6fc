"""GPU CVAE kernels against the FP64 oracle (Sec. 3.2, Sec. 4.2): init,
features, FP64 moments, gradients of the bfloat16 MFMA forward/backward,
AdamW, packing and decoder-only sampling."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import announce

pytestmark = pytest.mark.gpu

BF16_U = 2.0**-8  # unit roundoff of bfloat16 (8 significant bits)
FP8_U = 2.0**-4  # unit roundoff of FP8 E4M3 (4 significant bits)
# Gradients of the bfloat16 MFMA forward / backward against FP64: each
# gradient entry sums products of a few rounded operands over the batch, so
# independent roundings of size u average to ~u / 2 relative in L2 (measured
# 1.0e-3 to 2.7e-3 over the standard and Table 1 shapes); the batch-mean
# loss to ~u / 10.
GRAD_REL = 5e-3
LOSS_REL = 2e-3
MODELS = [0, 1, 2]


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda().contiguous()


@pytest.mark.parametrize("model", MODELS)
def test_init_matches_oracle(msst, oracle, model):
    announce(f"cvae init model={model}")
    shape = W.SHAPE_LIST[model]
    n = msst.cvae_param_count(model)
    master = torch.empty(n, dtype=torch.float32, device="cuda")
    msst.cvae_init(model, 77, master)
    ref = oracle.cvae_init(shape, 77)
    np.testing.assert_allclose(master.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)


def test_features_and_moments(msst, oracle):
    announce("cvae features + moments")
    n = 20000
    walk = msst.random_walk(n, seed=5, mode=1)
    torch.cuda.synchronize()
    w64 = {k: v.cpu().numpy().astype(np.float64) if v.dtype == torch.float32 else v.cpu().numpy()
           for k, v in walk.items()}
    w64["n_scatter"] = w64["n_scatter"].astype(np.uint32)
    for model in MODELS:
        p_in, p_out = [(2, 1), (3, 3), (7, 6)][model]
        cond = torch.empty((n, p_in), dtype=torch.float32, device="cuda")
        target = torch.empty((n, p_out), dtype=torch.float32, device="cuda")
        wk = {k: walk[k] for k in ("params", "n_scatter", "exit_param", "event_pos", "event_dir")}
        wk["n_scatter"] = walk["n_scatter"]
        msst.cvae_features(model, n, wk, 9, 100, None, cond, target)
        rc, rt = oracle.cvae_features(model, w64, seed=9, id_offset=100)
        np.testing.assert_allclose(cond.cpu().numpy(), rc, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(target.cpu().numpy(), rt, rtol=1e-5, atol=1e-6)
        # FP64 column moments of the float32 rows, against numpy in float64
        st = msst.make_stats(cond, target).cpu().numpy()
        c64 = cond.cpu().numpy().astype(np.float64)
        t64 = target.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(st[:p_in], c64.mean(0), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(st[16:16 + p_in], c64.std(0), rtol=1e-12)
        np.testing.assert_allclose(st[32:32 + p_out], t64.mean(0), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(st[48:48 + p_out], t64.std(0), rtol=1e-12)
        # standardised rows
        msst.cvae_features(model, n, wk, 9, 100, dev(st, torch.float64), cond, target)
        np.testing.assert_allclose(cond.cpu().numpy(), (rc - st[:p_in]) / st[16:16 + p_in], rtol=1e-5, atol=1e-5)


def test_select_rows_is_exact(msst):
    announce("select rows")
    walk = msst.random_walk(70001, seed=3, mode=1)
    ns = walk["n_scatter"].cpu().numpy()
    ek = walk["event_index"].cpu().numpy()
    rows = msst.select_rows(walk, 2).cpu().numpy()
    np.testing.assert_array_equal(rows, np.flatnonzero(ns >= 2))
    rows = msst.select_rows(walk, 2, 2).cpu().numpy()
    np.testing.assert_array_equal(rows, np.flatnonzero((ns >= 2) & (ek >= 2)))
    rows = msst.select_rows(walk, 10**9).cpu().numpy()
    assert rows.size == 0


def grad_case(msst, oracle, model, B, sample_rows=0, n_rows=None, kl_weight=1.0):
    shape = W.SHAPE_LIST[model]
    master64 = oracle.cvae_init(shape, seed=31 + model).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(model)
    n_rows = n_rows or B
    cond = rng.normal(size=(n_rows, shape["p_in"])).astype(np.float32)
    target = rng.normal(size=(n_rows, shape["p_out"])).astype(np.float32)
    seed, step = 1234, 7
    n = master64.size
    master = dev(master64)
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(3, dtype=torch.float64, device="cuda")
    ws = torch.empty(msst.cvae_workspace_size(model, B), dtype=torch.uint8, device="cuda")
    msst.cvae_train_step(model, master, None, None, None, dev(cond), dev(target), n_rows, B, sample_rows, seed, step,
                         0, ws, loss, grad, kl_weight=kl_weight)
    torch.cuda.synchronize()
    if sample_rows:
        words = np.array([oracle.philox_blocks(seed, oracle.TAG_CVAE_BATCH, b, step, 1)[0, 0] for b in range(B)],
                         dtype=np.uint64)
        rows = ((words * np.uint64(n_rows)) >> np.uint64(32)).astype(np.int64)
    else:
        rows = np.arange(B)
    l64, kl64, nll64, g64 = oracle.cvae_loss_grad(shape, master64, cond[rows].astype(np.float64),
                                                  target[rows].astype(np.float64), seed, step, kl_weight=kl_weight)
    return grad.cpu().numpy().astype(np.float64), g64, loss.cpu().numpy(), (l64, kl64, nll64)


@pytest.mark.parametrize("model", MODELS)
def test_gradient_parity_bf16(msst, oracle, model):
    """Gradients of the bfloat16 MFMA forward/backward against FP64 (tolerance
    ~10 bfloat16 roundoffs relative in L2; direction to cosine 0.999)."""
    announce(f"cvae grad parity model={model}")
    g, g64, loss, ref = grad_case(msst, oracle, model, B=256)
    rel = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    cos = g @ g64 / (np.linalg.norm(g) * np.linalg.norm(g64))
    print(f"model {model}: grad rel-L2 {rel:.3e}, cosine {cos:.6f}, loss {loss} vs {ref}")
    assert rel < GRAD_REL and cos > 0.999
    np.testing.assert_allclose(loss, ref, rtol=LOSS_REL, atol=1e-3)
    assert abs(loss[0] - loss[1] - loss[2]) < 1e-9 * abs(loss[0])


def test_gradient_parity_kl_weight(msst, oracle):
    announce("cvae grad kl weight")
    g, g64, loss, ref = grad_case(msst, oracle, 1, B=128, kl_weight=0.3)
    rel = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    assert rel < GRAD_REL


def test_gradient_parity_sampled_rows_and_ragged(msst, oracle):
    announce("cvae grad sampled rows")
    g, g64, loss, ref = grad_case(msst, oracle, 2, B=16 * 37, sample_rows=1, n_rows=5000)
    rel = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    assert rel < GRAD_REL
    np.testing.assert_allclose(loss, ref, rtol=LOSS_REL, atol=1e-3)


def test_adamw_step_matches_oracle(msst, oracle):
    announce("cvae adamw")
    model, B = 1, 128
    shape = W.SHAPE_LIST[model]
    master64 = oracle.cvae_init(shape, seed=3).astype(np.float32).astype(np.float64)
    n = master64.size
    rng = np.random.default_rng(4)
    m0 = (rng.normal(size=n) * 1e-3).astype(np.float32).astype(np.float64)
    v0 = (rng.uniform(size=n) * 1e-6).astype(np.float32).astype(np.float64)
    cond = rng.normal(size=(B, shape["p_in"])).astype(np.float32)
    target = rng.normal(size=(B, shape["p_out"])).astype(np.float32)
    master, m, v = dev(master64), dev(m0), dev(v0)
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    ws = torch.empty(msst.cvae_workspace_size(model, B), dtype=torch.uint8, device="cuda")
    adam = msst.adam_params(step=5, lr=1e-3, weight_decay=0.01)
    msst.cvae_train_step(model, master, m, v, adam, dev(cond), dev(target), B, B, 0, 1, 1, 0, ws, None, grad)
    torch.cuda.synchronize()
    p, mm, vv = master64.copy(), m0.copy(), v0.copy()
    oracle.adamw_step(p, mm, vv, grad.cpu().numpy().astype(np.float64), 5, lr=1e-3, weight_decay=0.01)
    np.testing.assert_allclose(master.cpu().numpy(), p, rtol=1e-6, atol=1e-8)
    # FP32 moments: beta m + (1 - beta) g loses ~1e-7 of max(|m|, |g|) absolutely
    np.testing.assert_allclose(m.cpu().numpy(), mm, rtol=1e-5, atol=1e-7 * np.abs(mm).max())
    np.testing.assert_allclose(v.cpu().numpy(), vv, rtol=1e-5, atol=1e-7 * np.abs(vv).max())


def test_training_reduces_loss_and_keeps_padding_zero(msst, oracle):
    announce("cvae training loop")
    model, B = 0, 1024
    n_rows = 1 << 15
    rng = np.random.default_rng(2)
    cond = rng.normal(size=(n_rows, 2)).astype(np.float32)
    target = (0.8 * cond[:, :1] - 0.3 * cond[:, 1:] ** 2 + 0.1 * rng.normal(size=(n_rows, 1))).astype(np.float32)
    cd, td = dev(cond), dev(target)
    n = msst.cvae_param_count(model)
    master = torch.empty(n, dtype=torch.float32, device="cuda")
    msst.cvae_init(model, 5, master)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    ws = torch.empty(msst.cvae_workspace_size(model, B), dtype=torch.uint8, device="cuda")
    loss = torch.zeros(3, dtype=torch.float64, device="cuda")
    hist = []
    for step in range(1, 401):
        msst.cvae_train_step(model, master, m, v, msst.adam_params(step, lr=3e-3), cd, td, n_rows, B, 1, 11, step, 0,
                             ws, loss)
        if step in (1, 400):
            hist.append(loss.cpu().numpy().copy())
    assert hist[1][0] < hist[0][0] - 0.5, hist
    mp = master.cpu().numpy()
    pad = ~_real_mask(W.SHAPE_LIST[model])
    assert np.all(mp[pad] == 0)


def _real_mask(shape):
    nl = shape["n_linear"]
    mask = np.zeros((2 * nl, 272), bool)
    for net in range(2):
        in0 = shape["latent"] + shape["p_in"] if net else shape["p_out"] + shape["p_in"]
        outl = 2 * shape["p_out"] if net else 2 * shape["latent"]
        for j in range(nl):
            n_in = in0 if j == 0 else shape["width"]
            n_out = outl if j == nl - 1 else shape["width"]
            Wm = np.zeros((16, 16), bool)
            Wm[:n_out, :n_in] = True
            b = np.zeros(16, bool)
            b[:n_out] = True
            mask[net * nl + j] = np.concatenate([Wm.ravel(), b])
    return mask.ravel()


@pytest.mark.parametrize("model", MODELS)
def test_sample_matches_bf16_emulating_oracle(msst, oracle, model):
    """Decoder sampling on MFMA against the oracle that rounds weights and layer
    inputs to bfloat16 exactly where the kernel does.  Remaining differences
    come from FP32 vs FP64 accumulation and transcendentals, except where such
    a difference flips a bfloat16 rounding (one bfloat16 ulp on one unit)."""
    announce(f"cvae sample model={model}")
    shape = W.SHAPE_LIST[model]
    master64 = oracle.cvae_init(shape, seed=50 + model).astype(np.float32).astype(np.float64)
    stats = W.random_stats(model, seed=model)
    n = 4000 + 37  # ragged last wave and tile
    cond = W.random_conditions(model, n, seed=model).astype(np.float32)
    packed = torch.empty(msst.cvae_packed_bytes(), dtype=torch.uint8, device="cuda")
    msst.cvae_pack(model, dev(master64), dev(stats, torch.float64), 1, packed)
    out = torch.empty((n, shape["p_out"]), dtype=torch.float32, device="cuda")
    msst.cvae_sample(packed, dev(cond), n, 99, 1000, out)
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.cvae_sample(shape, master64, stats, cond.astype(np.float64), 99, 1000, precision=oracle.PREC_BF16)
    scale = stats[48:48 + shape["p_out"]]
    err = np.abs(got - ref).max(axis=1) / scale.max()
    print(f"model {model}: median {np.median(err):.2e}, p99 {np.quantile(err, 0.99):.2e}, max {err.max():.2e}")
    assert np.quantile(err, 0.99) < 1e-4
    assert err.max() < 0.05
    ref64 = oracle.cvae_sample(shape, master64, stats, cond.astype(np.float64), 99, 1000)
    err64 = np.abs(got - ref64).max(axis=1) / scale.max()
    print(f"model {model}: error against the FP64 decoder median {np.median(err64):.2e}, p90 "
          f"{np.quantile(err64, 0.9):.2e}, max {err64.max():.2e} (bfloat16 unit roundoff {BF16_U:.2e})")
    # reduced-precision decoders against the exact one, in units of the
    # output's standard deviation: each output sums ~16 products of rounded
    # operands per layer over three layers, so a typical sample is off by a
    # fraction of the format's unit roundoff u and nine in ten by at most u
    # (measured median 0.23-0.35 u, p90 0.5-0.6 u)
    assert np.median(err64) < 0.5 * BF16_U and np.quantile(err64, 0.9) < BF16_U


def packed_scales(packed):
    """(out_scale, in_scale) of a packed decoder: the 4 + 4 floats after the
    header (8 int32) and the four 16-float standardisation blocks."""
    f = packed.cpu().view(torch.float32).numpy()
    return f[72:76].astype(np.float64), f[76:80].astype(np.float64)


@pytest.mark.parametrize("calibrated", [False, True])
@pytest.mark.parametrize("model", MODELS)
def test_sample_fp8_matches_fp8_emulating_oracle(msst, oracle, model, calibrated):
    """FP8 E4M3 decoders (per-layer weight scale max|W|/448, FP32 accumulation;
    with calibration rows also per-layer activation scales, powers of two)
    against the oracle rounding weights and layer inputs to E4M3 the same way,
    with the activation scales of its own calibration on the same rows.
    E4M3 keeps 4 significant bits (unit roundoff 2^-4), so rounding flips from
    FP32-vs-FP64 differences are rare but each moves an activation by ~6 %."""
    announce(f"cvae sample fp8 model={model} calibrated={calibrated}")
    shape = W.SHAPE_LIST[model]
    master64 = oracle.cvae_init(shape, seed=70 + model).astype(np.float32).astype(np.float64)
    stats = W.random_stats(model, seed=10 + model)
    n = 3000 + 21
    cond = W.random_conditions(model, n, seed=20 + model).astype(np.float32)
    packed = torch.empty(msst.cvae_packed_bytes(), dtype=torch.uint8, device="cuda")
    calib = cond[:1500]
    msst.cvae_pack(model, dev(master64), dev(stats, torch.float64), 2, packed,
                   calib=dev(calib) if calibrated else None)
    act = oracle.cvae_act_scales(shape, master64, stats, calib.astype(np.float64)) if calibrated else None
    out_sc, in_sc = packed_scales(packed)
    nl = shape["n_linear"]
    if calibrated:
        print(f"model {model}: activation scales {act}")
        np.testing.assert_array_equal(in_sc[:nl], 1.0 / act)
    else:
        np.testing.assert_array_equal(in_sc, 1.0)
    out = torch.empty((n, shape["p_out"]), dtype=torch.float32, device="cuda")
    msst.cvae_sample(packed, dev(cond), n, 5, 0, out)
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.cvae_sample(shape, master64, stats, cond.astype(np.float64), 5, 0, precision=oracle.PREC_FP8,
                             act_scales=act)
    scale = stats[48:48 + shape["p_out"]].max()
    err = np.abs(got - ref).max(axis=1) / scale
    print(f"model {model}: median {np.median(err):.2e}, p99 {np.quantile(err, 0.99):.2e}, max {err.max():.2e}")
    assert np.quantile(err, 0.99) < 1e-3
    assert err.max() < 0.2
    ref16 = oracle.cvae_sample(shape, master64, stats, cond.astype(np.float64), 5, 0, precision=oracle.PREC_BF16)
    e16 = np.abs(got - ref16).max(axis=1) / scale
    ref64 = oracle.cvae_sample(shape, master64, stats, cond.astype(np.float64), 5, 0)
    e64 = np.abs(got - ref64).max(axis=1) / scale
    print(f"model {model}: FP8 against the BF16 decoder: median {np.median(e16):.2e}; against FP64: median "
          f"{np.median(e64):.2e}, p90 {np.quantile(e64, 0.9):.2e} (E4M3 unit roundoff {FP8_U:.2e})")
    # the same rule as for bfloat16 with E4M3's unit roundoff (measured
    # median 0.14-0.37 u, p90 0.34-0.68 u)
    assert np.median(e64) < 0.5 * FP8_U and np.quantile(e64, 0.9) < FP8_U


@pytest.mark.parametrize("model", MODELS)
def test_resume_from_saved_state_is_bitwise(msst, tmp_path, model):
    announce(f"cvae training resumed from a saved state, model={model}")
    B, n_rows, steps, cut = 1024, 1 << 14, 12, 5
    p_in, p_out = [(2, 1), (3, 3), (7, 6)][model]
    rng = np.random.default_rng(40 + model)
    cd = dev(rng.normal(size=(n_rows, p_in)))
    td = dev(rng.normal(size=(n_rows, p_out)))
    stats = msst.make_stats(cd, td)
    n = msst.cvae_param_count(model)
    ws = torch.empty(msst.cvae_workspace_size(model, B), dtype=torch.uint8, device="cuda")

    def run(master, m, v, first, last):
        loss = torch.zeros(3, dtype=torch.float64, device="cuda")
        for step in range(first, last + 1):
            msst.cvae_train_step(model, master, m, v, msst.adam_params(step, lr=3e-3, weight_decay=0.01), cd, td,
                                 n_rows, B, 1, 31, step, 0, ws, loss, kl_weight=min(1.0, step / 8))
        return loss

    master = torch.empty(n, dtype=torch.float32, device="cuda")
    msst.cvae_init(model, 8, master)
    m, v = torch.zeros_like(master), torch.zeros_like(master)
    ref_loss = run(master, m, v, 1, steps)

    a = torch.empty(n, dtype=torch.float32, device="cuda")
    msst.cvae_init(model, 8, a)
    am, av = torch.zeros_like(a), torch.zeros_like(a)
    run(a, am, av, 1, cut)
    path = tmp_path / "state.safetensors"
    msst.save_training_state(path, model, a, am, av, cut, stats=stats, extra={"seed": 31})
    del a, am, av
    st = msst.load_training_state(path)
    assert st["step"] == cut and st["extra"] == {"seed": 31}
    assert torch.equal(st["stats"], stats)
    loss = run(st["master"], st["adam_m"], st["adam_v"], st["step"] + 1, steps)
    for k, ref in (("master", master), ("adam_m", m), ("adam_v", v)):
        assert torch.equal(st[k].view(torch.int32), ref.view(torch.int32)), k
    assert torch.equal(loss, ref_loss)


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_master_weight_shows_in_loss_and_gradient(msst, bad):
    """A non-finite master weight does not change the status; it reaches the
    loss and the gradient, where a caller tests for it."""
    announce(f"cvae non-finite master weight {bad}")
    model, B, n_rows = 1, 256, 4096
    rng = np.random.default_rng(6)
    cd, td = dev(rng.normal(size=(n_rows, 3))), dev(rng.normal(size=(n_rows, 3)))
    n = msst.cvae_param_count(model)
    master = torch.empty(n, dtype=torch.float32, device="cuda")
    msst.cvae_init(model, 3, master)
    ws = torch.empty(msst.cvae_workspace_size(model, B), dtype=torch.uint8, device="cuda")
    loss = torch.zeros(3, dtype=torch.float64, device="cuda")
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    msst.cvae_train_step(model, master, None, None, None, cd, td, n_rows, B, 0, 5, 1, 0, ws, loss, grad)
    assert torch.isfinite(loss).all() and torch.isfinite(grad).all()
    real = np.flatnonzero(_real_mask(W.SHAPE_LIST[model]))
    master[int(real[0])] = bad  # first weight of the encoder's first layer
    msst.cvae_train_step(model, master, None, None, None, cd, td, n_rows, B, 0, 5, 1, 0, ws, loss, grad)
    assert not torch.isfinite(loss[0]) and not torch.isfinite(grad).all()
