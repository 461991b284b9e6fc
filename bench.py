"""Benchmark: sphere-traced camera paths/s with the learned CVAE step against
plain random-walk (path tracing with next-event estimation) paths/s at
matched image RMSE, on the synthetic sphere + box scene (512 x 512,
256 samples per pixel, g = 0.8, albedo 0.995, sigma_t in {10, 20, 40, 80},
one point light).

One step = one sphere-traced render of the whole sweep (four images).  Before
the timed region the script generates CVAE training data with the GPU random
walk, trains the three CVAEs with the GPU forward/backward/AdamW kernels,
packs them to bfloat16, renders a high-sample plain reference per density and
times the plain tracer; after it, it reports the matched-RMSE speed-up,
roofline figures of the render kernel and the CPU oracle's rate.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU work per unit in 32-bit lane-operation slots (one per
# full-rate lane operation, four per quarter-rate one: transcendentals and
# 32-bit integer multiplies), from the operation count of the method:
#   plain collision: Philox block (10 rounds, 20 quarter-rate multiplies) 100,
#     uniforms 8, flight log 5, HG sample with its reciprocal 16, azimuth
#     sin/cos 8, orthonormal frame 16, rotation with rsq 22, position update
#     and exit test 13 (= 188, the walk event) plus the shadow ray to the
#     light (two primitive intervals ~100, exp and HG phase ~30, weight and
#     accumulation ~30) and the new ray's intervals: ~350;
#   learned step with one representative event: 7 Philox blocks ~700, 22
#     normals by Box-Muller ~240, 96 Softplus (two quarter-rate
#     transcendentals each) ~1150, standardisation, posterior noise and
#     de-standardisation ~250, exit frames ~120, shadow ray ~140: ~2600; each
#     further representative event adds its first-event block and an
#     EventGen decode (4 Philox blocks ~400, 10 normals ~110, 32 Softplus
#     ~380) and a shadow ray ~140: ~1000;
#   path: camera ray (one Philox block, pinhole direction) ~120, primary
#     intervals ~65, banking the sample ~15: ~200.
# achieved / peak is the fraction of the chip's lane slots the method's work
# would fill; the kernels' own counted slots (SQ_THREAD_CYCLES_VALU fit, see
# profiles/) are reported beside it.
ALG_PER_PATH = 200.0
ALG_PER_EVENT = 350.0
ALG_PER_STEP_ONE_EVENT = 2600.0
ALG_PER_EXTRA_EVENT = 1000.0
OPS_PER_PATH = 400.0         # counted: camera ray, primary intervals, banking the result
OPS_PER_EVENT = 460.0        # counted: one plain collision
OPS_PER_STEP = 5600.0        # counted: one learned step with one representative event
MFMA_FLOP_PER_STEP = 2944.0  # real decoder MACs x 2 (LengthGen + PathGen + EventGen)
OPS_PER_WALK_EVENT = 186.0   # one walk event: Philox block, HG sample, scatter, flight, exit test
PEAK_VALU_LANEOPS = 256 * 2.4e9 * 64   # 3.93e13 lane-op slots/s, non-packed FP32 VALU
CALIB_ROWS = 8192  # training conditions that calibrate the FP8 activation scales
PEAK_MFMA_BF16 = 2.5e15
PEAK_HBM_BYTES = 8.0e12
# active-lane VALU slots per decoded sample of cvae_sample for the standard
# shapes (latent 4, width 16, three layers), (model, precision 1 BF16 / 2 FP8)
SAMPLE_VALU_SLOTS = {(0, 1): 709.0, (0, 2): 793.0, (1, 1): 739.0, (1, 2): 823.0, (2, 1): 874.0, (2, 2): 958.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse(argv=None):
    """Command-line options (argv: a list in place of sys.argv)."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--train-samples", type=int, default=1 << 22)
    ap.add_argument("--ref-spp", type=int, default=4096)
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--spp", type=int, default=256)
    ap.add_argument("--tau-min", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--batch-min", type=int, default=0)
    ap.add_argument("--nee-samples", type=int, default=1)
    ap.add_argument("--nee-flags", type=int, default=1,
                    help="1 = direct light of learned steps before absorption, 2 = the paper's step as printed "
                         "(PathGen and EventGen for every step; the models are then trained on every walk record)")
    ap.add_argument("--min-chain", type=float, default=256.0,
                    help="cost rule: learned steps only where the deepest possible step bypasses at least this many "
                         "collisions (0 = always)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-table1", action="store_true")
    ap.add_argument("--table1-sweep", action="store_true",
                    help="also train and score every Table 1 architecture that fits one tile (untimed)")
    ap.add_argument("--no-absorption", action="store_true")
    ap.add_argument("--no-rgb", action="store_true")
    ap.add_argument("--no-mesh", action="store_true")
    ap.add_argument("--no-focus", action="store_true")
    ap.add_argument("--no-density", action="store_true")
    ap.add_argument("--jsonl", type=str, default=None,
                    help="also append the result line to this file (one JSON object per run)")
    ap.add_argument("--no-confirm", action="store_true", help="skip the plain tracer's run at the matched spp")
    ap.add_argument("--no-walk-full", action="store_true")
    ap.add_argument("--no-sample", action="store_true")
    ap.add_argument("--sample-rows", type=int, default=1 << 24)
    ap.add_argument("--walk-full-photons", type=int, default=1 << 24)
    ap.add_argument("--density-sigmas", type=str, default="80,160,320,640,1280")
    ap.add_argument("--density-albedo", type=float, default=0.9999)
    ap.add_argument("--density-width", type=int, default=256)
    ap.add_argument("--mesh-chunk", type=int, default=4,
                    help="samples per work unit in the mesh section (measured 7-8 %% faster than the renderer's "
                         "default of 8 at 512^2 x 256 spp)")
    ap.add_argument("--density-nee-samples", type=int, default=2,
                    help="representative events per learned step in the density sweep (its chains run to 10^4 "
                         "events, and a second event halves the heavy tail of their direct light)")
    ap.add_argument("--density-event-steps", type=int, default=100000,
                    help="AdamW steps of the EventGen beside the density sweep's default models (0: skip)")
    ap.add_argument("--absorption-sigma", type=float, default=80.0)
    ap.add_argument("--absorption-points", type=int, default=6)
    ap.add_argument("--restart-min", type=int, default=0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this size first (the reference kernel for HBM counters)")
    ap.add_argument("--c5-width", type=int, default=1024)
    ap.add_argument("--c5-spp", type=int, default=1024)
    ap.add_argument("--c5-ref-spp", type=int, default=4096)
    ap.add_argument("--no-oracle-anchor", action="store_true",
                    help="skip the FP64 oracle's plain renders of a regular pixel subset (z-test and RMSE anchor)")
    ap.add_argument("--oracle-spp", type=int, default=1024)
    ap.add_argument("--c5-oracle-spp", type=int, default=1024)
    ap.add_argument("--no-other-form", action="store_true",
                    help="skip the other form of the learned step (the paper's as printed when the default samples "
                         "the single-event parts exactly, and the reverse)")
    ap.add_argument("--diagnostics", action="store_true",
                    help="also render sphere tracing with exact in-sphere walks and a tau_min sweep (untimed)")
    return ap.parse_args(argv)


def train_models(M, torch, n_samples, steps, batch=4096, seed=0, kl_warmup=0.6, precision=1, shapes=None,
                 walk_kw=None):
    """Trains the three CVAEs (see train_and_pack) and returns (packed models
    in `precision`, per-model losses, seconds)."""
    packs, losses, t = train_and_pack(M, torch, n_samples, steps, batch, seed, kl_warmup, (precision,), shapes,
                                      walk_kw)
    return packs[precision], losses, t


def train_and_pack(M, torch, n_samples, steps, batch=4096, seed=0, kl_warmup=0.6, precisions=(1,), shapes=None,
                   walk_kw=None, timing=None, all_rows=False, model_steps=None):
    """GPU walk -> features -> FP64 standardisation -> AdamW training -> pack.

    The KL weight ramps linearly from 0 to 1 over the first kl_warmup of the
    steps (a guard against decoders that ignore the latent).  Returns
    ({precision: [three packed models]}, per-model losses, seconds).  shapes:
    three architecture dicts (default: width 16, three linear maps, latent 4);
    walk_kw: extra training-walk options (e.g. a focus region); timing: a dict
    that receives the walk's and the training steps' GPU times; model_steps:
    per-model step counts (LengthGen, PathGen, EventGen) in place of `steps`,
    each model on its own learning-rate and KL schedule."""
    t0 = time.time()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    walk = M.random_walk(n_samples, seed=seed, mode=1, **(walk_kw or {}))
    e1.record()
    torch.cuda.synchronize()
    if timing is not None:
        c = walk["counters"].cpu().numpy()
        timing["walk"] = dict(photons=n_samples, events=int(c[0]), seconds=e0.elapsed_time(e1) / 1e3)
    # the three models train at once, one stream each: a step is latency
    # bound (about one wave per CU), so their launches overlap on the GPU
    setups = [prepare_model(M, torch, walk, model, model if shapes is None else shapes[model], batch, seed,
                            all_rows=all_rows)
              for model in range(3)]
    streams = [torch.cuda.Stream() for _ in setups]
    cur = torch.cuda.current_stream()
    for st in streams:
        st.wait_stream(cur)
    n_steps = list(model_steps) if model_steps is not None else [steps] * 3
    t_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_ev[0].record()
    for step in range(1, max(n_steps) + 1):
        for su, st, n in zip(setups, streams, n_steps):
            if step <= n:
                train_step_model(M, su, step, n, kl_warmup, stream=st)
    for st in streams:
        cur.wait_stream(st)
    t_ev[1].record()
    torch.cuda.synchronize()
    if timing is not None:
        us = t_ev[0].elapsed_time(t_ev[1]) * 1e3 / max(n_steps)
        timing["train_step_us_three_models"] = us
        timing["train_samples_per_s_per_model"] = batch / (us * 1e-6)
    packs, losses = {p: [] for p in precisions}, []
    for su in setups:
        pk, loss = finish_model(M, torch, su, precisions)
        for p in precisions:
            packs[p].append(pk[p])
        losses.append(loss)
    torch.cuda.synchronize()
    if timing is not None:
        # the trained FP32 masters and standardisation constants, for the oracle
        timing["models"] = [dict(shape=dict(su["shape"]) if isinstance(su["shape"], dict) else
                                 dict(M.STANDARD_SHAPES[su["shape"]]),
                                 params=su["master"].double().cpu().numpy(), stats=su["stats"].cpu().numpy())
                            for su in setups]
    return packs, losses, time.time() - t0


def prepare_model(M, torch, walk, model, shape, batch=4096, seed=0, all_rows=False):
    """Features, FP64 standardisation, initial weights and AdamW state of one
    CVAE on the walk records."""
    n_samples = walk["n_scatter"].numel()
    p_in, p_out = [(2, 1), (3, 3), (7, 6)][model]
    # PathGen learns N >= 2 records and EventGen k >= 2 records: the
    # single-event cases are sampled exactly by the renderer (all_rows: every
    # record, for the paper's step as printed)
    rows = None if model == 0 or all_rows else M.select_rows(walk, 2, 2 if model == 2 else 0)
    n_rows = n_samples if rows is None else rows.numel()
    cond = torch.empty((n_rows, p_in), dtype=torch.float32, device="cuda")
    target = torch.empty((n_rows, p_out), dtype=torch.float32, device="cuda")
    M.cvae_features(model, n_rows, walk, seed + 1, 0, None, cond, target, rows=rows)
    stats = M.make_stats(cond, target)
    # raw conditions of the first rows: calibration of the FP8 activation scales
    calib = cond[:min(n_rows, CALIB_ROWS)].clone()
    M.cvae_features(model, n_rows, walk, seed + 1, 0, stats, cond, target, rows=rows)
    n = M.cvae_param_count(shape)
    master = torch.empty(n, dtype=torch.float32, device="cuda")
    M.cvae_init(shape, seed + 10 + model, master)
    return dict(model=model, shape=shape, n_rows=n_rows, cond=cond, target=target, stats=stats, master=master,
                calib=calib,
                m=torch.zeros_like(master), v=torch.zeros_like(master), batch=batch, seed=seed,
                ws=torch.empty(M.cvae_workspace_size(shape, batch), dtype=torch.uint8, device="cuda"),
                loss=torch.zeros(3, dtype=torch.float64, device="cuda"), first=None)


def train_step_model(M, su, step, steps, kl_warmup=0.6, stream=None):
    """One AdamW step (step = 1 .. steps) with the learning-rate schedule and
    the KL warm-up; keeps the first step's loss."""
    lr = 2e-3 if step < 0.5 * steps else (6e-4 if step < 0.8 * steps else 2e-4)
    beta = min(1.0, step / (kl_warmup * steps)) if kl_warmup > 0 else 1.0
    M.cvae_train_step(su["shape"], su["master"], su["m"], su["v"], M.adam_params(step, lr=lr), su["cond"],
                      su["target"], su["n_rows"], su["batch"], 1, su["seed"] + 20 + su["model"], step, 0, su["ws"],
                      su["loss"], stream=stream, kl_weight=beta)
    if step == 1:
        import torch
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            su["first"] = su["loss"].clone()


def finish_model(M, torch, su, precisions=(1,)):
    """Packs the trained model; returns ({precision: packed}, loss record)."""
    first, last = su["first"].cpu().numpy(), su["loss"].cpu().numpy().copy()
    packed = {}
    for p in precisions:
        pk = torch.empty(M.cvae_packed_bytes(), dtype=torch.uint8, device="cuda")
        M.cvae_pack(su["shape"], su["master"], su["stats"], p, pk, calib=su["calib"] if p == 2 else None)
        packed[p] = pk
    log(f"model {su['model']}: {su['n_rows']} rows, loss (total, KL, NLL) {first} -> {last}")
    return packed, dict(rows=int(su["n_rows"]), first=first.tolist(), last=last.tolist())


def train_one(M, torch, walk, model, shape, steps, batch=4096, seed=0, kl_warmup=0.6, precisions=(1,)):
    """Trains one CVAE on the walk records and packs it; returns ({precision:
    packed}, loss record)."""
    su = prepare_model(M, torch, walk, model, shape, batch, seed)
    for step in range(1, steps + 1):
        train_step_model(M, su, step, steps, kl_warmup)
    return finish_model(M, torch, su, precisions)


def table1_sweep(M, torch, W, n_samples, steps, n_eval=10000, seed=0):
    """The architecture sweep of Table 1: every examined (D, W, L) of each
    model (one 16-wide MFMA tile per layer, two for W = 20 or L = 9) is
    trained on the same walks, and its
    samples are compared with the walk on the Sec. 5.3 evaluation grid
    (sigma_t in {1, 4, 20, 100}, g in {-0.7, 0, 0.4, 0.9}, albedo 1) by the
    mean two-sample KS distance of log N (LengthGen), cos theta given the true
    N >= 2 (PathGen) and |X| given the true exit and N for k >= 2
    (EventGen)."""
    import numpy as np
    from scipy import stats as sps
    walk = M.random_walk(n_samples, seed=seed, mode=1)
    grid = [(s, g) for s in (1.0, 4.0, 20.0, 100.0) for g in (-0.7, 0.0, 0.4, 0.9)]
    truth = []
    for i, (s, g) in enumerate(grid):
        w = M.random_walk(n_eval, seed=900 + i, mode=1, st_range=(s, s), g_range=(g, g), albedo_range=(1.0, 1.0))
        truth.append({k: w[k].cpu().numpy().astype(np.float64) for k in ("n_scatter", "event_index", "exit_param",
                                                                          "event_pos")})

    def sample(pk, model, cond, sd):
        out = torch.empty((cond.shape[0], [1, 3, 6][model]), dtype=torch.float32, device="cuda")
        M.cvae_sample(pk, torch.as_tensor(cond, dtype=torch.float32).cuda(), cond.shape[0], sd, 0, out)
        return out.cpu().numpy().astype(np.float64)

    def score(pk, model):
        ks = []
        for i, ((s, g), t) in enumerate(zip(grid, truth)):
            n = t["n_scatter"]
            if model == 0:
                y = sample(pk, 0, np.stack([np.full(n.size, np.log(s)), np.full(n.size, g)], 1), 50 + i)[:, 0]
                nn = np.maximum(1.0, np.floor(np.exp(np.minimum(y, 20.0)) + 0.5))
                ks.append(sps.ks_2samp(np.log(n), np.log(nn)).statistic)
                continue
            sel = (n >= 2) if model == 1 else (n >= 2) & (t["event_index"] >= 2)
            if sel.sum() < 200:
                continue
            ep = t["exit_param"][:, sel]
            base = [np.full(sel.sum(), np.log(s)), np.full(sel.sum(), g)]
            if model == 1:
                y = sample(pk, 1, np.stack(base + [np.log(n[sel])], 1), 50 + i)
                ks.append(sps.ks_2samp(ep[0], np.clip(y[:, 0], -1, 1)).statistic)
            else:
                cond = np.stack(base + [np.ones(sel.sum()), ep[0], ep[1], ep[2], np.log(n[sel])], 1)
                y = sample(pk, 2, cond, 50 + i)
                xl = np.minimum(np.linalg.norm(y[:, :3], axis=1), 1.0)
                ks.append(sps.ks_2samp(np.linalg.norm(t["event_pos"][:, sel], axis=0), xl).statistic)
        return float(np.mean(ks))

    rows = []
    for model in range(3):
        gspec = W.TABLE1_GRID[model]
        for D in gspec["D"]:
            for Wd in gspec["W"]:
                for L in gspec["L"]:
                    shape = W.table1_shape(model, D, Wd, L)
                    row = dict(model=model, D=D, W=Wd, L=L, final=W.TABLE1_FINAL[model] == dict(D=D, W=Wd, L=L))
                    if not W.table1_fits(shape):
                        row["built"] = False
                        rows.append(row)
                        continue
                    pk, loss = train_one(M, torch, walk, model, shape, steps, seed=seed)
                    row.update(built=True, ks=score(pk[1], model), loss=loss["last"][0])
                    log(f"Table 1 sweep model {model} D={D} W={Wd} L={L}: mean KS {row['ks']:.3f}")
                    rows.append(row)
    return rows


RENDER_SOURCES = ("paper_2011_03082_amd/csrc/render.hip", "paper_2011_03082_amd/csrc/device.hpp",
                  "paper_2011_03082_amd/csrc/packed.hpp", "paper_2011_03082_amd/csrc/mfma.hpp")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "render_kernel_hbm_traffic.md")


def render_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in RENDER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per render launch of the timed workload from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when that summary is
    missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source digest") != render_source_digest():
        return None
    try:
        return float(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def primary_hit_labels(cam, prims):
    """Per pixel of the camera (row-major, pixel centres): 0 where the primary
    ray misses every primitive, else 1 + the index of the primitive it enters
    first (pinhole camera of the renderer's ABI: forward, right and up axes
    scaled by tan(vfov / 2) and the aspect ratio).  Measurement only: it
    splits a render's per-pixel event and step counters by the part of the
    body a pixel sees, the voluminous sphere or the thin box arm of the
    sphere + box scene (the stand-in for the two kinds of geometry whose
    event counts Sec. 5.4 compares)."""
    import numpy as np
    w, h = int(cam["width"]), int(cam["height"])
    eye = np.asarray(cam["eye"], np.float64)
    f = np.asarray(cam["look_at"], np.float64) - eye
    f /= np.linalg.norm(f)
    rt = np.cross(f, np.asarray(cam["up"], np.float64))
    rt /= np.linalg.norm(rt)
    uv = np.cross(rt, f)
    th = np.tan(0.5 * np.radians(cam["vfov_deg"]))
    px, py = np.meshgrid(np.arange(w) + 0.5, np.arange(h) + 0.5)
    sx, sy = 2.0 * px / w - 1.0, 1.0 - 2.0 * py / h
    d = f + (sx * th * w / h)[..., None] * rt + (sy * th)[..., None] * uv
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    best = np.full((h, w), np.inf)
    label = np.zeros((h, w), np.int32)
    for i, p in enumerate(np.asarray(prims, np.float64)):
        q = eye - p[1:4]
        if p[0] == 0.0:  # sphere: nearest root of |q + t d|^2 = r^2
            b = d @ q
            disc = b * b - (q @ q - p[4] ** 2)
            with np.errstate(invalid="ignore"):
                t0, t1 = -b - np.sqrt(disc), -b + np.sqrt(disc)
            hit = (disc > 0.0) & (t1 > 0.0)
            t = np.where(t0 > 0.0, t0, t1)
        else:  # box: slabs
            with np.errstate(divide="ignore", invalid="ignore"):
                ta = (-p[4:7] - q) / d
                tb = (p[4:7] - q) / d
            lo = np.nanmax(np.minimum(ta, tb), axis=-1)
            hi = np.nanmin(np.maximum(ta, tb), axis=-1)
            hit = (lo < hi) & (hi > 0.0)
            t = np.where(lo > 0.0, lo, hi)
        nearer = hit & (t < best)
        best = np.where(nearer, t, best)
        label = np.where(nearer, i + 1, label)
    return label.reshape(-1)


def region_counts(img, labels, spp, names):
    """Events and sphere steps per path over the pixels of each label
    (names: {label: name}): mean, 99th percentile and maximum of the
    per-pixel means."""
    import numpy as np
    ev = img["events"].cpu().numpy().astype(np.float64) / spp
    st = img["steps"].cpu().numpy().astype(np.float64) / spp
    out = {}
    for lab, name in names.items():
        m = labels == lab
        if not m.any():
            continue
        out[name] = dict(pixels=int(m.sum()), events_per_path=float(ev[m].mean()),
                         events_p99=float(np.percentile(ev[m], 99)), events_max=float(ev[m].max()),
                         steps_per_path=float(st[m].mean()), steps_p99=float(np.percentile(st[m], 99)))
    return out


def image_moments(img, spp):
    s = img["sum"].double() + img["comp"].double()
    mean = s / spp
    var = img["sumsq"].double() / spp - mean * mean
    return mean, var.clamp_min(0)


def oracle_threads():
    """Host threads for the oracle: the process's CPU share (OMP_NUM_THREADS
    where set, as on the GPU hosts), else the visible cores, at most 64."""
    n = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(n if n > 0 else (os.cpu_count() or 1), 64))


def cpu_model_name():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def default_chunk(npix, spp):
    """The renderer's default samples per work unit (the rule its C header
    states for ms_render_desc.chunk = 0)."""
    c = min(64, -(-npix * spp // (1 << 23)))
    if npix * -(-spp // c) > (1 << 24):
        c = -(-npix * spp // (1 << 24))
    return min(spp, max(2, c))


def subset_pixels(width, height, stride=16):
    """Every stride-th pixel in x and y (the centre of each stride x stride block)."""
    import numpy as np
    return np.array([y * width + x for y in range(stride // 2, height, stride)
                     for x in range(stride // 2, width, stride)], np.int32)


def oracle_subset(oracle, scene, cam, light, med, spp, seed, stride=16):
    """FP64 plain path tracing with next-event estimation on every
    stride-th pixel in x and y: per-pixel mean and one-sample variance."""
    import numpy as np
    pix = subset_pixels(cam["width"], cam["height"], stride)
    t0 = time.time()
    o = oracle.render(scene, cam, light, med, method=oracle.METHOD_PLAIN_NEE, spp=spp, seed=seed, pixels=pix,
                      n_threads=oracle_threads())
    mean = o["sum"] / spp
    return dict(pix=pix, mean=mean, var=np.maximum(o["sumsq"] / spp - mean * mean, 0.0), spp=spp,
                seconds=time.time() - t0)


def anchor_stats(sub, ref_mean, ref_var, ref_spp, images, pt_var):
    """The GPU reference against the oracle subset: per-pixel z = (R - O) /
    sqrt(var R / n_R + var O / n_O) over pixels with any light (RMS ~1 and a
    global z of the summed difference within a few units when both estimate
    the same image), each image's RMSE against the oracle with the
    oracle's own noise removed (images: name -> per-pixel means, numpy), and
    the plain tracer's mean one-sample variance on the same pixels (pt_var:
    its per-pixel variance image), which a matched-RMSE comparison on the
    subset sets against those RMSEs."""
    import numpy as np
    p = sub["pix"]
    ov = sub["var"] / sub["spp"]
    rv = ref_var[p] / ref_spp
    d = ref_mean[p] - sub["mean"]
    v = rv + ov
    # pixels with any light; radiances near 1e-20 have squares that flush to
    # zero in the GPU's binary32 sums, so variances below 1e-12 of the largest
    # are taken as none (such pixels add nothing to any RMSE either)
    lit = v > 1e-12 * v.max()
    z = d[lit] / np.sqrt(v[lit])
    out = dict(pixels=int(p.size), lit_pixels=int(lit.sum()), oracle_spp=sub["spp"], oracle_seconds=sub["seconds"],
               z_rms=float(np.sqrt(np.mean(z * z))), z_mean=float(z.mean()), z_max=float(np.abs(z).max()),
               z_global=float(d[lit].sum() / np.sqrt(v[lit].sum())),
               reference_rmse_vs_oracle=float(np.sqrt(max(np.mean(d * d) - ov.mean(), 1e-30))),
               pt_var_subset=float(pt_var[p].mean()))
    for name, m in images.items():
        e2 = float(np.mean((m[p] - sub["mean"]) ** 2) - ov.mean())
        out[f"rmse_{name}_vs_oracle"] = float(np.sqrt(max(e2, 1e-30)))
        # the same pixels against the GPU reference: equal within noise when
        # the reference is unbiased, whatever the subset's own sampling error
        e2r = float(np.mean((m[p] - ref_mean[p]) ** 2) - rv.mean())
        out[f"rmse_{name}_vs_reference_on_subset"] = float(np.sqrt(max(e2r, 1e-30)))
    return out


def c5_section(M, W, torch, packs, args, timed):
    """64-sphere scene over a 256^3 FP16 distance grid, 1024^2 x 1024 spp,
    sigma_t = 100: sphere tracing with FP8 and BF16 decoders against the plain
    tracer; image error against a high-sample plain render (whose own noise is
    subtracted)."""
    import numpy as np
    width, spp, res = args.c5_width, args.c5_spp, 256
    prims = W.scene_c5(seed=0)
    grid = M.build_sdf_grid(prims, res)
    cam, light, med = W.camera_c5(width, width), W.light_c5(), W.medium_c5()
    rend = M.Renderer(prims, cam, light, grid=grid)
    img, t_ref = timed(lambda: rend.render(med, method=1, spp=args.c5_ref_spp, seed=77), warm=False)
    ref, ref_var = image_moments(img, args.c5_ref_spp)
    means = {}
    ref_noise2 = float(ref_var.mean()) / args.c5_ref_spp
    out = {"workload": f"64 spheres (seed 0) over a {res}^3 FP16 distance grid, {width}x{width}, {spp} spp, "
                       f"sigma_t=100, g=0.8, albedo=0.995, point light + NEE",
           "reference": f"plain tracer at {args.c5_ref_spp} spp ({t_ref:.1f} s)"}
    runs = [("pt", dict(method=1)), ("st_bf16", dict(method=2, packed=packs[1])),
            ("st_fp8", dict(method=2, packed=packs[2]))]
    for name, opt in runs:
        if opt["method"] == 2:
            opt.update(tau_min=args.tau_min, nee_samples=args.nee_samples, flags=args.nee_flags,
                       min_chain=args.min_chain)
        rend.render(med, spp=16, seed=5, **opt)  # warm-up
        img, t = timed(lambda: rend.render(med, spp=spp, seed=6, **opt))
        c = img["counters"].cpu().numpy()
        mean, var = image_moments(img, spp)
        means[name] = mean.cpu().numpy()
        if name == "pt":
            pt_var_np = var.cpu().numpy()
        err2 = float(((mean - ref) ** 2).mean())
        rm = float(np.sqrt(max(err2 - ref_noise2, 1e-30)))
        out[name] = dict(ms=t * 1e3, paths_per_s=float(c[0] / t), events_per_path=float(c[1] / c[0]),
                         steps_per_path=float(c[2] / c[0]), rmse=rm, mean_var=float(var.mean()),
                         mean=float(mean.mean()))
        log(f"C5 {name}: {t * 1e3:.1f} ms, {c[0] / t:.3e} paths/s, RMSE {rm:.3e}")
    out["ref_mean"] = float(ref.mean())
    out["ref_noise_rms"] = float(np.sqrt(ref_noise2))
    pt = out["pt"]
    for name in ("st_bf16", "st_fp8"):
        r = out[name]
        s_star = pt["mean_var"] / max(r["rmse"] ** 2, 1e-30)
        r["speedup_matched_rmse"] = s_star * width * width / pt["paths_per_s"] / (r["ms"] / 1e3)
    if not args.no_oracle_anchor:
        import oracle
        log(f"C5 oracle anchor: every 16th pixel at {args.c5_oracle_spp} spp")
        sub = oracle_subset(oracle, oracle.Scene(prims), cam, light, med, args.c5_oracle_spp, 78, stride=16)
        out["oracle_anchor"] = anchor_stats(sub, ref.cpu().numpy(), ref_var.cpu().numpy(), args.c5_ref_spp, means,
                                            pt_var_np)
        a = out["oracle_anchor"]
        for name in ("st_bf16", "st_fp8"):
            r = out[name]
            r["speedup_matched_rmse_oracle"] = (a["pt_var_subset"] / a[f"rmse_{name}_vs_oracle"] ** 2 * width * width
                                                / pt["paths_per_s"] / (r["ms"] / 1e3))
        log(f"C5 oracle anchor: z rms {a['z_rms']:.2f}, global z {a['z_global']:+.2f}; RMSE vs oracle "
            + ", ".join(f"{n} {a[f'rmse_{n}_vs_oracle']:.3e}" for n in means))
    return out


def c4_tau(sigma_t, args, g=0.8, r_max=0.999):
    """tau_min of a sphere + box launch as the render kernel applies it: the
    cost rule (min_chain) turns learned steps off where even the deepest
    sphere (the unit sphere's centre, radius 0.999 after the 0.1 % shrink)
    bypasses too few collisions."""
    t_max = sigma_t * min(r_max, 200.0 / sigma_t)
    if args.min_chain > 0 and 0.5 * t_max * t_max * (1.0 - g) < args.min_chain:
        return 1e30
    return args.tau_min


def cpu_baseline(oracle, W, args, models):
    """The oracle's sphere tracer with the CVAE step (FP64 decoders on the same
    trained FP32 masters and standardisation constants the GPU renders) on
    random pixel subsets of the four timed images, same estimator options:
    all host threads of the process's CPU share for about args.cpu_seconds,
    then one thread for a quarter of that."""
    import numpy as np
    threads = oracle_threads()
    prims = W.scene_c4()
    cam = W.camera_c4(args.width, args.width)
    light = W.light_c4()
    scene = oracle.Scene(prims)
    rng = np.random.default_rng(0)
    spp = 4

    def run(n_threads, seconds):
        paths, t_total, it, npx = 0, 0.0, 0, 64
        while t_total < seconds:
            for s in W.C4_SIGMAS:
                pix = np.sort(rng.choice(args.width * args.width, npx, replace=False)).astype(np.int32)
                t0 = time.time()
                oracle.render(scene, cam, light, W.medium_c4(s), method=oracle.METHOD_ST,
                              sampler=oracle.SAMPLER_CVAE, models=models, tau_min=c4_tau(s, args), spp=spp,
                              seed=50 + it, pixels=pix, n_threads=n_threads, nee_samples=args.nee_samples,
                              flags=args.nee_flags)
                t_total += time.time() - t0
                paths += npx * spp
            npx = min(2 * npx, 1 << 14)
            it += 1
        return paths, t_total

    paths, t_all = run(threads, args.cpu_seconds)
    paths1, t_one = run(1, args.cpu_seconds / 4)
    return {"value": paths / t_all, "unit": "paths/s", "cores": threads, "kind": "oracle",
            "single_core_paths_per_s": paths1 / t_one, "cpu_model": cpu_model_name(),
            "sample": f"{paths} paths (random pixel subsets x {spp} spp of each of the four sigma_t images, "
                      f"sigma_t in {list(W.C4_SIGMAS)}) of the timed workload: ST + CVAE decoders in FP64 on the "
                      f"trained FP32 masters and standardisation constants the GPU renders, tau_min "
                      f"{args.tau_min}, {args.nee_samples} representative events; {t_all:.1f} s on {threads} "
                      f"threads; single thread {paths1} paths in {t_one:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding over GPUs by Philox id "
              "ranges is designed but not implemented", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2011_03082_amd as M
    import workloads as W

    torch.cuda.set_device(0)
    M.lib()
    width, spp = args.width, args.spp
    sigmas = W.C4_SIGMAS
    rend = M.Renderer(W.scene_c4(), W.camera_c4(width, width), W.light_c4())
    npix = width * width
    stream = torch.cuda.current_stream()
    kw = dict(blocks_per_cu=args.blocks_per_cu, cvae_batch_min=args.batch_min, chunk=args.chunk,
              restart_min=args.restart_min)

    def timed(fn, warm=True):
        # one untimed call first (buffers, caches), then the timed one: every
        # tracer is timed warm
        if warm:
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / 1e3

    def timed_images(fns):
        # the calls queued back to back behind an untimed run of the first, so
        # that no interval holds the host's enqueue time (as the sphere
        # tracer's timed steps run back to back): their outputs and mean time
        fns[0]()
        evs, outs = [], []
        for fn in fns:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            outs.append(fn())
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        return outs, float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs])) / 1e3

    def timed_mean(fn, reps):
        # reps identical calls: the last output and the mean time
        outs, t = timed_images([fn] * max(1, reps))
        return outs[-1], t

    def rmse(img, s):
        mean, _ = image_moments(img, spp)
        return float(torch.sqrt(((mean.float() - ref[s]) ** 2).mean()))

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log("training CVAEs on GPU random-walk data")
    tim = {}
    paper_step = bool(args.nee_flags & 2)
    packs, losses, t_train = train_and_pack(M, torch, args.train_samples, args.train_steps, precisions=(1, 2),
                                            timing=tim, all_rows=paper_step)
    packed = packs[1]

    # plain reference (debiased by its own noise) and plain timing per density
    ref, ref_noise2, pt, ref_var_np, pt_mean_np, pt_var_np = {}, {}, {}, {}, {}, {}
    for s in sigmas:
        med = W.medium_c4(s)
        img = rend.render(med, method=1, spp=args.ref_spp, seed=1000, **kw)
        mean, var = image_moments(img, args.ref_spp)
        ref[s] = mean.float()
        ref_var_np[s] = var.cpu().numpy()
        ref_noise2[s] = float(var.mean()) / args.ref_spp
        img, t = timed_mean(lambda: rend.render(med, method=1, spp=spp, seed=2000, **kw), args.steps)
        pm_, var = image_moments(img, spp)
        pt_mean_np[s] = pm_.cpu().numpy()
        pt_var_np[s] = var.cpu().numpy()
        c = img["counters"].cpu().numpy()
        pt[s] = dict(time=t, paths=int(c[0]), events=int(c[1]), var=float(var.mean()), rmse=rmse(img, s))
        log(f"PT sigma_t={s}: {t * 1e3:.1f} ms, {c[0] / t:.3e} paths/s, events/path {c[1] / c[0]:.2f}")

    def st_render(s, seed, **extra):
        opts = dict(method=2, sampler=0, packed=packed, spp=spp, seed=seed, tau_min=args.tau_min,
                    nee_samples=args.nee_samples, flags=args.nee_flags, min_chain=args.min_chain)
        opts.update(kw)
        opts.update(extra)
        return rend.render(W.medium_c4(s), **opts)

    def st_scored(s, seed0, **extra):
        # args.steps sphere-traced images, one seed each, timed back to back:
        # the last image, the mean time, the RMSE (mean square over the images,
        # the reference's own noise removed) and the mean of the image means
        ims, t = timed_images([(lambda j=j: st_render(s, seed0 + 100000 * j, **extra))
                               for j in range(max(1, args.steps))])
        e2 = float(np.mean([rmse(im, s) ** 2 for im in ims]))
        r = float(np.sqrt(max(e2 - ref_noise2[s], 1e-30)))
        m = float(np.mean([float(image_moments(im, spp)[0].mean()) for im in ims]))
        return ims[-1], t, r, m

    for w in range(args.warmup):
        for s in sigmas:
            st_render(s, 3000 + w)
    torch.cuda.synchronize()
    mk = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    ev = [[mk() for _ in sigmas] for _ in range(args.steps)]
    t_start = time.time()
    last, outs = {}, {s: [] for s in sigmas}
    for k in range(args.steps):
        for i, s in enumerate(sigmas):
            ev[k][i][0].record(stream)
            last[s] = st_render(s, 4000 + k)
            ev[k][i][1].record(stream)
            outs[s].append(last[s])
    torch.cuda.synchronize()
    wall = time.time() - t_start
    t_sigma = {s: float(np.mean([ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(args.steps)])) / 1e3
               for i, s in enumerate(sigmas)}
    ms_per_step = sum(t_sigma.values()) * 1e3
    paths_per_step = npix * spp * len(sigmas)
    value = paths_per_step / (ms_per_step / 1e3)

    # matched RMSE: the plain tracer needs S* = mean per-pixel variance /
    # RMSE_ST^2 samples per pixel (RMSE_ST with the reference's own noise
    # removed) to reach the sphere tracer's error, at its measured rate.
    # RMSE_ST^2 is the mean over the timed steps' images (one seed each): a
    # learned step lights a whole chain from one event, so its squared error
    # is heavy-tailed and one image estimates it less steadily
    details, counters = {}, np.zeros(4)
    tot_st, tot_pt = 0.0, 0.0
    for s in sigmas:
        img = last[s]
        c = img["counters"].cpu().numpy()
        counters += c
        r_raw2 = float(np.mean([rmse(im, s) ** 2 for im in outs[s]]))
        r_st = float(np.sqrt(max(r_raw2 - ref_noise2[s], 1e-30)))
        r_pt = float(np.sqrt(max(pt[s]["rmse"] ** 2 - ref_noise2[s], 1e-30)))
        s_star = pt[s]["var"] / r_st**2
        t_pt_match = s_star * npix / (pt[s]["paths"] / pt[s]["time"])
        mean_st = float(np.mean([float(image_moments(im, spp)[0].mean()) for im in outs[s]]))
        # confirmation: the plain tracer actually run at ceil(S*) spp (its own
        # seed), its RMSE and time beside the sphere tracer's
        s_conf = max(1, int(np.ceil(s_star)))
        confirm = None
        if not args.no_confirm:
            med_s = W.medium_c4(s)
            # the timed renders' samples per work unit (the header's default
            # rule at spp), so that only the sample count differs
            unit = args.chunk or default_chunk(npix, spp)
            kw_c = dict(kw, chunk=min(unit, s_conf))
            img_c, t_c = timed_mean(lambda: rend.render(med_s, method=1, spp=s_conf, seed=2501, **kw_c), args.steps)
            mc, _ = image_moments(img_c, s_conf)
            r_conf = float(np.sqrt(max(float(((mc.float() - ref[s]) ** 2).mean()) - ref_noise2[s], 1e-30)))
            confirm = dict(spp=s_conf, rmse=r_conf, ms=t_c * 1e3, speedup=t_c / t_sigma[s])
        details[str(s)] = dict(
            pt_confirm=confirm,
            rmse_st=r_st, rmse_pt_same_spp=r_pt, ref_noise_rms=float(np.sqrt(ref_noise2[s])),
            mean_st=mean_st, mean_ref=float(ref[s].double().mean()),
            mean_bias=mean_st / float(ref[s].double().mean()) - 1.0,
            st_paths_per_s=float(c[0] / t_sigma[s]), st_steps_per_path=float(c[2] / c[0]),
            st_events_per_path=float(c[1] / c[0]), pt_events_per_path=pt[s]["events"] / pt[s]["paths"],
            pt_paths_per_s=pt[s]["paths"] / pt[s]["time"], matched_spp_pt=s_star,
            speedup_matched_rmse=t_pt_match / t_sigma[s])
        log(f"ST sigma_t={s}: {t_sigma[s] * 1e3:.1f} ms, rmse {r_st:.3e} (PT@{spp} {r_pt:.3e}), "
            f"mean {mean_st:.4e} vs ref {details[str(s)]['mean_ref']:.4e}, matched PT spp {s_star:.1f}, "
            f"speed-up {t_pt_match / t_sigma[s]:.2f}"
            + ("" if confirm is None else f"; plain run at {s_conf} spp: rmse {confirm['rmse']:.3e}, "
               f"{confirm['ms']:.1f} ms ({confirm['speedup']:.2f})"))
        tot_st += t_sigma[s]
        tot_pt += t_pt_match
    # FP64 oracle anchor: the oracle's plain tracer on every 4th pixel in x and
    # y of each image (16384 pixels); z-test of the GPU reference, RMSE of both
    # tracers against it, and the matched-RMSE speed-up on those pixels alone.
    # Many pixels at fewer samples: a learned step's direct light comes from one
    # representative event weighted by the whole bypassed chain, so a few pixels
    # carry much of the sphere tracer's squared error, and a sparser subset
    # misestimates it by up to 15 % (1/64 of the pixels at sigma_t 80)
    if not args.no_oracle_anchor:
        import oracle
        o_scene = oracle.Scene(W.scene_c4())
        tot_st_o, tot_pt_o = 0.0, 0.0
        for i, s in enumerate(sigmas):
            sub = oracle_subset(oracle, o_scene, W.camera_c4(width, width), W.light_c4(), W.medium_c4(s),
                                args.oracle_spp, 11000 + i, stride=4)
            ims = {f"st{j}": image_moments(im, spp)[0].cpu().numpy() for j, im in enumerate(outs[s])}
            a = anchor_stats(sub, ref[s].double().cpu().numpy(), ref_var_np[s], args.ref_spp,
                             dict(ims, pt=pt_mean_np[s]), pt_var_np[s])
            # the sphere tracer's error on the subset: the mean square over its images
            for key in ("vs_oracle", "vs_reference_on_subset"):
                a[f"rmse_st_{key}"] = float(np.sqrt(np.mean([a.pop(f"rmse_{j}_{key}") ** 2 for j in ims])))
            t_pt_o = a["pt_var_subset"] / a["rmse_st_vs_oracle"] ** 2 * npix / (pt[s]["paths"] / pt[s]["time"])
            a["speedup_matched_rmse_oracle"] = t_pt_o / t_sigma[s]
            details[str(s)]["oracle_anchor"] = a
            tot_st_o += t_sigma[s]
            tot_pt_o += t_pt_o
            log(f"oracle anchor sigma_t={s}: {a['lit_pixels']} lit of {a['pixels']} pixels at {args.oracle_spp} spp "
                f"({a['oracle_seconds']:.1f} s): z rms {a['z_rms']:.2f}, global z {a['z_global']:+.2f}; RMSE vs oracle "
                f"ST {a['rmse_st_vs_oracle']:.3e}, PT {a['rmse_pt_vs_oracle']:.3e}, speed-up "
                f"{a['speedup_matched_rmse_oracle']:.2f}")
    pt_rate = sum(pt[s]["paths"] for s in sigmas) / sum(pt[s]["time"] for s in sigmas)
    # share of camera paths that hit the object: an opaque, black medium (albedo
    # below 2^-24: the roulette ends every path at its first collision)
    # (every hitting path has exactly one collision and is absorbed there)
    hit = rend.render(dict(sigma_t=1e6, g=0.0, albedo=1e-9), method=1, spp=16, seed=8000)
    hc = hit["counters"].cpu().numpy()
    hit_fraction = float(hc[1] / hc[0])

    # the paper's final architectures (Table 1) on the same data and images
    table1 = None
    if not args.no_table1:
        log("Table 1 final architectures")
        pk1, losses1, t1 = train_and_pack(M, torch, args.train_samples, args.train_steps,
                                          shapes=W.TABLE1_SHAPES, all_rows=paper_step)
        table1 = {"shapes": W.TABLE1_SHAPES, "train_seconds": t1,
                  "loss_last": [l["last"] for l in losses1]}
        for s in sigmas:
            img, t, r_st, _ = st_scored(s, 6001, packed=pk1[1])
            s_star = pt[s]["var"] / r_st**2
            t_pt_match = s_star * npix / (pt[s]["paths"] / pt[s]["time"])
            table1[str(s)] = dict(ms=t * 1e3, rmse_st=r_st, speedup_matched_rmse=t_pt_match / t,
                                  rmse_st_default_arch=details[str(s)]["rmse_st"])
            log(f"Table 1 sigma_t={s}: {t * 1e3:.1f} ms, rmse {r_st:.3e} (default {details[str(s)]['rmse_st']:.3e}), "
                f"speed-up {t_pt_match / t:.2f}")

    # the other form of the learned step, same images and estimator options
    # otherwise: the paper's step as printed (PathGen and EventGen for every
    # case, models trained on every walk record) beside the default with the
    # single-event parts sampled exactly, or the reverse
    other = None
    if not args.no_other_form:
        o_flags = args.nee_flags ^ 2
        o_paper = bool(o_flags & 2)
        name = "the paper's step as printed" if o_paper else "exact single-event parts"
        log(f"learned step, other form: {name}")
        pko, _, to = train_and_pack(M, torch, args.train_samples, args.train_steps, all_rows=o_paper)
        other = {"form": name, "flags": o_flags, "nee_samples": args.nee_samples, "train_seconds": to}
        tot_o, tot_om = 0.0, 0.0
        for s in sigmas:
            img, t, r_st, mean_o = st_scored(s, 6201, packed=pko[1], flags=o_flags)
            c = img["counters"].cpu().numpy()
            t_m = pt[s]["var"] / r_st**2 * npix / (pt[s]["paths"] / pt[s]["time"])
            other[str(s)] = dict(ms=t * 1e3, rmse_st=r_st, steps_per_path=float(c[2] / c[0]), mean_st=mean_o,
                                 mean_bias=mean_o / details[str(s)]["mean_ref"] - 1.0,
                                 speedup_matched_rmse=t_m / t, rmse_st_default=details[str(s)]["rmse_st"])
            tot_o += t
            tot_om += t_m
            log(f"{name} sigma_t={s}: {t * 1e3:.1f} ms, rmse {r_st:.3e} (default {details[str(s)]['rmse_st']:.3e}), "
                f"bias {other[str(s)]['mean_bias']:+.4f}, speed-up {t_m / t:.2f}")
        other["speedup_matched_rmse"] = tot_om / tot_o

    # (sigma_t r, g)-weighted training data: half the walks from the region
    # the renders use (g near 0.8, sigma_t r above tau_min)
    focus = None
    if not args.no_focus:
        log("focus-weighted training data")
        fkw = dict(focus_fraction=0.5, focus_st_range=(args.tau_min, 200.0), focus_g_range=(0.7, 0.9))
        pkf, _, tf = train_and_pack(M, torch, args.train_samples, args.train_steps, walk_kw=fkw,
                                    all_rows=paper_step)
        focus = dict(fkw, train_seconds=tf)
        for s in sigmas:
            img, t, r_st, _ = st_scored(s, 6101, packed=pkf[1])
            s_star = pt[s]["var"] / r_st**2
            focus[str(s)] = dict(ms=t * 1e3, rmse_st=r_st,
                                 speedup_matched_rmse=s_star * npix / (pt[s]["paths"] / pt[s]["time"]) / t)
            log(f"focus sigma_t={s}: {t * 1e3:.1f} ms, rmse {r_st:.3e}, speed-up "
                f"{focus[str(s)]['speedup_matched_rmse']:.2f}")

    # RGB medium: one (sigma_t, albedo) per colour channel, each channel its
    # own trace (Philox key seed + c); speed-up at matched RMSE per channel
    rgb = None
    if not args.no_rgb:
        media = [dict(sigma_t=s_, g=0.8, albedo=a_) for s_, a_ in ((20.0, 0.999), (40.0, 0.995), (80.0, 0.99))]
        ref_rgb = rend.render_rgb(media, method=1, spp=args.ref_spp // 2, seed=9000, **kw)
        rgb = {"media": media}
        img_pt, t_pt = timed(lambda: rend.render_rgb(media, method=1, spp=spp, seed=9100, **kw))
        img_st, t_st = timed(lambda: rend.render_rgb(media, method=2, sampler=0, packed=packed, spp=spp, seed=9200,
                                                     tau_min=args.tau_min, nee_samples=args.nee_samples,
                                                     flags=args.nee_flags, min_chain=args.min_chain, **kw))
        e2_st = e2_pt = v_pt = 0.0
        for c in range(3):
            pick = lambda im: {k: v[c] for k, v in im.items() if k != "counters"}
            rm, rv = image_moments(pick(ref_rgb), args.ref_spp // 2)
            noise2 = float(rv.mean()) / (args.ref_spp // 2)
            pm, pv = image_moments(pick(img_pt), spp)
            sm, _ = image_moments(pick(img_st), spp)
            e2_st += max(float(((sm - rm) ** 2).mean()) - noise2, 1e-30)
            e2_pt += max(float(((pm - rm) ** 2).mean()) - noise2, 1e-30)
            v_pt += float(pv.mean())
        rgb.update(pt_ms=t_pt * 1e3, st_ms=t_st * 1e3, rmse_pt=float(np.sqrt(e2_pt / 3)), rmse_st=float(np.sqrt(e2_st / 3)),
                   speedup_matched_rmse=(v_pt / e2_st) / spp * t_pt / t_st)
        log(f"RGB: PT {t_pt * 1e3:.1f} ms, ST {t_st * 1e3:.1f} ms, rmse {rgb['rmse_pt']:.2e} / {rgb['rmse_st']:.2e}, "
            f"speed-up {rgb['speedup_matched_rmse']:.2f}")

    # a closed triangle mesh (a star-shaped body with a thin spike, 20 480
    # triangles through the BVH), radii from a 128^3 grid built on the mesh
    mesh = None
    if not args.no_mesh:
        tris = W.mesh_blob(0, 5)
        lo, hi = (-1.2, -1.2, -1.2), (1.2, 1.2, 1.2)
        t0 = time.time()
        grid = M.build_sdf_grid(None, 128, lo, hi, tris=tris)
        t_grid = time.time() - t0
        mr = M.Renderer(None, W.camera_mesh(width, width), W.light_c4(), grid=grid, grid_lo=lo, grid_hi=hi, tris=tris)
        mesh = {"workload": f"closed mesh, {tris.shape[0]} triangles, {width}x{width}, {spp} spp, g=0.8, albedo=0.995",
                "grid_seconds": t_grid}
        kw_m = dict(kw, chunk=args.chunk or args.mesh_chunk)
        for s_ in (40.0, 80.0):
            med = W.medium_c4(s_)
            img = mr.render(med, method=1, spp=args.ref_spp // 2, seed=9300, **kw_m)
            rm, rv = image_moments(img, args.ref_spp // 2)
            noise2 = float(rv.mean()) / (args.ref_spp // 2)
            img_pt, t_pt = timed(lambda: mr.render(med, method=1, spp=spp, seed=9400, **kw_m))
            pm, pv = image_moments(img_pt, spp)
            img_st, t_st = timed(lambda: mr.render(med, method=2, sampler=0, packed=packed, spp=spp, seed=9500,
                                                   tau_min=args.tau_min, nee_samples=args.nee_samples,
                                                   flags=args.nee_flags, min_chain=args.min_chain, **kw_m))
            sm, _ = image_moments(img_st, spp)
            e_st = max(float(((sm - rm) ** 2).mean()) - noise2, 1e-30)
            e_pt = max(float(((pm - rm) ** 2).mean()) - noise2, 1e-30)
            c = img_st["counters"].cpu().numpy()
            mesh[str(s_)] = dict(pt_ms=t_pt * 1e3, st_ms=t_st * 1e3, rmse_pt=float(np.sqrt(e_pt)),
                                 rmse_st=float(np.sqrt(e_st)), st_steps_per_path=float(c[2] / c[0]),
                                 speedup_matched_rmse=float(pv.mean()) / e_st / spp * t_pt / t_st)
            log(f"mesh sigma_t={s_}: PT {t_pt * 1e3:.1f} ms, ST {t_st * 1e3:.1f} ms, rmse {np.sqrt(e_pt):.2e} / "
                f"{np.sqrt(e_st):.2e}, speed-up {mesh[str(s_)]['speedup_matched_rmse']:.2f}")

    # absorption sweep (the paper's absorption experiment): one density, the
    # absorption 1 - albedo doubled from 2e-4; rendering time and error of
    # both tracers at the same spp, matched-RMSE speed-up
    absorption = None
    if not args.no_absorption:
        absorption = []
        s_abs = args.absorption_sigma
        for k in range(args.absorption_points):
            a = 2e-4 * 2 ** k
            med = dict(W.medium_c4(s_abs), albedo=1.0 - a)
            img = rend.render(med, method=1, spp=args.ref_spp // 2, seed=7000 + k, **kw)
            r_mean, r_var = image_moments(img, args.ref_spp // 2)
            r_noise2 = float(r_var.mean()) / (args.ref_spp // 2)
            img_pt, t_pt = timed(lambda: rend.render(med, method=1, spp=spp, seed=7100 + k, **kw))
            pm, pv = image_moments(img_pt, spp)
            img_st, t_st = timed(lambda: rend.render(med, method=2, sampler=0, packed=packed, spp=spp, seed=7200 + k,
                                                     tau_min=args.tau_min, nee_samples=args.nee_samples,
                                                     flags=args.nee_flags, min_chain=args.min_chain, **kw))
            sm, _ = image_moments(img_st, spp)
            e_st = float(np.sqrt(max(float(((sm - r_mean) ** 2).mean()) - r_noise2, 1e-30)))
            e_pt = float(np.sqrt(max(float(((pm - r_mean) ** 2).mean()) - r_noise2, 1e-30)))
            s_star = float(pv.mean()) / e_st**2
            row = dict(absorption=a, pt_ms=t_pt * 1e3, st_ms=t_st * 1e3, rmse_pt=e_pt, rmse_st=e_st,
                       speedup_matched_rmse=s_star / spp * t_pt / t_st)
            absorption.append(row)
            log(f"absorption {a:.1e}: PT {t_pt * 1e3:.1f} ms, ST {t_st * 1e3:.1f} ms, rmse {e_pt:.2e} / {e_st:.2e}, "
                f"speed-up {row['speedup_matched_rmse']:.2f}")

    # standalone decoder sampling (cvae_sample) of each trained model, BF16
    # and FP8: conditions resident in HBM, timed launch after a warm-up.
    # VALU work per sample is the kernel's own active-lane count
    # (SQ_THREAD_CYCLES_VALU per row, committed sampling profile); HBM bytes
    # are the conditions read and the samples written
    sample = None
    if not args.no_sample:
        sample = {}
        n_s = args.sample_rows
        for m in range(3):
            sh = M.STANDARD_SHAPES[m]
            cond = torch.randn((n_s, sh["p_in"]), dtype=torch.float32, device="cuda",
                               generator=torch.Generator(device="cuda").manual_seed(m))
            out_s = torch.empty((n_s, sh["p_out"]), dtype=torch.float32, device="cuda")
            for prec, pname in ((1, "bf16"), (2, "fp8")):
                pk = packs[prec][m]
                _, t_s = timed(lambda: M.cvae_sample(pk, cond, n_s, 12, 0, out_s))
                rate = n_s / t_s
                slots = SAMPLE_VALU_SLOTS[(m, prec)]
                nbytes = 4 * (sh["p_in"] + sh["p_out"])
                row = dict(rows=n_s, seconds=t_s, samples_per_s=rate, valu_slots_per_sample=slots,
                           valu_frac=rate * slots / PEAK_VALU_LANEOPS, hbm_bytes_per_sample=nbytes,
                           hbm_frac=rate * nbytes / PEAK_HBM_BYTES)
                sample[f"model{m}_{pname}"] = row
                log(f"cvae_sample model {m} {pname.upper()}: {n_s} rows in {t_s * 1e3:.2f} ms, {rate:.3e} samples/s, "
                    f"VALU {row['valu_frac']:.2f} of peak, HBM {row['hbm_frac']:.2f}")
            del cond, out_s

    # training-data walk at its full size (2^24 photons, parameters drawn per
    # photon as in training), both representative-event weightings; outputs
    # and workspace allocated before the timed launch, counters reset inside
    walk_full = None
    if not args.no_walk_full:
        walk_full = {}
        n_w = args.walk_full_photons
        for name, ew in (("albedo_power", 0), ("uniform", 1)):
            desc = M.walk_desc(n_w, seed=0, mode=1, event_weighting=ew)
            wout = M.alloc_walk_outputs(n_w, 1)
            wws = torch.empty(M.ms_random_walk_workspace_size(desc), dtype=torch.uint8, device="cuda")
            M.ms_random_walk(desc, wout, wws)  # warm-up
            wout["counters"].zero_()
            _, t_w = timed(lambda: M.ms_random_walk(desc, wout, wws), warm=False)
            cw = wout["counters"].cpu().numpy()
            walk_full[name] = dict(photons=n_w, events=int(cw[0]), seconds=t_w, events_per_s=cw[0] / t_w,
                                   max_chain=int(cw[3]),
                                   roofline_frac=cw[0] * OPS_PER_WALK_EVENT / t_w / PEAK_VALU_LANEOPS)
            log(f"walk {n_w} photons ({name}): {t_w * 1e3:.1f} ms, {cw[0]:.3e} events, {cw[0] / t_w:.3e} events/s, "
                f"longest chain {int(cw[3])}")
            del wout, wws

    # density sweep (the paper's density experiments, Sec. 5.4: doubling
    # densities of a nearly non-absorbing medium): smaller image, same
    # matched-RMSE procedure, plus the mean bias of the sphere tracer
    density = None
    if not args.no_density:
        density = []
        # the same recipe with EventGen trained longer: the image bias of the
        # learned steps is EventGen's (placement of the representative
        # events); fitting it longer trades that bias for variance
        pk_ev = None
        if args.density_event_steps > 0:
            pk_ev = train_and_pack(M, torch, args.train_samples, args.train_steps,
                                   model_steps=(args.train_steps, args.train_steps, args.density_event_steps))[0][1]
        dw = args.density_width
        drend = M.Renderer(W.scene_c4(), W.camera_c4(dw, dw), W.light_c4())
        labels = primary_hit_labels(W.camera_c4(dw, dw), W.scene_c4())
        region_names = {1: "sphere", 2: "box_arm"}
        for k, s_ in enumerate(float(x) for x in args.density_sigmas.split(",")):
            med = dict(W.medium_c4(s_), albedo=args.density_albedo)
            img = drend.render(med, method=1, spp=args.ref_spp, seed=9000 + k, **kw)
            r_mean, r_var = image_moments(img, args.ref_spp)
            r_noise2 = float(r_var.mean()) / args.ref_spp
            reps = max(1, args.steps)
            img_pt, t_pt = timed_mean(lambda: drend.render(med, method=1, spp=spp, seed=9100 + k, **kw), reps)
            pm, pv = image_moments(img_pt, spp)

            def st_images(pk, seed0):
                # reps images, one seed each, timed back to back: their mean
                # time, the mean square of their errors and their mean
                ims, t = timed_images([
                    (lambda j=j: drend.render(med, method=2, sampler=0, packed=pk, spp=spp, seed=seed0 + 100000 * j,
                                              tau_min=args.tau_min, nee_samples=args.density_nee_samples,
                                              flags=args.nee_flags, min_chain=args.min_chain, **kw))
                    for j in range(reps)])
                means = [image_moments(im, spp)[0] for im in ims]
                e2 = float(np.mean([float(((m - r_mean) ** 2).mean()) for m in means]))
                return ims[-1], t, float(np.sqrt(max(e2 - r_noise2, 1e-30))), float(np.mean([float(m.mean()) for m in means]))

            img_st, t_st, e_st, sm_mean = st_images(packed, 9200 + k)
            e_pt = float(np.sqrt(max(float(((pm - r_mean) ** 2).mean()) - r_noise2, 1e-30)))
            cp, cs = img_pt["counters"].cpu().numpy(), img_st["counters"].cpu().numpy()
            row = dict(sigma_t=s_, pt_ms=t_pt * 1e3, st_ms=t_st * 1e3, rmse_pt=e_pt, rmse_st=e_st,
                       pt_events_per_path=float(cp[1] / cp[0]), st_events_per_path=float(cs[1] / cs[0]),
                       st_steps_per_path=float(cs[2] / cs[0]),
                       st_mean_bias=sm_mean / float(r_mean.mean()) - 1.0,
                       speedup_matched_rmse=float(pv.mean()) / e_st**2 / spp * t_pt / t_st,
                       regions=dict(pt=region_counts(img_pt, labels, spp, region_names),
                                    st=region_counts(img_st, labels, spp, region_names)))
            if pk_ev is not None:
                _, t_long, e_ev, se_mean = st_images(pk_ev, 9300 + k)
                row.update(event_long=dict(eventgen_steps=args.density_event_steps, st_ms=t_long * 1e3, rmse_st=e_ev,
                                           st_mean_bias=se_mean / float(r_mean.mean()) - 1.0,
                                           speedup_matched_rmse=float(pv.mean()) / e_ev**2 / spp * t_pt / t_long))
            density.append(row)
            log(f"density sigma_t={s_:g} (albedo {args.density_albedo}): PT {t_pt * 1e3:.1f} ms "
                f"({row['pt_events_per_path']:.1f} events/path), ST {t_st * 1e3:.1f} ms "
                f"({row['st_events_per_path']:.1f} events + {row['st_steps_per_path']:.2f} steps), "
                f"rmse {e_pt:.2e} / {e_st:.2e}, bias {row['st_mean_bias']:+.3f}, "
                f"speed-up {row['speedup_matched_rmse']:.2f}")
            for name in region_names.values():
                rp, rs = row["regions"]["pt"].get(name), row["regions"]["st"].get(name)
                if rp and rs:
                    log(f"  {name} ({rp['pixels']} px): PT {rp['events_per_path']:.1f} events/path "
                        f"(p99 {rp['events_p99']:.0f}), ST {rs['events_per_path']:.1f} events "
                        f"(p99 {rs['events_p99']:.0f}) + {rs['steps_per_path']:.2f} steps")

    sweep = None
    if args.table1_sweep:
        log("Table 1 architecture sweep")
        sweep = table1_sweep(M, torch, W, args.train_samples, args.train_steps)

    diag = None
    if args.diagnostics:
        diag = {}
        for s in sigmas:
            img, t = timed(lambda: st_render(s, 5000, sampler=1))
            diag[f"exact_walk_{s}"] = dict(rmse=float(np.sqrt(max(rmse(img, s) ** 2 - ref_noise2[s], 1e-30))),
                                           time_ms=t * 1e3)
            for tau in (0.1, 1.0, 4.0, 8.0):
                img, t = timed(lambda: st_render(s, 5000, tau_min=tau))
                diag[f"tau_{tau}_{s}"] = dict(rmse=float(np.sqrt(max(rmse(img, s) ** 2 - ref_noise2[s], 1e-30))),
                                              time_ms=t * 1e3)
            log(f"diag sigma_t={s}: " + ", ".join(f"{k}: {v['rmse']:.3e} / {v['time_ms']:.1f} ms"
                                                  for k, v in diag.items() if k.endswith(f"_{s}")))

    # roofline of the render kernel from the algorithmic VALU work of the timed
    # step (the method's operation count per path, collision and learned
    # step), and beside it the kernel's own counted lane slots
    alg_step = ALG_PER_STEP_ONE_EVENT + (args.nee_samples - 1) * ALG_PER_EXTRA_EVENT
    alg = counters[0] * ALG_PER_PATH + counters[1] * ALG_PER_EVENT + counters[2] * alg_step
    achieved = alg / (ms_per_step / 1e3)
    ops = counters[0] * OPS_PER_PATH + counters[1] * OPS_PER_EVENT + counters[2] * OPS_PER_STEP
    counted = ops / (ms_per_step / 1e3)
    traffic = measured_traffic()
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_LANEOPS / 1e12,
                "unit": "T lane-op/s", "frac": achieved / PEAK_VALU_LANEOPS, "traffic": traffic,
                "work_per_unit": {"path": ALG_PER_PATH, "collision": ALG_PER_EVENT, "learned_step": alg_step},
                "units": {"paths": int(counters[0]), "collisions": int(counters[1]), "learned_steps": int(counters[2])},
                "counted_achieved": counted / 1e12, "counted_frac": counted / PEAK_VALU_LANEOPS,
                "mfma_tflops": counters[2] * MFMA_FLOP_PER_STEP / (ms_per_step / 1e3) / 1e12,
                "mfma_frac": counters[2] * MFMA_FLOP_PER_STEP / (ms_per_step / 1e3) / PEAK_MFMA_BF16}

    c5 = None
    if not args.no_c5:
        log("C5: 64-sphere grid scene, FP8 / BF16 / plain")
        c5 = c5_section(M, W, torch, packs, args, timed)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the CPU oracle")
        cpu = cpu_baseline(oracle, W, args, tim["models"])

    result = {
        "metric": "sphere-traced paths/s (CVAE) vs plain random-walk paths/s at matched RMSE",
        "value": value, "unit": "paths/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": f"sphere+box SDF scene {width}x{width}, {spp} spp, g=0.8, albedo=0.995, "
                               f"sigma_t in {list(sigmas)}, point light + NEE, CVAE decoders BF16 on MFMA, "
                               f"tau_min={args.tau_min}, {args.nee_samples} representative event(s) per step"
                               + (", direct light before absorption" if args.nee_flags & 1 else "")
                               + (", the paper's step as printed" if args.nee_flags & 2 else "")
                               + (f", learned steps only where the deepest step bypasses >= {args.min_chain:g} "
                                  "collisions" if args.min_chain > 0 else ""),
                   "paths_per_step": paths_per_step, "parallelism": "single GPU"},
        "plain_paths_per_s": pt_rate,
        "object_hit_fraction": hit_fraction,
        "object_hitting_paths_per_s": value * hit_fraction,
        "plain_object_hitting_paths_per_s": pt_rate * hit_fraction,
        "speedup_matched_rmse": tot_pt / tot_st,
        "speedup_matched_rmse_oracle": (tot_pt_o / tot_st_o) if not args.no_oracle_anchor else None,
        "per_sigma": details,
        "train": {"seconds": t_train, "loss_first_last": losses, "steps_per_model": args.train_steps,
                  "step_us_three_models_concurrent": tim.get("train_step_us_three_models"),
                  "samples_per_s_per_model": tim.get("train_samples_per_s_per_model")},
        "walk": dict(tim["walk"], events_per_s=tim["walk"]["events"] / tim["walk"]["seconds"],
                     roofline_frac=tim["walk"]["events"] * OPS_PER_WALK_EVENT / tim["walk"]["seconds"] / PEAK_VALU_LANEOPS,
                     workload="training walks (sigma_t r log-uniform [0.1, 200], g U[-0.9, 0.95], albedo U[0.9, 1])"),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "c5": c5,
        "table1": table1,
        "other_step_form": other,
        "table1_sweep": sweep,
        "cvae_sample": sample,
        "walk_full": None if walk_full is None else dict(
            walk_full, workload=f"training walks, {args.walk_full_photons} photons, sigma_t r log-uniform [0.1, 200], "
                                "g U[-0.9, 0.95], albedo U[0.9, 1]"),
        "density_sweep": None if density is None else {
            "workload": f"sphere+box scene {args.density_width}x{args.density_width}, {spp} spp, g=0.8, "
                        f"albedo={args.density_albedo}, doubling sigma_t, {args.density_nee_samples} representative "
                        f"events per learned step", "rows": density},
        "absorption_sweep": absorption,
        "rgb": rgb,
        "mesh": mesh,
        "focus_training": focus,
        "diagnostics": diag,
        "wall_s_timed": wall,
    }
    line = json.dumps(result)
    print(line, flush=True)
    if args.jsonl:
        with open(args.jsonl, "a") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
