"""Quality of the GPU-trained CVAEs against the random walk they learn
(Sec. 5.3 evaluation grid: sigma_t in {1, 4, 20, 100}, g in {-0.7, 0, 0.4,
0.9}, albedo 1, 10 000 samples each), and what the trained networks gain in a
render over untrained ones.  The paper reports these distributions only as
plots, so there is no published figure to match ("parity unpinned"); the
bounds asserted here sit above the distances measured for this training
recipe (2^22 walks, 20 000 AdamW steps) and below what an untrained or
broken model gives, so a regression in training or sampling fails them."""
import numpy as np
import pytest
import torch
from scipy import stats

import workloads as W
from conftest import announce

pytestmark = pytest.mark.gpu

SIGMAS = (1.0, 4.0, 20.0, 100.0)
GS = (-0.7, 0.0, 0.4, 0.9)
N_EVAL = 10000


@pytest.fixture(scope="module")
def trained(msst):
    """Models of both forms of the learned step: with the single-event cases
    left to exact sampling (PathGen on N >= 2, EventGen on k >= 2; the
    benchmark's default) and trained on every walk record (the paper's step
    as printed)."""
    import bench
    out = {}
    for all_rows in (True, False):
        packs, losses, _ = bench.train_and_pack(msst, torch, 1 << 22, 20000, all_rows=all_rows)
        out[all_rows] = (packs[1], losses)
    return out


def sample(msst, packed, model, cond, seed):
    n, p_out = cond.shape[0], [1, 3, 6][model]
    out = torch.empty((n, p_out), dtype=torch.float32, device="cuda")
    msst.cvae_sample(packed[model], torch.as_tensor(cond, dtype=torch.float32).cuda(), n, seed, 0, out)
    return out.cpu().numpy().astype(np.float64)


def pipeline(msst, packed, st, g, n, seed, paper):
    """LengthGen -> PathGen -> EventGen chained as a learned step takes them;
    with paper=False the single-event parts are sampled exactly (N = 1: one
    HG scatter, alpha = beta = 0; the representative event is the centre
    with probability 1/N at albedo 1)."""
    lst = np.full(n, np.log(st))
    gg = np.full(n, g)
    y = sample(msst, packed, 0, np.stack([lst, gg], 1), seed)[:, 0]
    N = np.maximum(1.0, np.floor(np.exp(np.minimum(y, 20.0)) + 0.5))
    p = sample(msst, packed, 1, np.stack([lst, gg, np.log(N)], 1), seed + 1)
    ct = np.clip(p[:, 0], -1, 1)
    al, be = p[:, 1], p[:, 2]
    ga = np.sqrt(np.maximum(0, 1 - al**2 - be**2))
    nl = np.sqrt(al**2 + be**2 + ga**2)
    al, be = al / nl, be / nl
    rng = np.random.default_rng(seed)
    one = N < 2
    if not paper:
        xi = rng.uniform(size=n)
        hg = (1 + g * g - ((1 - g * g) / (1 - g + 2 * g * xi)) ** 2) / (2 * g) if g != 0 else 2 * xi - 1
        ct = np.where(one, hg, ct)
        al = np.where(one, 0.0, al)
        be = np.where(one, 0.0, be)
    e = sample(msst, packed, 2, np.stack([lst, gg, np.ones(n), ct, al, be, np.log(N)], 1), seed + 2)
    X = e[:, :3]
    xl = np.linalg.norm(X, axis=1)
    X = np.where(xl[:, None] > 1, X / xl[:, None], X)
    if not paper:
        first = one | (rng.uniform(size=n) <= 1.0 / N)
        X = np.where(first[:, None], 0.0, X)
    return N, ct, al, be, X


# Asserted bounds on the medians over the 16 settings of the two-sample KS
# distance (learned against walk).  Measured with this recipe (medians of
# log N, cos theta, alpha, beta, |X|): exact single-event parts 0.141, 0.111,
# 0.042, 0.069, 0.208; every record learned 0.141, 0.118, 0.071, 0.090, 0.493
# (EventGen must then reproduce the point mass of |X| at 0 that the first
# event, at the sphere's centre, puts there).
BOUNDS = {
    False: {"log N": 0.2, "cos theta": 0.15, "alpha | N > 1": 0.08, "beta | N > 1": 0.1, "|X|": 0.3},
    True: {"log N": 0.2, "cos theta": 0.15, "alpha | N > 1": 0.1, "beta | N > 1": 0.12, "|X|": 0.6},
}


@pytest.mark.parametrize("paper", [True, False])
def test_learned_distributions_against_the_walk(msst, trained, paper):
    announce(f"quality grid paper={paper}")
    packed, losses = trained[paper]
    print("training loss first -> last:", losses)
    rows = []
    for st in SIGMAS:
        for g in GS:
            w = msst.random_walk(N_EVAL, seed=int(st * 10 + (g + 1) * 100), mode=1, st_range=(st, st),
                                 g_range=(g, g), albedo_range=(1.0, 1.0))
            n_gt = w["n_scatter"].cpu().numpy().astype(np.float64)
            ep = w["exit_param"].cpu().numpy().astype(np.float64)
            X_gt = w["event_pos"].cpu().numpy().T.astype(np.float64)
            N, ct, al, be, X = pipeline(msst, packed, st, g, N_EVAL, seed=int(st * 7 + g * 13 + 50), paper=paper)
            d_n = stats.ks_2samp(np.log(n_gt), np.log(N)).statistic
            d_ct = stats.ks_2samp(ep[0], ct).statistic
            m_gt, m = n_gt > 1, N > 1
            ok = m_gt.sum() > 50 and m.sum() > 50
            d_al = stats.ks_2samp(ep[1][m_gt], al[m]).statistic if ok else np.nan
            d_be = stats.ks_2samp(ep[2][m_gt], be[m]).statistic if ok else np.nan
            d_x = stats.ks_2samp(np.linalg.norm(X_gt, axis=1), np.linalg.norm(X, axis=1)).statistic
            rows.append((st, g, d_n, n_gt.mean(), N.mean(), d_ct, d_al, d_be, d_x))
    print("sigma_t     g   KS(logN)  E[N]gt   E[N]cvae  KS(cos)  KS(alpha|N>1)  KS(beta|N>1)  KS(|X|)")
    for r in rows:
        print(f"{r[0]:7.1f} {r[1]:5.1f}   {r[2]:.3f}  {r[3]:9.2f} {r[4]:9.2f}   {r[5]:.3f}    {r[6]:.3f}"
              f"          {r[7]:.3f}         {r[8]:.3f}")
    arr = np.array(rows)
    med = {"log N": np.median(arr[:, 2]), "cos theta": np.median(arr[:, 5]),
           "alpha | N > 1": np.nanmedian(arr[:, 6]), "beta | N > 1": np.nanmedian(arr[:, 7]),
           "|X|": np.median(arr[:, 8])}
    print("median KS: " + ", ".join(f"{k} {v:.3f}" for k, v in med.items()))
    for k, v in med.items():
        assert v < BOUNDS[paper][k], (k, v)
    assert np.all(np.abs(np.log(arr[:, 4] / arr[:, 3])) < np.log(2.0))


def test_trained_networks_beat_untrained_in_a_render(msst, oracle, trained):
    """What the learning gains: image error of sphere tracing with the trained
    decoders against the same decoders untrained, both against a plain
    path-traced reference."""
    announce("trained vs untrained render error")
    packed, _ = trained[False]
    cam = W.camera_c4(128, 128)
    rend = msst.Renderer(W.scene_c4(), cam, W.light_c4())
    med = W.medium_c4(40.0)
    ref = rend.render(med, method=1, spp=4096, seed=1)
    refm = (ref["sum"].double() + ref["comp"].double()) / 4096
    untrained = []
    for m in range(3):
        master = torch.empty(msst.cvae_param_count(m), dtype=torch.float32, device="cuda")
        msst.cvae_init(m, 123 + m, master)
        p = torch.empty(msst.cvae_packed_bytes(), dtype=torch.uint8, device="cuda")
        msst.cvae_pack(m, master, torch.as_tensor(W.render_test_stats(m), dtype=torch.float64).cuda(), 1, p)
        untrained.append(p)

    def err(pk):
        img = rend.render(med, method=2, sampler=0, packed=pk, spp=256, seed=2, tau_min=2.0)
        mean = (img["sum"].double() + img["comp"].double()) / 256
        return float(torch.sqrt(((mean - refm) ** 2).mean())), float(mean.mean())

    e_tr, m_tr = err(packed)
    e_un, m_un = err(untrained)
    print(f"RMSE trained {e_tr:.4e} (mean {m_tr:.4e}), untrained {e_un:.4e} (mean {m_un:.4e}), "
          f"reference mean {float(refm.mean()):.4e}")
    assert e_tr < 0.5 * e_un
