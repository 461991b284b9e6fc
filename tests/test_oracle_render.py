"""Pins of the oracle geometry and renderers (Sec. 3, Sec. 4.3): brute-force
geometry, a single-scattering closed form by quadrature, and the regrouping
identity between the plain path tracer and sphere tracing with exact walks."""
import numpy as np
import pytest
from scipy import integrate

import workloads as W


@pytest.fixture(scope="module")
def c4(oracle):
    return oracle.Scene(W.scene_c4())


def inside_union(prims, p):
    for pr in prims:
        q = p - pr[1:4]
        if pr[0] == W.PRIM_SPHERE and q @ q < pr[4] ** 2:
            return True
        if pr[0] == W.PRIM_BOX and np.all(np.abs(q) < pr[4:7]):
            return True
    return False


def test_intervals_brute_force(oracle, c4):
    prims = W.scene_c4()
    rng = np.random.default_rng(1)
    for _ in range(60):
        o = rng.uniform(-3, 3, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        iv = c4.intervals(o, d)
        ts = np.linspace(-8, 8, 4001)
        ins = np.array([inside_union(prims, o + t * d) for t in ts])
        pred = np.zeros_like(ins)
        for a, b in iv:
            pred |= (ts > a) & (ts < b)
        # disagreement only within a grid step of an interval end
        bad = ts[ins != pred]
        ends = np.array([e for ab in iv for e in ab]) if iv else np.array([1e9])
        assert all(np.min(np.abs(ends - t)) < 0.005 for t in bad)
        for k in range(len(iv) - 1):
            assert iv[k][1] < iv[k + 1][0]  # sorted and disjoint


def test_sdf_values(oracle, c4):
    assert abs(c4.sdf([0, 0, 0]) + 1.0) < 1e-12
    assert abs(c4.sdf([0, 0, 2.0]) - 1.0) < 1e-12
    assert abs(c4.sdf([2.5, 0, 0]) - 0.5) < 1e-7        # box face at x = 2.0
    assert abs(c4.sdf([2.5, 0.9, 0]) - np.hypot(0.5, 0.5)) < 1e-7  # box edge
    assert abs(c4.sdf([1.8, 0.0, 0.0]) + 0.2) < 1e-7    # inside the arm


def test_conservative_radius_inside(oracle, c4):
    prims = W.scene_c4()
    rng = np.random.default_rng(2)
    dirs = rng.normal(size=(400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    n_in = 0
    for _ in range(300):
        p = rng.uniform([-1, -1, -1], [2, 1, 1])
        r = c4.conservative_radius(p)
        if not inside_union(prims, p):
            assert r == 0.0
            continue
        n_in += 1
        assert r > 0
        for dv in dirs:
            assert inside_union(prims, p + r * dv)
    assert n_in > 50


def test_sdf_grid_round_toward_zero_and_conservative(oracle):
    prims = W.scene_c5(seed=0)
    sc = oracle.Scene(prims)
    res = 32
    grid = sc.build_grid(res)
    vals = grid.view(np.float16).astype(np.float64)
    h = 2.0 / res
    rng = np.random.default_rng(3)
    for idx in rng.integers(0, res**3, 400):
        k, j, i = idx // (res * res), (idx // res) % res, idx % res
        p = -1 + (np.array([i, j, k]) + 0.5) * h
        exact = sc.sdf(p)
        assert abs(vals[idx]) <= abs(exact) + 1e-15
        assert abs(vals[idx] - exact) <= abs(exact) * 2**-10 + 2**-24
    gs = oracle.Scene(prims, sdf_fp16=grid)
    for _ in range(2000):
        p = rng.uniform(-1, 1, 3)
        r = gs.conservative_radius(p)
        assert r <= max(0.0, -sc.sdf(p)) + 1e-12


def single_scatter_expectation(sigma_t, g, phi, light, eye, d):
    """phi * int sigma_t e^{-sigma_t (t - a)} I rho_g(d . w_L) e^{-sigma_t d_t} / |x_L - x|^2 dt
    for a ray (eye, d) through the unit sphere: the first-event term of the
    direct-lighting sum (Eq. directLighting) in closed form along the ray."""
    xL, I = np.array(light["pos"]), light["intensity"]
    b = eye @ d
    c = eye @ eye - 1.0
    a, e = -b - np.sqrt(b * b - c), -b + np.sqrt(b * b - c)

    def f(t):
        x = eye + t * d
        wl = xL - x
        dist = np.linalg.norm(wl)
        wl = wl / dist
        bb = x @ wl
        dt = -bb + np.sqrt(bb * bb - (x @ x - 1.0))
        cos = d @ wl
        rho = (1 - g * g) / (1 + g * g - 2 * g * cos) ** 1.5 / (4 * np.pi)
        return sigma_t * np.exp(-sigma_t * (t - a)) * I * rho * np.exp(-sigma_t * dt) / dist**2

    return phi * integrate.quad(f, a, e, epsabs=1e-14, limit=400)[0]


@pytest.mark.parametrize("sigma_t,g", [(2.0, 0.8), (5.0, -0.3)])
def test_single_scattering_closed_form(oracle, sigma_t, g):
    scene = oracle.Scene(W.scene_sphere(1.0))
    res = 40000  # tiny pixels: the jitter moves the ray by < 1e-5 rad
    cam = dict(eye=(0.0, 0.3, 4.0), look_at=(0.0, 0.0, 0.0), up=(0, 1, 0), vfov_deg=30.0,
               width=res, height=res)
    light = dict(pos=(1.5, 3.0, 3.0), intensity=10.0)
    phi = 1e-4
    pix = (res // 2 + 2000) * res + res // 2 - 3000
    spp = 40000
    out = oracle.render(scene, cam, light, dict(sigma_t=sigma_t, g=g, albedo=phi), spp=spp,
                        pixels=[pix], seed=5)
    mean = out["sum"][0] / spp
    var = out["sumsq"][0] / spp - mean**2
    # the centre ray of that pixel
    px, py = pix % res, pix // res
    f = np.array(cam["look_at"]) - np.array(cam["eye"])
    f /= np.linalg.norm(f)
    rt = np.cross(f, cam["up"])
    rt /= np.linalg.norm(rt)
    uv = np.cross(rt, f)
    th = np.tan(np.radians(cam["vfov_deg"]) / 2)
    sx = (2 * (px + 0.5) / res - 1) * th
    sy = (1 - 2 * (py + 0.5) / res) * th
    d = f + sx * rt + sy * uv
    d /= np.linalg.norm(d)
    exp = single_scatter_expectation(sigma_t, g, phi, light, np.array(cam["eye"], float), d)
    assert exp > 0
    assert abs(mean - exp) < 5 * np.sqrt(var / spp) + 1e-3 * exp, (mean, exp)


def small_c4(sigma_t, w=24):
    return W.camera_c4(w, w), W.light_c4(), W.medium_c4(sigma_t)


@pytest.mark.parametrize("exact", [False, True])
def test_event_cap_only_touches_longer_paths(oracle, c4, exact):
    """max_events ends a path at the collision after the cap (a sphere step
    counting once): paths with at most cap collisions are unchanged, bit for
    bit, and no path records more than cap."""
    cam, light, med = small_c4(40.0)
    kw = (dict(method=oracle.METHOD_ST, sampler=oracle.SAMPLER_EXACT_WALK) if exact
          else dict(method=oracle.METHOD_PLAIN_NEE))
    full = oracle.render(c4, cam, light, med, spp=1, seed=6, **kw)
    n_full = full["events"].astype(np.int64) + full["steps"]
    assert n_full.max() > 6
    for cap in (1, 3, 6):
        a = oracle.render(c4, cam, light, med, spp=1, seed=6, max_events=cap, **kw)
        n = a["events"].astype(np.int64) + a["steps"]
        short = n_full <= cap
        np.testing.assert_array_equal(a["sum"][short], full["sum"][short])
        np.testing.assert_array_equal(n[short], n_full[short])
        assert (n[~short] == cap).all()
        # a truncated path keeps the light it gathered before the cap: a
        # prefix of the same stream's nonnegative terms
        assert (a["sum"][~short] <= full["sum"][~short] * (1 + 1e-12)).all()
        assert (a["sum"][~short] < full["sum"][~short]).any()
    if exact:
        assert full["steps"].sum() > 0


def test_sphere_tracing_without_steps_is_plain(oracle, c4):
    cam, light, med = small_c4(10.0)
    a = oracle.render(c4, cam, light, med, method=oracle.METHOD_PLAIN_NEE, spp=4, seed=1)
    b = oracle.render(c4, cam, light, med, method=oracle.METHOD_ST, sampler=oracle.SAMPLER_EXACT_WALK,
                      tau_min=1e30, spp=4, seed=1)
    np.testing.assert_array_equal(a["sum"], b["sum"])
    assert b["steps"].sum() == 0


@pytest.mark.parametrize("sigma_t", [10.0, 40.0])
def test_exact_walk_sphere_steps_match_plain_path_tracing(oracle, c4, sigma_t):
    """Sphere tracing with the exact in-sphere walk regroups the plain walk, so
    the two estimators share their expectation (Sec. 3, Sec. 4.3)."""
    cam, light, med = small_c4(sigma_t, 16)
    spp = 256
    a = oracle.render(c4, cam, light, med, method=oracle.METHOD_PLAIN_NEE, spp=spp, seed=2)
    b = oracle.render(c4, cam, light, med, method=oracle.METHOD_ST, sampler=oracle.SAMPLER_EXACT_WALK,
                      spp=spp, seed=3)
    n = spp * cam["width"] * cam["height"]

    def mean_se(o):
        m = o["sum"].sum() / n
        v = o["sumsq"].sum() / n - m * m
        return m, np.sqrt(v / n)

    ma, sa = mean_se(a)
    mb, sb = mean_se(b)
    assert abs(ma - mb) < 5 * np.hypot(sa, sb), (ma, mb, sa, sb)
    assert b["steps"].sum() > 0
    # per-pixel agreement in aggregate
    va = a["sumsq"] / spp - (a["sum"] / spp) ** 2
    vb = b["sumsq"] / spp - (b["sum"] / spp) ** 2
    z = (a["sum"] - b["sum"]) / spp / np.sqrt((va + vb) / spp + 1e-30)
    lit = (va + vb) > 0
    assert abs(z[lit].mean()) < 5 / np.sqrt(lit.sum())
    assert 0.7 < z[lit].std() < 1.3


def test_learned_step_estimators_share_their_expectation(oracle, c4):
    """Averaging K representative events (also K set per step by the chain
    length N), or adding the direct light of every learned step before its
    absorption test with weight sum_i albedo^i instead of survivors only with
    that sum over albedo^N, leaves the expectation of the sphere-traced
    estimator unchanged (Sec. 3.2, Sec. 4.3); the models are untrained but
    fixed, so all the variants estimate the same quantity."""
    cam, light, _ = small_c4(40.0, 12)
    med = dict(sigma_t=40.0, g=0.8, albedo=0.95)
    models = [dict(shape=W.SHAPE_LIST[m], params=oracle.cvae_init(W.SHAPE_LIST[m], seed=70 + m),
                   stats=W.render_test_stats(m)) for m in range(3)]
    spp = 192
    n = spp * cam["width"] * cam["height"]
    res = []
    for i, (k, flags, chain) in enumerate([(1, 0, 0), (3, 0, 0), (1, oracle.NEE_BEFORE_ABSORPTION, 0),
                                            (2, oracle.NEE_BEFORE_ABSORPTION, 0),
                                            (4, oracle.NEE_BEFORE_ABSORPTION, 3), (3, 0, 2)]):
        o = oracle.render(c4, cam, light, med, method=oracle.METHOD_ST, sampler=oracle.SAMPLER_CVAE,
                          models=models, tau_min=1.0, spp=spp, seed=40 + i, nee_samples=k, flags=flags,
                          nee_chain=chain)
        m = o["sum"].sum() / n
        res.append((m, np.sqrt((o["sumsq"].sum() / n - m * m) / n), o["steps"].sum()))
    m0, s0, st0 = res[0]
    assert st0 > 1000
    for m, s, _ in res[1:]:
        assert abs(m - m0) < 5 * np.hypot(s, s0), res
    # the default order with one sample is unchanged by the new fields
    a = oracle.render(c4, cam, light, med, method=oracle.METHOD_ST, sampler=oracle.SAMPLER_CVAE, models=models,
                      tau_min=1.0, spp=2, seed=40)
    b = oracle.render(c4, cam, light, med, method=oracle.METHOD_ST, sampler=oracle.SAMPLER_CVAE, models=models,
                      tau_min=1.0, spp=2, seed=40, nee_samples=0)
    np.testing.assert_array_equal(a["sum"], b["sum"])


def test_events_per_step_follow_the_chain_length(oracle):
    """nee_chain: a step of N events takes min(nee_samples, 1 + (N - 1) //
    nee_chain) representative events.  The rule follows N alone, so a step
    whose chain asks for one event is the one-event step bit for bit (the same
    draws), and one whose chain asks for all nee_samples events is the
    uniform step with that many."""
    models = [dict(shape=W.SHAPE_LIST[m], params=oracle.cvae_init(W.SHAPE_LIST[m], seed=80 + m),
                   stats=W.render_test_stats(m)) for m in range(3)]
    med = dict(sigma_t=40.0, g=0.8, albedo=0.99)
    p, d, r = np.array([0.1, 0.0, 0.2]), np.array([0.0, 0.6, 0.8]), 0.5
    kw = dict(models=models, flags=oracle.NEE_BEFORE_ABSORPTION)
    seen = set()
    for path_id in range(300):
        a = oracle.sphere_step(med, p, d, r, path_id, nee_samples=4, nee_chain=6, **kw)
        n = int(a["N"])
        k = min(4, 1 + (n - 1) // 6)
        assert a["n_rep"] == k
        seen.add(k)
        same = oracle.sphere_step(med, p, d, r, path_id, nee_samples=k, **kw)
        for key in ("x", "w", "nee_w", "N", "psi", "c0"):
            np.testing.assert_array_equal(a[key], same[key])
        np.testing.assert_array_equal(a["X"][:k], same["X"][:k])
        np.testing.assert_array_equal(a["first"][:k], same["first"][:k])
    assert seen >= {1, 2}, seen
