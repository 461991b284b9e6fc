"""Pins of the oracle random walk (Sec. 3.1) against closed forms, quadrature,
invariants and symbolic identities.  CPU only."""
import numpy as np
import pytest
from scipy import integrate, stats

G_VALUES = [-0.7, 0.0, 0.4, 0.9]


def hg_pdf_mu(g, mu):
    """Density of the cosine under HG: 2 pi rho_g, written from Eq. 1."""
    return 0.5 * (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5


@pytest.mark.parametrize("g", G_VALUES + [0.95, -0.9])
def test_hg_eval_normalised_with_mean_cosine_g(oracle, g):
    tot = integrate.quad(lambda m: 2 * np.pi * oracle.hg_eval(g, m), -1, 1, epsabs=1e-12, limit=200)[0]
    mean = integrate.quad(lambda m: 2 * np.pi * m * oracle.hg_eval(g, m), -1, 1, epsabs=1e-12, limit=200)[0]
    assert abs(tot - 1) < 1e-9
    assert abs(mean - g) < 1e-9


@pytest.mark.parametrize("g", G_VALUES + [0.95, -0.9])
def test_hg_sample_inverts_cdf_by_quadrature(oracle, g):
    for xi in [1e-6, 0.01, 0.2, 0.5, 0.77, 0.999, 1.0]:
        mu = oracle.hg_sample(g, xi)
        F = integrate.quad(lambda m: hg_pdf_mu(g, m), -1, mu, epsabs=1e-13, limit=200)[0]
        assert abs(F - xi) < 1e-9, (g, xi, mu, F)


@pytest.mark.parametrize("g", G_VALUES)
def test_hg_sample_moments(oracle, g):
    n = 200000
    xi = (np.arange(n) + 0.5) / n  # midpoint rule of the quantile integral
    mu = np.array([oracle.hg_sample(g, x) for x in xi])
    assert abs(mu.mean() - g) < 1e-4
    assert abs((mu**2).mean() - (1 + 2 * g * g) / 3) < 1e-4


def test_hg_stable_form_identity():
    """The cancellation-free HG inversion used by the GPU equals the textbook one."""
    import sympy as sp
    g, xi = sp.symbols("g xi", real=True)
    a = 2 * xi - 1
    s = (1 - g**2) / (1 - g + 2 * g * xi)
    textbook = (1 + g**2 - s**2) / (2 * g)
    stable = (a + g) / (1 + g * a) + g * (1 - a**2) * (1 - g**2) / (2 * (1 + g * a) ** 2)
    assert sp.simplify(textbook - stable) == 0
    assert sp.simplify(stable.subs(g, 0) - a) == 0  # isotropic limit without a branch
    assert sp.simplify(stable.subs(xi, 0) + 1) == 0 and sp.simplify(stable.subs(xi, 1) - 1) == 0
    # the GPU evaluates mu and sin(theta) through 1 - mu and 1 + mu in these forms
    q = 1 + g * a
    one_minus = 2 * (1 - g) ** 2 * (1 - xi) * (1 + g * xi) / q**2
    one_plus = 2 * (1 + g) ** 2 * xi * (1 - g + g * xi) / q**2
    assert sp.simplify(1 - textbook - one_minus) == 0
    assert sp.simplify(1 + textbook - one_plus) == 0


def test_onb_orthonormal_right_handed(oracle):
    rng = np.random.default_rng(5)
    ns = list(rng.normal(size=(500, 3)))
    ns += [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]), np.array([1.0, 0, 0]),
           np.array([0, 1.0, 1e-17]), np.array([1e-9, 0, -1.0])]
    for n in ns:
        n = n / np.linalg.norm(n)
        b1, b2 = oracle.onb(n)
        M = np.stack([b1, b2, n])
        np.testing.assert_allclose(M @ M.T, np.eye(3), atol=1e-12)
        np.testing.assert_allclose(np.cross(b1, b2), n, atol=1e-12)


def test_scatter_dir_cosine_and_azimuth(oracle):
    rng = np.random.default_rng(6)
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        mu, az = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
        nd = oracle.scatter_dir(d, mu, az)
        b1, b2 = oracle.onb(d)
        assert abs(np.linalg.norm(nd) - 1) < 1e-12
        assert abs(nd @ d - mu) < 1e-12
        assert abs(np.arctan2(nd @ b2, nd @ b1) % (2 * np.pi) - az) < 1e-9


@pytest.mark.parametrize("st", [0.05, 0.5, 1.5, 3.0])
def test_escape_probability(oracle, st):
    """P(N = 1) = exp(-sigma_t r): no second interaction before the boundary."""
    n = 200000
    w = oracle.random_walk(n, seed=11, sigma_t=st, g=0.3, albedo=1.0, radius=1.0)
    p = np.exp(-st)
    phat = (w["n_scatter"] == 1).mean()
    assert abs(phat - p) < 5 * np.sqrt(p * (1 - p) / n) + 1e-12


@pytest.mark.parametrize("st,g", [(0.5, 0.8), (1.5, -0.5), (2.0, 0.0)])
def test_two_event_probability_quadrature(oracle, st, g):
    """P(N = 2) = int_0^r st e^{-st s} int p_HG(mu) e^{-st t(s, mu)} dmu ds."""
    r = 1.0

    def inner(s):
        f = lambda mu: hg_pdf_mu(g, mu) * np.exp(-st * (-s * mu + np.sqrt(r * r - s * s * (1 - mu * mu))))
        return integrate.quad(f, -1, 1, epsabs=1e-12, limit=200)[0]

    p2 = integrate.quad(lambda s: st * np.exp(-st * s) * inner(s), 0, r, epsabs=1e-12, limit=200)[0]
    n = 400000
    w = oracle.random_walk(n, seed=12, sigma_t=st, g=g, albedo=1.0, radius=r)
    phat = (w["n_scatter"] == 2).mean()
    assert abs(phat - p2) < 5 * np.sqrt(p2 * (1 - p2) / n), (phat, p2)


@pytest.mark.parametrize("g", [-0.7, 0.4, 0.9])
def test_single_event_exit_is_hg(oracle, g):
    w = oracle.random_walk(200000, seed=13, sigma_t=1.0, g=g, albedo=1.0)
    one = w["n_scatter"] == 1
    ct = w["exit_param"][0, one]
    cdf = lambda m: np.array([integrate.quad(lambda x: hg_pdf_mu(g, x), -1, v)[0] for v in np.atleast_1d(m)])
    grid = np.linspace(-1, 1, 2001)
    Fg = cdf(grid)
    assert stats.kstest(ct, lambda m: np.interp(m, grid, Fg)).pvalue > 1e-4
    xh = w["exit_pos"][:, one]
    np.testing.assert_allclose(w["exit_dir"][:, one], xh, atol=1e-9)
    np.testing.assert_allclose(w["exit_param"][1:, one], 0, atol=1e-9)


def test_no_absorption_at_unit_albedo(oracle):
    w = oracle.random_walk(50000, seed=14, sigma_t=10.0, g=0.8, albedo=1.0, radius=2.0)
    assert w["absorbed"].sum() == 0 and w["truncated"].sum() == 0
    r = np.linalg.norm(w["exit_pos"], axis=0)
    np.testing.assert_allclose(r, 2.0, rtol=1e-12)
    assert np.all(np.sum(w["exit_pos"] * w["exit_dir"], axis=0) > 0)


def test_absorbing_walk_is_prefix_of_free_walk(oracle):
    n = 50000
    free = oracle.random_walk(n, seed=15, sigma_t=5.0, g=0.5, albedo=1.0)
    ab = oracle.random_walk(n, seed=15, sigma_t=5.0, g=0.5, albedo=0.9)
    A = ab["absorbed"].astype(bool)
    assert np.all(ab["n_scatter"][A] <= free["n_scatter"][A])
    np.testing.assert_array_equal(ab["n_scatter"][~A], free["n_scatter"][~A])
    np.testing.assert_allclose(ab["exit_pos"][:, ~A], free["exit_pos"][:, ~A], atol=0)
    # P(A = 1) = 1 - E[albedo^N_free]
    p = 1 - np.mean(0.9 ** free["n_scatter"].astype(float))
    assert abs(A.mean() - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_scale_invariance(oracle):
    a = oracle.random_walk(20000, seed=16, sigma_t=8.0, g=0.6, albedo=0.97, radius=1.0)
    b = oracle.random_walk(20000, seed=16, sigma_t=2.0, g=0.6, albedo=0.97, radius=4.0)
    same = a["n_scatter"] == b["n_scatter"]
    assert same.mean() > 0.9999
    np.testing.assert_allclose(b["exit_pos"][:, same] / 4.0, a["exit_pos"][:, same], atol=1e-9)
    np.testing.assert_allclose(b["exit_param"][:, same], a["exit_param"][:, same], atol=1e-9)


def test_truncation_flag(oracle):
    w = oracle.random_walk(1000, seed=17, sigma_t=50.0, g=0.0, albedo=1.0, max_events=1)
    assert np.all(w["n_scatter"] == 1)
    esc = np.linalg.norm(w["exit_pos"], axis=0) >= 1 - 1e-12
    assert np.all(w["truncated"].astype(bool) == ~esc)


def fixed_training(oracle, n, st, g, phi, weighting, seed=18):
    return oracle.random_walk(n, seed=seed, mode=oracle.WALK_TRAINING, st_range=(st, st),
                              g_range=(g, g), albedo_range=(phi, phi), event_weighting=weighting)


def test_training_matches_analog_trajectory(oracle):
    n = 20000
    a = oracle.random_walk(n, seed=18, sigma_t=6.0, g=0.2, albedo=1.0)
    t = fixed_training(oracle, n, 6.0, 0.2, 1.0, oracle.EVENT_ALBEDO_POWER)
    np.testing.assert_array_equal(a["n_scatter"], t["n_scatter"])
    np.testing.assert_allclose(a["exit_pos"], t["exit_pos"], atol=1e-12)
    np.testing.assert_allclose(a["exit_param"], t["exit_param"], atol=1e-12)


def test_training_single_event_summary(oracle):
    t = fixed_training(oracle, 50000, 1.0, 0.5, 0.95, oracle.EVENT_ALBEDO_POWER)
    one = t["n_scatter"] == 1
    assert one.sum() > 1000
    assert np.all(t["event_index"][one] == 1)
    np.testing.assert_allclose(t["event_pos"][:, one], 0, atol=1e-12)
    ez = np.broadcast_to(np.array([[0], [0], [1.0]]), t["event_dir"][:, one].shape)
    np.testing.assert_allclose(t["event_dir"][:, one], ez, atol=1e-12)
    np.testing.assert_allclose(t["exit_param"][1:, one], 0, atol=1e-9)


@pytest.mark.parametrize("weighting,phi", [(0, 0.8), (1, 0.8), (0, 1.0)])
def test_representative_event_law(oracle, weighting, phi):
    """k | N is albedo^k / Lambda^(N) (albedo-power) or uniform (Sec. 4.3)."""
    t = fixed_training(oracle, 300000, 3.0, 0.0, phi, weighting)
    for N in (3, 5):
        sel = t["n_scatter"] == N
        k = t["event_index"][sel]
        w = np.ones(N) if weighting == 1 else phi ** np.arange(1, N + 1)
        exp = w / w.sum() * sel.sum()
        obs = np.bincount(k, minlength=N + 1)[1:]
        assert stats.chisquare(obs, exp).pvalue > 1e-4, (N, obs, exp)


def test_exit_symmetries(oracle):
    t = fixed_training(oracle, 100000, 4.0, 0.5, 1.0, 0)
    al = t["exit_param"][1]
    assert stats.ks_2samp(al, -al).pvalue > 1e-3
    psi = np.arctan2(t["exit_pos"][1], t["exit_pos"][0])
    assert stats.kstest((psi + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-4
    # canonical frame: exit lies in the xz-plane, so X, W are rotated the same way
    r = np.linalg.norm(t["event_pos"], axis=0)
    assert np.all(r <= 1 + 1e-12)
    np.testing.assert_allclose(np.linalg.norm(t["event_dir"], axis=0), 1, atol=1e-12)


def test_training_parameter_ranges(oracle):
    t = oracle.random_walk(50000, seed=19, mode=oracle.WALK_TRAINING)
    st, g, phi = t["params"]
    u = np.log(st / 0.1) / np.log(2000.0)
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert stats.kstest((g + 0.9) / 1.85, "uniform").pvalue > 1e-4
    assert stats.kstest((phi - 0.9) / 0.1, "uniform").pvalue > 1e-4
    assert st.min() > 0.1 and st.max() <= 200.0


def test_focus_weighted_training_parameters(oracle):
    """(sigma_t r, g)-weighted data: with probability f the parameters come
    from the focus box, so the box holds a fraction f + (1 - f) P_main(box)
    of the photons; f = 0 leaves the draws unchanged; f = 1 is the focus
    ranges' own log-uniform / uniform law."""
    n = 40000
    kw = dict(seed=23, mode=oracle.WALK_TRAINING, focus_st_range=(10.0, 20.0), focus_g_range=(0.7, 0.9),
              max_events=64)
    base = oracle.random_walk(n, **dict(kw, focus_fraction=0.0))
    plain = oracle.random_walk(n, seed=23, mode=oracle.WALK_TRAINING, max_events=64)
    np.testing.assert_array_equal(base["params"], plain["params"])
    f = 0.3
    t = oracle.random_walk(n, **dict(kw, focus_fraction=f))
    st, g, phi = t["params"]
    inside = (st >= 10.0) & (st <= 20.0) & (g >= 0.7) & (g <= 0.9)
    p_main = np.log(2.0) / np.log(2000.0) * 0.2 / 1.85
    p = f + (1 - f) * p_main
    z = (inside.mean() - p) / np.sqrt(p * (1 - p) / n)
    assert abs(z) < 5, (inside.mean(), p)
    np.testing.assert_array_equal(phi, base["params"][2])  # the albedo draw is untouched
    full = oracle.random_walk(n, **dict(kw, focus_fraction=1.0))
    st1, g1, _ = full["params"]
    assert stats.kstest(np.log(st1 / 10.0) / np.log(2.0), "uniform").pvalue > 1e-4
    assert stats.kstest((g1 - 0.7) / 0.2, "uniform").pvalue > 1e-4



def _lambert_entry(rng, x, n_in, oracle):
    """Direction cosine-weighted about the inward normal n_in."""
    b1, b2 = oracle.onb(n_in)
    u1, u2 = rng.random(), rng.random()
    a = 2.0 * np.pi * u2
    return np.sqrt(u1) * n_in + np.sqrt(1.0 - u1) * (np.cos(a) * b1 + np.sin(a) * b2)


def _mean_path(oracle, scene, entry, sigma_t, g, n, seed):
    """Mean path length inside and mean collision count of walks entering
    through `entry(rng) -> (x, d)`; the exits come from the oracle's exact
    ray intervals of the scene (entry points lie on its binary32 surface),
    the scattering from its HG inversion and direction update."""
    rng = np.random.default_rng(seed)
    lengths, colls = np.empty(n), np.empty(n)
    for i in range(n):
        x, d = entry(rng)
        total, k = 0.0, 0
        for _ in range(100000):
            t_exit = None
            for t0, t1 in scene.intervals(x, d):
                if t0 <= 1e-7 < t1:
                    t_exit = t1
            assert t_exit is not None
            fl = -np.log(1.0 - rng.random()) / sigma_t
            if fl >= t_exit:
                total += t_exit
                break
            total += fl
            x = x + fl * d
            k += 1
            d = oracle.scatter_dir(d, oracle.hg_sample(g, rng.random()), 2.0 * np.pi * rng.random())
        lengths[i], colls[i] = total, k
    return lengths, colls


@pytest.mark.parametrize("body,sigma_t,g", [("sphere", 0.5, 0.0), ("sphere", 3.0, 0.8), ("box", 3.0, -0.5),
                                            ("box", 1.0, 0.6)])
def test_mean_path_length_is_four_volume_over_surface(oracle, body, sigma_t, g):
    """Invariance of the mean path length (Blanco and Fournier, Europhys.
    Lett. 61, 2003): light entering a non-absorbing convex body uniformly
    over its surface, cosine-weighted about the inward normal, travels 4V/S
    inside on average whatever sigma_t and g are (4R/3 for a sphere of radius
    R, 4 abc / (ab + bc + ca) for a box of half-extents a, b, c), and makes
    sigma_t times that many collisions.  The exits are the oracle's exact ray
    intervals, so a wrong root or slab there, or a flight rate other than
    sigma_t, moves the mean."""
    if body == "sphere":
        rad, c = float(np.float32(0.7)), np.array([0.1, -0.2, 0.3], np.float32).astype(np.float64)
        scene = oracle.Scene(np.array([[0, *c, rad, 0, 0, 0]], np.float32))
        expect = 4.0 * rad / 3.0

        def entry(rng):
            z = 2.0 * rng.random() - 1.0
            ph = 2.0 * np.pi * rng.random()
            nrm = np.array([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z])
            return c + rad * nrm, _lambert_entry(rng, c + rad * nrm, -nrm, oracle)
    else:
        h = np.array([0.8, 0.4, 0.3], np.float32).astype(np.float64)
        scene = oracle.Scene(np.array([[1, 0.2, -0.1, 0.3, *h, 0]], np.float32))
        c = np.array([0.2, -0.1, 0.3], np.float32).astype(np.float64)
        area = np.array([h[1] * h[2], h[0] * h[2], h[0] * h[1]])
        expect = 4.0 * h.prod() / (h[0] * h[1] + h[1] * h[2] + h[2] * h[0])

        def entry(rng):
            ax = rng.choice(3, p=area / area.sum())
            side = 1.0 if rng.random() < 0.5 else -1.0
            x = c + h * (2.0 * rng.random(3) - 1.0)
            x[ax] = c[ax] + side * h[ax]
            n_in = np.zeros(3)
            n_in[ax] = -side
            return x, _lambert_entry(rng, x, n_in, oracle)
    n = 8000
    lengths, colls = _mean_path(oracle, scene, entry, sigma_t, g, n, seed=11)
    se_l = lengths.std() / np.sqrt(n)
    se_k = colls.std() / np.sqrt(n)
    assert abs(lengths.mean() - expect) < 4.5 * se_l, (lengths.mean(), expect, se_l)
    assert abs(colls.mean() - sigma_t * expect) < 4.5 * se_k, (colls.mean(), sigma_t * expect, se_k)
