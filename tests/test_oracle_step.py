"""Pins of the oracle's learned sphere step (Sec. 4.1 Eq. (transform) and the
exit frame, Sec. 4.3 representative-event law, Sec. 3.1 single scatter).

The step is driven by "bias-only" decoders: every weight is zero, the mean
biases are zero and the log-variance biases sit at the -12 floor, so the
standardised output is e^-6 eps; with de-standardisation mean_y = v and
std_y = 1e-13 the decoder answers v to about 1e-15.  That turns each model
into a constant and leaves only the step's own arithmetic to check:

* round trip: a training walk record (N, cos theta, alpha, beta, X, W) fed
  back through the step, for an arbitrary entry point p, radius r and entry
  direction d, must land on the walk's own exit point and direction and its
  representative event, rotated by the step's azimuth about d and placed in
  the sphere -- computed here from the walk's raw exit vectors, not from the
  parameterisation;
* the first representative event is the centre with probability
  albedo / sum_{i<=N} albedo^i (chi-square against the brute-force sum);
* a one-event step is a single Henyey-Greenstein scatter: the exit cosine
  about d follows the HG law (KS against its closed-form CDF) and the exit
  direction is radial.
"""
import numpy as np
import pytest
from scipy import stats as sps

import workloads as W

LV_FLOOR = -12.0
TINY_STD = 1e-13


def constant_model(oracle, model, values):
    """A decoder (and unused encoder) that samples `values` almost exactly."""
    shape = W.SHAPE_LIST[model]
    params = np.zeros(oracle.n_params(shape))
    nl = shape["n_linear"]
    last = (2 * nl - 1) * oracle.LAYER_FLOATS + 16 * 16  # biases of the decoder's output layer
    p_out = shape["p_out"]
    params[last + p_out: last + 2 * p_out] = LV_FLOOR
    st = np.zeros(64)
    st[16:32] = 1.0
    st[48:64] = 1.0
    st[32:32 + p_out] = values
    st[48:48 + p_out] = TINY_STD
    return dict(shape=shape, params=params, stats=st)


def constant_models(oracle, N, exit_param=(1.0, 0.0, 0.0), event=(0.1, 0.2, 0.3, 0.0, 0.0, 1.0)):
    return [constant_model(oracle, 0, [np.log(N)]), constant_model(oracle, 1, list(exit_param)),
            constant_model(oracle, 2, list(event))]


def rot_z(psi, v):
    c, s = np.cos(psi), np.sin(psi)
    return np.array([c * v[0] - s * v[1], s * v[0] + c * v[1], v[2]])


def to_world(oracle, d, v):
    """v given in the frame (e1, e2, d) of the orthonormal basis around d."""
    e1, e2 = oracle.onb(d)
    return v[0] * e1 + v[1] * e2 + v[2] * np.asarray(d)


def random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_bias_only_decoders_are_constants(oracle):
    """The device the other pins rely on: each model samples its value to ~1e-14."""
    vals = [[np.log(7.0)], [0.3, -0.2, 0.4], [0.1, -0.5, 0.2, 0.6, 0.0, -0.8]]
    for m in range(3):
        cm = constant_model(oracle, m, vals[m])
        cond = W.random_conditions(m, 64, 3)
        y = oracle.cvae_sample(cm["shape"], cm["params"], cm["stats"], cond, seed=5)
        np.testing.assert_allclose(y, np.tile(vals[m], (64, 1)), atol=1e-13, rtol=0)


def test_step_reproduces_training_walk_records(oracle):
    """Eq. (transform) and the exit frame of Sec. 4.1 are inverted exactly."""
    walk = oracle.random_walk(6000, seed=21, mode=oracle.WALK_TRAINING, st_range=(2.0, 60.0))
    n, k = walk["n_scatter"], walk["event_index"]
    rows = np.flatnonzero((n >= 2) & (k >= 2))[:150]
    assert rows.size == 150
    rng = np.random.default_rng(4)
    n_event = 0
    for i in rows:
        st, g = walk["params"][0, i], walk["params"][1, i]
        xw, ww = walk["exit_pos"][:, i], walk["exit_dir"][:, i]
        Xc, Wc = walk["event_pos"][:, i], walk["event_dir"][:, i]
        models = constant_models(oracle, float(n[i]), walk["exit_param"][:, i], np.r_[Xc, Wc])
        p, d, r = rng.uniform(-2, 2, 3), random_unit(rng), rng.uniform(0.2, 2.0)
        med = dict(sigma_t=st / r, g=g, albedo=1.0)
        s = oracle.sphere_step(med, p, d, r, path_id=int(i) + 1000, models=models, nee_samples=4)
        assert s["survived"] and s["N"] == n[i] and s["n_rep"] == 4
        # the walk's exit, turned about w_in from its own azimuth to the step's
        turn = s["psi"] - np.arctan2(xw[1], xw[0])
        np.testing.assert_allclose(s["x"], p + r * to_world(oracle, d, rot_z(turn, xw)), atol=1e-9)
        np.testing.assert_allclose(s["w"], to_world(oracle, d, rot_z(turn, ww)), atol=1e-9)
        for j in range(4):
            if s["first"][j]:
                np.testing.assert_array_equal(s["X"][j], p)
                np.testing.assert_allclose(s["W"][j], d, atol=1e-15)
                continue
            n_event += 1
            np.testing.assert_allclose(s["X"][j], p + r * to_world(oracle, d, rot_z(s["psi"], Xc)), atol=1e-9)
            np.testing.assert_allclose(s["W"][j], to_world(oracle, d, rot_z(s["psi"], Wc)), atol=1e-9)
    assert n_event > 300


def test_paper_step_uses_eventgen_for_every_event(oracle):
    """The paper's order (no exact first event): every representative event
    is EventGen's, placed by the same map."""
    rng = np.random.default_rng(8)
    ev = np.array([0.3, -0.1, 0.2, 0.0, 0.6, 0.8])
    for trial in range(40):
        models = constant_models(oracle, 3.0, (0.2, 0.1, -0.3), ev)
        p, d, r = rng.uniform(-1, 1, 3), random_unit(rng), 0.7
        s = oracle.sphere_step(dict(sigma_t=20.0, g=0.5, albedo=0.95), p, d, r, path_id=trial, models=models,
                               nee_samples=3, flags=oracle.STEP_PAPER | oracle.NEE_BEFORE_ABSORPTION)
        assert not s["first"].any()
        for j in range(3):
            np.testing.assert_allclose(s["X"][j], p + r * to_world(oracle, d, rot_z(s["psi"], ev[:3])), atol=1e-9)


@pytest.mark.parametrize("N", [2, 5, 20])
@pytest.mark.parametrize("phi", [0.9, 1.0])
def test_first_event_law(oracle, N, phi):
    """P(representative event = the first) = albedo / Lambda^(N), Lambda^(N)
    summed term by term (Sec. 4.3)."""
    lam = sum(phi ** i for i in range(1, N + 1))
    p1 = phi / lam
    models = constant_models(oracle, float(N))
    K, steps = 16, 2500
    hits = 0
    for t in range(steps):
        s = oracle.sphere_step(dict(sigma_t=10.0, g=0.3, albedo=phi), [0, 0, 0], [0, 0, 1], 1.0, path_id=t,
                               models=models, nee_samples=K, flags=oracle.NEE_BEFORE_ABSORPTION)
        hits += int(s["first"].sum())
    total = K * steps
    chi2 = (hits - total * p1) ** 2 / (total * p1) + (hits - total * p1) ** 2 / (total * (1 - p1))
    assert sps.chi2.sf(chi2, 1) > 1e-4, (hits / total, p1)


def hg_cdf(g, mu):
    """Closed-form CDF of the Henyey-Greenstein cosine (Eq. 1 integrated)."""
    if abs(g) < 1e-12:
        return 0.5 * (mu + 1.0)
    return (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * mu) ** -0.5 - 1.0 / (1 + g))


@pytest.mark.parametrize("g", [0.8, -0.4])
def test_single_event_step_is_one_hg_scatter(oracle, g):
    """N = 1: the exit cosine about the entry direction is HG(g) and the exit
    direction is radial (alpha = beta = 0)."""
    models = constant_models(oracle, 1.0, (0.9, 0.3, 0.3))  # PathGen would be wrong if asked
    rng = np.random.default_rng(9)
    cosines = []
    for t in range(4000):
        p, d, r = rng.uniform(-1, 1, 3), random_unit(rng), rng.uniform(0.3, 1.5)
        s = oracle.sphere_step(dict(sigma_t=5.0 / r, g=g, albedo=1.0), p, d, r, path_id=t, models=models)
        assert s["N"] == 1 and s["first"][0]
        u = (s["x"] - p) / r
        np.testing.assert_allclose(np.linalg.norm(u), 1.0, atol=1e-12)
        np.testing.assert_allclose(s["w"], u, atol=1e-12)
        cosines.append(float(u @ d))
    ks = sps.kstest(cosines, lambda m: np.array([hg_cdf(g, x) for x in np.atleast_1d(m)]))
    assert ks.pvalue > 1e-4, ks
