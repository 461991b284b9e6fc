"""Pins of the oracle's triangle-mesh geometry (the polygon-mesh boundary of
Sec. 3 and Sec. 5): an icosphere against the analytic sphere, the blob mesh
against its own radial function, closedness of every line, and conservative
radii from an FP16 grid built on the mesh."""
import numpy as np
import pytest

import workloads as W


def unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


@pytest.fixture(scope="module")
def sphere_mesh(oracle):
    v, f = W.icosphere(4)
    R = 0.7
    tris = (R * v)[f].reshape(-1, 9).astype(np.float32)
    return oracle.Scene(None, tris=tris), R


@pytest.fixture(scope="module")
def blob(oracle):
    return oracle.Scene(None, tris=W.mesh_blob(0, 3))


def test_icosphere_intervals_match_the_sphere(sphere_mesh):
    sc, R = sphere_mesh
    rng = np.random.default_rng(0)
    # chord error of a subdivision-4 icosphere: edges span ~0.07 rad, so the
    # faces lie within R (1 - cos 0.04) ~ 6e-4 of the sphere
    for _ in range(200):
        d = unit(rng.normal(size=3))
        o = rng.uniform(-2, 2, 3)
        b = o @ d
        h2 = o @ o - b * b
        iv = sc.intervals(o, d)
        if h2 > (0.8 * R) ** 2:  # misses or grazes: skip the grazing band
            if h2 > (1.05 * R) ** 2:
                assert len(iv) == 0
            continue
        s = np.sqrt(R * R - h2)
        assert len(iv) == 1
        np.testing.assert_allclose(iv[0], (-b - s, -b + s), atol=3e-3)


def test_icosphere_signed_distance(sphere_mesh, oracle):
    sc, R = sphere_mesh
    rng = np.random.default_rng(1)
    p = rng.uniform(-1.2, 1.2, (300, 3))
    sd = np.array([sc.sdf(x) for x in p])
    np.testing.assert_allclose(sd, np.linalg.norm(p, axis=1) - R, atol=1.5e-3)


def test_blob_inside_test_follows_the_radial_function(blob):
    rng = np.random.default_rng(2)
    p = rng.uniform(-1.2, 1.2, (600, 3))
    r = np.linalg.norm(p, axis=1)
    rr = W.blob_radius(p / r[:, None], 0)
    far = np.abs(r - rr) > 0.05  # away from the polygonal approximation band
    sd = np.array([blob.sdf(x) for x in p[far]])
    np.testing.assert_array_equal(sd < 0, (r < rr)[far])


def test_every_line_crosses_the_closed_mesh_an_even_number_of_times(blob):
    rng = np.random.default_rng(3)
    for _ in range(300):
        o = unit(rng.normal(size=3)) * rng.uniform(0.0, 0.4)  # inside the core (radius >= 0.49)
        d = unit(rng.normal(size=3))
        iv = blob.intervals(o, d)
        assert len(iv) >= 1
        # the origin lies inside: one interval contains t = 0
        assert sum(a <= 0.0 <= b for a, b in iv) == 1
        for a, b in iv:
            assert a < b


def test_grid_radii_on_the_mesh_are_conservative(oracle, blob):
    res, lo, hi = 32, (-1.2, -1.2, -1.2), (1.2, 1.2, 1.2)
    grid = blob.build_grid(res, lo, hi)
    sc = oracle.Scene(None, sdf_fp16=grid, lo=lo, hi=hi, tris=W.mesh_blob(0, 3))
    rng = np.random.default_rng(4)
    checked = 0
    for x in rng.uniform(-0.6, 0.6, (400, 3)):
        r = sc.conservative_radius(x)
        if r <= 0.0:
            continue
        checked += 1
        q = x + r * unit(rng.normal(size=(64, 3)))
        assert all(blob.sdf(y) <= 1e-9 for y in q)
    assert checked > 60
