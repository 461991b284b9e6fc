"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds only input descriptions and seeded generators (scene
constants, cameras, lights, media, random weights and conditions).  It holds
none of the method's arithmetic, so both the GPU library and the CPU oracle
can be fed from it without sharing code.

The paper's meshes are not available; the scenes are synthetic stand-ins with
the structure of its workloads: a voluminous body with a thin part (sphere
plus box arm), density doubling, strong forward scattering g = 0.8 and
albedo near one.
"""
import numpy as np

PRIM_SPHERE, PRIM_BOX = 0, 1

# ---------------------------------------------------------------- walks
WALK_C1 = dict(n_photons=100_000, seed=0, sigma_t=10.0, g=0.8, albedo=0.99, radius=1.0)
WALK_C2 = dict(n_photons=1 << 24, seed=0, st_range=(0.1, 200.0), g_range=(-0.9, 0.95),
               albedo_range=(0.9, 1.0))

# ---------------------------------------------------------------- CVAE shapes
SHAPES = {
    "length": dict(model=0, p_in=2, p_out=1, latent=4, width=16, n_linear=3),
    "path": dict(model=1, p_in=3, p_out=3, latent=4, width=16, n_linear=3),
    "event": dict(model=2, p_in=7, p_out=6, latent=4, width=16, n_linear=3),
}
SHAPE_LIST = [SHAPES["length"], SHAPES["path"], SHAPES["event"]]

# Table 1: the hidden-layer counts D, widths W and latent sizes L examined
# per model, and the final (highlighted) setting; n_linear = D + 1.
TABLE1_GRID = {
    0: dict(p_in=2, p_out=1, D=(1, 2, 3), W=(4, 8, 12), L=(2, 6)),
    1: dict(p_in=3, p_out=3, D=(1, 2, 3), W=(8, 12, 16), L=(5, 9)),
    2: dict(p_in=7, p_out=6, D=(1, 2, 3), W=(12, 16, 20), L=(5, 9)),
}
TABLE1_FINAL = {0: dict(D=2, W=8, L=2), 1: dict(D=2, W=16, L=5), 2: dict(D=2, W=16, L=5)}


def table1_shape(model, D, W, L):
    g = TABLE1_GRID[model]
    return dict(model=model, p_in=g["p_in"], p_out=g["p_out"], latent=L, width=W, n_linear=D + 1)


def table1_fits(shape, limit=32):
    """Every width of both networks (hidden units, inputs p_out + p_in and
    latent + p_in, outputs 2 p_out and 2 latent) within `limit`: 32 for the
    training and sampling kernels (one or two 16-wide MFMA tiles per layer),
    16 for the renderer's in-kernel decoders (one tile)."""
    return (shape["width"] <= limit and shape["p_out"] + shape["p_in"] <= limit
            and shape["latent"] + shape["p_in"] <= limit and 2 * shape["p_out"] <= limit
            and 2 * shape["latent"] <= limit)


TABLE1_SHAPES = [table1_shape(m, **TABLE1_FINAL[m]) for m in range(3)]
TRAIN_C3 = dict(batch=4096, n_samples=1 << 22, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                weight_decay=0.0)


# ---------------------------------------------------------------- scenes
def prim_sphere(c, r):
    return [PRIM_SPHERE, c[0], c[1], c[2], r, 0.0, 0.0, 0.0]


def prim_box(c, half):
    return [PRIM_BOX, c[0], c[1], c[2], half[0], half[1], half[2], 0.0]


def scene_c4():
    """Unit sphere at the origin united with a 1.6 x 0.8 x 0.8 box arm centred at (1.2, 0, 0)."""
    return np.array([prim_sphere((0, 0, 0), 1.0), prim_box((1.2, 0, 0), (0.8, 0.4, 0.4))], np.float32)


def scene_sphere(r=1.0):
    return np.array([prim_sphere((0, 0, 0), r)], np.float32)


def scene_c5(seed=0, n=64):
    """64 spheres, radii U(0.05, 0.3), centres U(-0.7, 0.7)^3, from a seeded generator."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.7, 0.7, size=(n, 3))
    r = rng.uniform(0.05, 0.3, size=n)
    return np.array([prim_sphere(c[i], r[i]) for i in range(n)], np.float32)


# ---------------------------------------------------------------- triangle meshes
def icosphere(subdiv):
    """Unit icosphere: vertices [v, 3] float64 and faces [f, 3] (outward
    counter-clockwise), each face split into four `subdiv` times."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(x, np.float64) / np.linalg.norm(x) for x in v]
    for _ in range(subdiv):
        mid, nf = {}, []

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return np.array(verts), np.array(f, np.int64)


def blob_radius(u, seed=0):
    """Radial function r(u) of the star-shaped test body for unit directions
    u [n, 3]: a lumpy core of radius ~0.55 and one thin spike (an 'ear')
    along a seeded direction."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    ph = rng.uniform(0, 2 * np.pi, 3)
    lump = 0.06 * np.sin(4 * u[:, 0] + ph[0]) * np.sin(3 * u[:, 1] + ph[1]) * np.sin(2 * u[:, 2] + ph[2])
    spike = 0.55 * np.maximum(0.0, (u @ a - 0.9) / 0.1) ** 1.5
    return 0.55 + lump + spike


def mesh_blob(seed=0, subdiv=4):
    """Closed triangle mesh [f, 9] (float32 vertex triples, outward winding)
    of the star-shaped body blob_radius: an icosphere with each vertex moved
    to radius r(u) -- a voluminous body with a thin part, standing in for the
    paper's scanned meshes."""
    v, f = icosphere(subdiv)
    v = v * blob_radius(v, seed)[:, None]
    return v[f].reshape(-1, 9).astype(np.float32)


def camera_mesh(width=512, height=512):
    return dict(eye=(0.0, 0.3, 3.0), look_at=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=40.0,
                width=width, height=height)


def camera_c4(width=512, height=512):
    return dict(eye=(0.5, 0.6, 4.5), look_at=(0.5, 0.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=40.0,
                width=width, height=height)


def light_c4():
    return dict(pos=(1.5, 3.0, 3.0), intensity=10.0)


def medium_c4(sigma_t):
    return dict(sigma_t=float(sigma_t), g=0.8, albedo=0.995)


C4_SIGMAS = (10.0, 20.0, 40.0, 80.0)
C4 = dict(width=512, height=512, spp=256, sigmas=C4_SIGMAS)


def camera_c5(width=1024, height=1024):
    return dict(eye=(0.0, 0.0, 3.2), look_at=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=40.0,
                width=width, height=height)


def light_c5():
    return dict(pos=(2.0, 2.5, 3.0), intensity=10.0)


def medium_c5():
    return dict(sigma_t=100.0, g=0.8, albedo=0.995)


# ---------------------------------------------------------------- random inputs
def random_conditions(model, n, seed):
    """Raw (unstandardised) conditions spanning the training ranges of each model."""
    rng = np.random.default_rng(seed)
    lst = rng.uniform(np.log(0.1), np.log(200.0), n)
    g = rng.uniform(-0.9, 0.95, n)
    if model == 0:
        return np.stack([lst, g], 1)
    logn = rng.uniform(0.0, 8.0, n)
    if model == 1:
        return np.stack([lst, g, logn], 1)
    phi = rng.uniform(0.9, 1.0, n)
    ct = rng.uniform(-1, 1, n)
    a = rng.uniform(-0.7, 0.7, n)
    b = rng.uniform(-0.7, 0.7, n)
    return np.stack([lst, g, phi, ct, a, b, logn], 1)


def random_stats(model, seed):
    """Plausible standardisation constants [mean_c, std_c, mean_y, std_y] (16 each)."""
    rng = np.random.default_rng(seed)
    st = np.zeros(64)
    st[16:32] = 1.0
    st[48:64] = 1.0
    p_in, p_out = [(2, 1), (3, 3), (7, 6)][model]
    st[:p_in] = rng.normal(0, 0.5, p_in)
    st[16:16 + p_in] = rng.uniform(0.5, 2.0, p_in)
    st[32:32 + p_out] = rng.normal(0, 0.5, p_out)
    st[48:48 + p_out] = rng.uniform(0.3, 1.5, p_out)
    return st


def render_test_stats(model):
    """Standardisation constants that make untrained (random) decoders emit
    plausible outputs for render parity tests: N around 20, cos(theta) around
    0.3, representative events inside the unit ball."""
    st = np.zeros(64)
    st[16:32] = 1.0
    st[48:64] = 1.0
    if model == 0:
        st[0:2] = [2.0, 0.4]
        st[16:18] = [1.5, 0.5]
        st[32], st[48] = np.log(20.0), 0.5
    elif model == 1:
        st[0:3] = [2.0, 0.4, 3.0]
        st[16:19] = [1.5, 0.5, 1.0]
        st[32:35] = [0.3, 0.0, 0.0]
        st[48:51] = [0.4, 0.3, 0.3]
    else:
        st[0:7] = [2.0, 0.4, 0.95, 0.3, 0.0, 0.0, 3.0]
        st[16:23] = [1.5, 0.5, 0.03, 0.5, 0.3, 0.3, 1.0]
        st[32:38] = [0.0, 0.0, 0.3, 0.0, 0.0, 0.5]
        st[48:54] = [0.25, 0.25, 0.25, 0.4, 0.4, 0.4]
    return st
