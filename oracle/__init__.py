"""FP64 CPU oracle for learned sphere tracing (arXiv 2011.03082) -- ctypes binding.

TEST INFRASTRUCTURE ONLY: the plain, slow, double-precision reference that the
HIP library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.  It shares no code with the GPU library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

TAG_WALK_EVENT, TAG_WALK_PARAM, TAG_CVAE_INIT, TAG_CVAE_BATCH = 0, 1, 2, 3
TAG_CVAE_REPARAM, TAG_CVAE_SAMPLE, TAG_RENDER_PIXEL, TAG_RENDER_PATH = 4, 5, 6, 7
TAG_SCENE, TAG_DEQUANT = 8, 9
WALK_ANALOG, WALK_TRAINING = 0, 1
EVENT_ALBEDO_POWER, EVENT_UNIFORM = 0, 1
PREC_FP64, PREC_BF16, PREC_FP8 = 0, 1, 2
METHOD_PLAIN_NEE, METHOD_ST = 1, 2
SAMPLER_CVAE, SAMPLER_EXACT_WALK = 0, 1
NEE_BEFORE_ABSORPTION = 1  # render flag: CVAE steps add direct light before the absorption test
STEP_PAPER = 2  # render flag: the learned step as printed (PathGen and EventGen for every case)
MAX_NEE = 16
LAYER_FLOATS = 16 * 16 + 16  # one-tile shapes (every network width <= 16)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 64))


class _Shape(C.Structure):
    _fields_ = [("model", C.c_int32), ("p_in", C.c_int32), ("p_out", C.c_int32),
                ("latent", C.c_int32), ("width", C.c_int32), ("n_linear", C.c_int32)]


class _WalkDesc(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("photon_offset", C.c_uint64), ("n_photons", C.c_uint64),
                ("mode", C.c_int32), ("event_weighting", C.c_int32),
                ("sigma_t", C.c_double), ("g", C.c_double), ("albedo", C.c_double),
                ("radius", C.c_double), ("st_range", C.c_double * 2), ("g_range", C.c_double * 2),
                ("albedo_range", C.c_double * 2), ("max_events", C.c_uint32),
                ("n_threads", C.c_int32), ("focus_fraction", C.c_double),
                ("focus_st_range", C.c_double * 2), ("focus_g_range", C.c_double * 2)]


class _WalkOut(C.Structure):
    _fields_ = [("params", C.c_void_p), ("n_scatter", C.c_void_p), ("event_index", C.c_void_p),
                ("absorbed", C.c_void_p), ("truncated", C.c_void_p), ("exit_pos", C.c_void_p),
                ("exit_dir", C.c_void_p), ("exit_param", C.c_void_p), ("event_pos", C.c_void_p),
                ("event_dir", C.c_void_p)]


class _Scene(C.Structure):
    _fields_ = [("prims", C.c_void_p), ("n_prims", C.c_int32), ("sdf_fp16", C.c_void_p),
                ("res", C.c_int32), ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("tris", C.c_void_p),
                ("n_tris", C.c_int32)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("look_at", C.c_double * 3), ("up", C.c_double * 3),
                ("vfov_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Light(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("intensity", C.c_double)]


class _Medium(C.Structure):
    _fields_ = [("sigma_t", C.c_double), ("g", C.c_double), ("albedo", C.c_double)]


class _RenderDesc(C.Structure):
    _fields_ = [("method", C.c_int32), ("sampler", C.c_int32), ("precision", C.c_int32),
                ("shapes", _Shape * 3), ("params", C.c_void_p * 3), ("stats", C.c_void_p * 3),
                ("act_scales", C.c_void_p * 3), ("tau_min", C.c_double), ("st_max", C.c_double),
                ("spp", C.c_int32), ("seed", C.c_uint64), ("sample_offset", C.c_uint64),
                ("max_events", C.c_uint32), ("pixels", C.c_void_p), ("n_pixels", C.c_int64),
                ("n_threads", C.c_int32), ("nee_samples", C.c_int32), ("flags", C.c_int32),
                ("nee_chain", C.c_int32)]


class _StepResult(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("w", C.c_double * 3), ("X", (C.c_double * 3) * MAX_NEE),
                ("W", (C.c_double * 3) * MAX_NEE), ("first", C.c_int * MAX_NEE), ("n_rep", C.c_int),
                ("nee_w", C.c_double), ("N", C.c_double), ("survived", C.c_int), ("psi", C.c_double)]


class _ImageOut(C.Structure):
    _fields_ = [("sum", C.c_void_p), ("sumsq", C.c_void_p), ("events", C.c_void_p),
                ("steps", C.c_void_p)]


def lib():
    """Loads liboracle.so, building it first if it is missing."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        vp, u64, u32, i32, i64, dbl = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32, C.c_int64, C.c_double
        L.or_philox4x32_10.argtypes = [vp, vp, vp]
        L.or_philox_blocks.argtypes = [u64, u32, u64, u32, C.c_int, vp]
        L.or_u01.argtypes = [u32]
        L.or_u01.restype = dbl
        L.or_hg_eval.argtypes = [dbl, dbl]
        L.or_hg_eval.restype = dbl
        L.or_hg_sample.argtypes = [dbl, dbl]
        L.or_hg_sample.restype = dbl
        L.or_onb.argtypes = [vp, vp, vp]
        L.or_scatter_dir.argtypes = [vp, dbl, dbl]
        L.or_random_walk.argtypes = [C.POINTER(_WalkDesc), C.POINTER(_WalkOut)]
        L.or_softplus.argtypes = [dbl]
        L.or_softplus.restype = dbl
        L.or_round_bf16.argtypes = [dbl]
        L.or_round_bf16.restype = dbl
        L.or_round_fp8_e4m3.argtypes = [dbl]
        L.or_round_fp8_e4m3.restype = dbl
        L.or_cvae_param_count.argtypes = [C.POINTER(_Shape)]
        L.or_cvae_param_count.restype = i64
        L.or_cvae_init.argtypes = [C.POINTER(_Shape), u64, vp]
        L.or_cvae_loss_grad.argtypes = [C.POINTER(_Shape), vp, i32, vp, vp, u64, i64, u64, dbl, vp, vp, vp]
        L.or_cvae_loss_grad.restype = dbl
        L.or_adamw_step.argtypes = [i32, vp, vp, vp, vp, dbl, dbl, dbl, dbl, dbl, i64]
        L.or_cvae_sample.argtypes = [C.POINTER(_Shape), vp, vp, i32, vp, vp, i64, u64, u64, vp]
        L.or_cvae_decode.argtypes = [C.POINTER(_Shape), vp, i32, vp, vp, vp, vp, vp]
        L.or_cvae_act_scales.argtypes = [C.POINTER(_Shape), vp, vp, vp, i64, vp]
        L.or_cvae_features.argtypes = [i32, i64, vp, vp, vp, vp, vp, u64, u64, vp, vp]
        L.or_scene_sdf.argtypes = [C.POINTER(_Scene), vp]
        L.or_scene_sdf.restype = dbl
        L.or_ray_intervals.argtypes = [C.POINTER(_Scene), vp, vp, vp, vp, C.c_int]
        L.or_ray_intervals.restype = C.c_int
        L.or_conservative_radius.argtypes = [C.POINTER(_Scene), vp]
        L.or_conservative_radius.restype = dbl
        L.or_build_sdf_grid.argtypes = [C.POINTER(_Scene), i32, vp, vp, vp]
        L.or_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Light),
                                C.POINTER(_Medium), C.POINTER(_RenderDesc), C.POINTER(_ImageOut)]
        L.or_sphere_step.argtypes = [C.POINTER(_RenderDesc), C.POINTER(_Medium), u64, u32, vp, vp, dbl,
                                     C.POINTER(_StepResult)]
        L.or_sphere_step.restype = u32
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _shape(s):
    return _Shape(s["model"], s["p_in"], s["p_out"], s["latent"], s["width"], s["n_linear"])


# ---------------------------------------------------------------- randomness
def philox4x32_10(counter, key):
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_blocks(seed, tag, ident, c0, n):
    out = np.zeros((n, 4), np.uint32)
    lib().or_philox_blocks(seed, tag, ident, c0, n, _p(out))
    return out


def u01(word):
    return lib().or_u01(int(word))


# ---------------------------------------------------------------- scattering
def hg_eval(g, cos_theta):
    return lib().or_hg_eval(float(g), float(cos_theta))


def hg_sample(g, xi):
    return lib().or_hg_sample(float(g), float(xi))


def onb(n):
    n = np.ascontiguousarray(n, dtype=np.float64)
    b1, b2 = np.zeros(3), np.zeros(3)
    lib().or_onb(_p(n), _p(b1), _p(b2))
    return b1, b2


def scatter_dir(d, mu, azimuth):
    d = np.array(d, dtype=np.float64)
    lib().or_scatter_dir(_p(d), float(mu), float(azimuth))
    return d


def random_walk(n_photons, seed=0, photon_offset=0, mode=WALK_ANALOG, sigma_t=10.0, g=0.8,
                albedo=0.99, radius=1.0, st_range=(0.1, 200.0), g_range=(-0.9, 0.95),
                albedo_range=(0.9, 1.0), event_weighting=EVENT_ALBEDO_POWER,
                max_events=1 << 20, n_threads=None, focus_fraction=0.0, focus_st_range=(1.0, 1.0),
                focus_g_range=(0.0, 0.0)):
    """Random walks from the centre of a sphere (Sec. 3.1); planar outputs."""
    n = int(n_photons)
    out = {
        "params": np.zeros((3, n)), "n_scatter": np.zeros(n, np.uint32),
        "event_index": np.zeros(n, np.uint32), "absorbed": np.zeros(n, np.uint8),
        "truncated": np.zeros(n, np.uint8), "exit_pos": np.zeros((3, n)),
        "exit_dir": np.zeros((3, n)), "exit_param": np.zeros((3, n)),
        "event_pos": np.zeros((3, n)), "event_dir": np.zeros((3, n)),
    }
    d = _WalkDesc(seed, photon_offset, n, mode, event_weighting, sigma_t, g, albedo, radius,
                  (C.c_double * 2)(*st_range), (C.c_double * 2)(*g_range),
                  (C.c_double * 2)(*albedo_range), max_events,
                  n_threads if n_threads else default_threads(), focus_fraction,
                  (C.c_double * 2)(*focus_st_range), (C.c_double * 2)(*focus_g_range))
    o = _WalkOut(*[_p(out[k]) for k in ("params", "n_scatter", "event_index", "absorbed",
                                         "truncated", "exit_pos", "exit_dir", "exit_param",
                                         "event_pos", "event_dir")])
    lib().or_random_walk(C.byref(d), C.byref(o))
    return out


# ---------------------------------------------------------------- CVAE
SHAPES = {
    "length": dict(model=0, p_in=2, p_out=1, latent=4, width=16, n_linear=3),
    "path": dict(model=1, p_in=3, p_out=3, latent=4, width=16, n_linear=3),
    "event": dict(model=2, p_in=7, p_out=6, latent=4, width=16, n_linear=3),
}


def n_params(shape):
    s = _shape(shape)
    return int(lib().or_cvae_param_count(C.byref(s)))


def layer_stride(shape):
    """Row stride S of a layer's S x S weight block (16 or 32)."""
    lf = n_params(shape) // (2 * shape["n_linear"])
    return 16 if lf == 16 * 16 + 16 else 32


def softplus(x):
    return lib().or_softplus(float(x))


def round_bf16(x):
    return lib().or_round_bf16(float(x))


def round_fp8_e4m3(x):
    return lib().or_round_fp8_e4m3(float(x))


def cvae_init(shape, seed):
    p = np.zeros(n_params(shape))
    s = _shape(shape)
    lib().or_cvae_init(C.byref(s), seed, _p(p))
    return p


def cvae_loss_grad(shape, params, cond, target, seed, step, id_offset=0, want_grad=True, kl_weight=1.0):
    params = np.ascontiguousarray(params, dtype=np.float64)
    cond = np.ascontiguousarray(cond, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    B = cond.shape[0]
    grad = np.zeros(n_params(shape)) if want_grad else None
    kl, nll = C.c_double(), C.c_double()
    s = _shape(shape)
    loss = lib().or_cvae_loss_grad(C.byref(s), _p(params), B, _p(cond), _p(target), seed, step,
                                   id_offset, kl_weight, _p(grad), C.byref(kl), C.byref(nll))
    return loss, kl.value, nll.value, grad


def adamw_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    lib().or_adamw_step(params.size, _p(params), _p(m), _p(v), _p(grad), lr, beta1, beta2, eps,
                        weight_decay, step)


def cvae_decode(shape, params, z, cond_std, precision=PREC_FP64, act_scales=None):
    params = np.ascontiguousarray(params, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    cs = np.ascontiguousarray(cond_std, dtype=np.float64)
    mu, lv = np.zeros(16), np.zeros(16)
    s = _shape(shape)
    a = None if act_scales is None else np.ascontiguousarray(act_scales, dtype=np.float64)
    lib().or_cvae_decode(C.byref(s), _p(params), precision, _p(a), _p(z), _p(cs), _p(mu), _p(lv))
    return mu[: shape["p_out"]], lv[: shape["p_out"]]


def cvae_sample(shape, params, stats, cond, seed, id_offset=0, precision=PREC_FP64, act_scales=None):
    params = np.ascontiguousarray(params, dtype=np.float64)
    stats = np.ascontiguousarray(stats, dtype=np.float64)
    cond = np.ascontiguousarray(cond, dtype=np.float64)
    n = cond.shape[0]
    out = np.zeros((n, shape["p_out"]))
    s = _shape(shape)
    a = None if act_scales is None else np.ascontiguousarray(act_scales, dtype=np.float64)
    lib().or_cvae_sample(C.byref(s), _p(params), _p(stats), precision, _p(a), _p(cond), n, seed,
                         id_offset, _p(out))
    return out


def cvae_act_scales(shape, params, stats, cond):
    """Per-layer FP8 activation scales (powers of two) of the decoder from raw
    calibration conditions [n, p_in]; z of row i from the sampler's seed-0
    stream, id i."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    stats = np.ascontiguousarray(stats, dtype=np.float64)
    cond = np.ascontiguousarray(cond, dtype=np.float64)
    out = np.zeros(8)
    lib().or_cvae_act_scales(C.byref(_shape(shape)), _p(params), _p(stats), _p(cond), cond.shape[0], _p(out))
    return out[: shape["n_linear"]].copy()


def cvae_features(model, walk, seed, id_offset=0):
    n = walk["n_scatter"].size
    p_in = [2, 3, 7][model]
    p_out = [1, 3, 6][model]
    cond, target = np.zeros((n, p_in)), np.zeros((n, p_out))
    arrs = [np.ascontiguousarray(walk[k], dtype=(np.uint32 if k == "n_scatter" else np.float64))
            for k in ("params", "n_scatter", "exit_param", "event_pos", "event_dir")]
    lib().or_cvae_features(model, n, *[_p(a) for a in arrs], seed, id_offset, _p(cond), _p(target))
    return cond, target


# ---------------------------------------------------------------- scenes and rendering
class Scene:
    """Primitives [n, 8] or, with tris ([n, 9] float32 vertex triples of a
    closed mesh), the mesh interior; optional FP16 distance grid."""

    def __init__(self, prims, sdf_fp16=None, lo=(-1, -1, -1), hi=(1, 1, 1), tris=None):
        self.prims = np.ascontiguousarray(prims if prims is not None else np.zeros((0, 8)),
                                          dtype=np.float32).reshape(-1, 8)
        self.grid = None if sdf_fp16 is None else np.ascontiguousarray(sdf_fp16, dtype=np.uint16)
        self.tris = None if tris is None else np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 9)
        res = 0 if self.grid is None else int(round(self.grid.size ** (1 / 3)))
        self.c = _Scene(_p(self.prims), self.prims.shape[0], _p(self.grid), res,
                        (C.c_float * 3)(*lo), (C.c_float * 3)(*hi), _p(self.tris),
                        0 if self.tris is None else self.tris.shape[0])

    def sdf(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        return lib().or_scene_sdf(C.byref(self.c), _p(p))

    def intervals(self, o, d, cap=16):
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        t0, t1 = np.zeros(cap), np.zeros(cap)
        m = lib().or_ray_intervals(C.byref(self.c), _p(o), _p(d), _p(t0), _p(t1), cap)
        return list(zip(t0[:m], t1[:m]))

    def conservative_radius(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        return lib().or_conservative_radius(C.byref(self.c), _p(p))

    def build_grid(self, res, lo=(-1, -1, -1), hi=(1, 1, 1)):
        out = np.zeros(res ** 3, np.uint16)
        lo_a = np.array(lo, np.float32)
        hi_a = np.array(hi, np.float32)
        lib().or_build_sdf_grid(C.byref(self.c), res, _p(lo_a), _p(hi_a), _p(out))
        return out


def render(scene, camera, light, medium, method=METHOD_PLAIN_NEE, sampler=SAMPLER_CVAE,
           precision=PREC_FP64, models=None, tau_min=0.1, st_max=200.0, spp=1, seed=0,
           sample_offset=0, max_events=1 << 20, pixels=None, n_threads=None, nee_samples=1, flags=0,
           nee_chain=0):
    """Renders (a pixel subset of) an image; returns per-pixel sums over spp.

    camera: dict(eye, look_at, up, vfov_deg, width, height); light: dict(pos,
    intensity); medium: dict(sigma_t, g, albedo); models: list of three dicts
    with keys shape, params (float64 master weights), stats (64 doubles) and
    optionally act_scales.
    """
    cam = _Camera((C.c_double * 3)(*camera["eye"]), (C.c_double * 3)(*camera["look_at"]),
                  (C.c_double * 3)(*camera["up"]), camera["vfov_deg"], camera["width"],
                  camera["height"])
    lt = _Light((C.c_double * 3)(*light["pos"]), light["intensity"])
    md = _Medium(medium["sigma_t"], medium["g"], medium["albedo"])
    rd, keep = _render_desc(method, sampler, precision, models, tau_min, st_max, seed, nee_samples, flags,
                            nee_chain)
    rd.spp, rd.sample_offset, rd.max_events = spp, sample_offset, max_events
    npx = camera["width"] * camera["height"]
    if pixels is not None:
        px = np.ascontiguousarray(pixels, dtype=np.int32)
        keep.append(px)
        rd.pixels = px.ctypes.data
        rd.n_pixels = px.size
        npx = px.size
    rd.n_threads = n_threads if n_threads else default_threads()
    res = {k: np.zeros(npx) for k in ("sum", "sumsq", "events", "steps")}
    img = _ImageOut(*[_p(res[k]) for k in ("sum", "sumsq", "events", "steps")])
    lib().or_render(C.byref(scene.c), C.byref(cam), C.byref(lt), C.byref(md), C.byref(rd),
                    C.byref(img))
    return res


def _render_desc(method, sampler, precision, models, tau_min, st_max, seed, nee_samples, flags, nee_chain=0):
    """Render descriptor and the arrays it points into (keep them alive)."""
    keep = []
    rd = _RenderDesc()
    rd.method, rd.sampler, rd.precision = method, sampler, precision
    for i in range(3):
        if models is not None:
            m = models[i]
            rd.shapes[i] = _shape(m["shape"])
            prm = np.ascontiguousarray(m["params"], dtype=np.float64)
            st = np.ascontiguousarray(m["stats"], dtype=np.float64)
            keep += [prm, st]
            rd.params[i] = prm.ctypes.data
            rd.stats[i] = st.ctypes.data
            if m.get("act_scales") is not None:
                a = np.ascontiguousarray(m["act_scales"], dtype=np.float64)
                keep.append(a)
                rd.act_scales[i] = a.ctypes.data
        else:
            rd.shapes[i] = _shape(list(SHAPES.values())[i])
    rd.tau_min, rd.st_max, rd.seed = tau_min, st_max, seed
    rd.nee_samples, rd.flags, rd.nee_chain = nee_samples, flags, nee_chain
    rd.max_events = 1 << 20
    return rd, keep


def sphere_step(medium, p, d, r, path_id, c0=0, models=None, sampler=SAMPLER_CVAE, precision=PREC_FP64,
                seed=0, nee_samples=1, flags=0, nee_chain=0):
    """One sphere step around p (radius r, entered along unit d) for the path
    with Philox id path_id, its draw counter at c0: the learned step (models as
    for render) or the exact in-sphere walk.  Returns the world-frame exit,
    representative events, weights, N, survival, psi and the counter after
    the step."""
    rd, keep = _render_desc(METHOD_ST, sampler, precision, models, 0.0, 200.0, seed, nee_samples, flags, nee_chain)
    md = _Medium(medium["sigma_t"], medium["g"], medium["albedo"])
    pa = np.ascontiguousarray(p, dtype=np.float64)
    da = np.ascontiguousarray(d, dtype=np.float64)
    out = _StepResult()
    c_end = lib().or_sphere_step(C.byref(rd), C.byref(md), int(path_id), int(c0), _p(pa), _p(da), float(r),
                                 C.byref(out))
    k = max(1, nee_samples)
    return dict(x=np.array(out.x[:]), w=np.array(out.w[:]), X=np.array([out.X[i][:] for i in range(k)]),
                W=np.array([out.W[i][:] for i in range(k)]), first=np.array(out.first[:k], bool),
                n_rep=out.n_rep, nee_w=out.nee_w, N=out.N, survived=bool(out.survived), psi=out.psi,
                c0=int(c_end))
