"""ctypes mirror of include/msst.h and the loader of libmsst.so."""
import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmsst.so")

MS_OK, MS_ERR_INVALID_ARGUMENT, MS_ERR_DEVICE, MS_ERR_UNSUPPORTED, MS_ERR_WORKSPACE_TOO_SMALL = 0, -1, -2, -3, -4
TAG_WALK_EVENT, TAG_WALK_PARAM, TAG_CVAE_INIT, TAG_CVAE_BATCH = 0, 1, 2, 3
TAG_CVAE_REPARAM, TAG_CVAE_SAMPLE, TAG_RENDER_PIXEL, TAG_RENDER_PATH = 4, 5, 6, 7
TAG_SCENE, TAG_DEQUANT = 8, 9
WALK_ANALOG, WALK_TRAINING = 0, 1
EVENT_ALBEDO_POWER, EVENT_UNIFORM = 0, 1
MODEL_LENGTH, MODEL_PATH, MODEL_EVENT = 0, 1, 2
PREC_BF16, PREC_FP8 = 1, 2
PRIM_SPHERE, PRIM_BOX = 0, 1
METHOD_PLAIN_NEE, METHOD_ST = 1, 2
SAMPLER_CVAE, SAMPLER_EXACT_WALK = 0, 1
RENDER_NEE_BEFORE_ABSORPTION, RENDER_STEP_PAPER = 1, 2


class MsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libmsst status {status}: {message}")
        self.status = status


class WalkDesc(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("photon_offset", C.c_uint64), ("n_photons", C.c_uint64),
                ("mode", C.c_int32), ("event_weighting", C.c_int32),
                ("sigma_t", C.c_double), ("g", C.c_double), ("albedo", C.c_double), ("radius", C.c_double),
                ("st_range", C.c_double * 2), ("g_range", C.c_double * 2), ("albedo_range", C.c_double * 2),
                ("max_events", C.c_uint32), ("blocks_per_cu", C.c_int32), ("focus_fraction", C.c_double),
                ("focus_st_range", C.c_double * 2), ("focus_g_range", C.c_double * 2)]


class WalkOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("params", "n_scatter", "event_index", "absorbed", "truncated",
                                           "exit_pos", "exit_dir", "exit_param", "event_pos", "event_dir",
                                           "counters")]


class CvaeShape(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("model", "p_in", "p_out", "latent", "width", "n_linear")]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double), ("step", C.c_int64)]


class Scene(C.Structure):
    _fields_ = [("prims", C.c_void_p), ("n_prims", C.c_int32), ("sdf_fp16", C.c_void_p), ("res", C.c_int32),
                ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("tris", C.c_void_p), ("n_tris", C.c_int32),
                ("bvh", C.c_void_p), ("n_nodes", C.c_int32)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class Light(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("intensity", C.c_float)]


class Medium(C.Structure):
    _fields_ = [("sigma_t", C.c_float), ("g", C.c_float), ("albedo", C.c_float)]


class RenderDesc(C.Structure):
    _fields_ = [("method", C.c_int32), ("sampler", C.c_int32), ("packed", C.c_void_p * 3),
                ("tau_min", C.c_float), ("st_max", C.c_float), ("spp", C.c_int32), ("chunk", C.c_int32),
                ("seed", C.c_uint64), ("sample_offset", C.c_uint64), ("max_events", C.c_uint32),
                ("blocks_per_cu", C.c_int32), ("cvae_batch_min", C.c_int32), ("restart_min", C.c_int32), ("max_wait", C.c_int32),
                ("nee_samples", C.c_int32),
                ("flags", C.c_int32), ("min_chain", C.c_float), ("nee_chain", C.c_int32)]


class ImageOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("sum", "comp", "sumsq", "events", "steps", "counters")]


_vp, _u64, _u32, _i32, _i64, _sz = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32, C.c_int64, C.c_size_t
_P = C.POINTER

SIGNATURES = {
    "ms_abi_version": ([], C.c_int32),
    "ms_last_error": ([], C.c_char_p),
    "ms_philox_fill": ([_u64, _u32, _u64, _i64, _u32, _i32, _vp, _vp], C.c_int32),
    "ms_random_walk_workspace_size": ([_P(WalkDesc), _P(_sz)], C.c_int32),
    "ms_random_walk": ([_P(WalkDesc), _P(WalkOut), _vp, _sz, _vp], C.c_int32),
    "cvae_param_count": ([_P(CvaeShape), _P(_sz)], C.c_int32),
    "cvae_init": ([_P(CvaeShape), _u64, _vp, _vp], C.c_int32),
    "cvae_features": ([_i32, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _u64, _u64, _vp, _vp, _vp, _vp], C.c_int32),
    "ms_select_rows_workspace_size": ([_i64, _P(_sz)], C.c_int32),
    "ms_select_rows": ([_i64, _vp, _vp, _u32, _u32, _vp, _vp, _vp, _sz, _vp], C.c_int32),
    "ms_column_moments_workspace_size": ([_i64, _i32, _P(_sz)], C.c_int32),
    "ms_column_moments": ([_vp, _i64, _i32, _vp, _vp, _sz, _vp], C.c_int32),
    "cvae_workspace_size": ([_P(CvaeShape), _i32, _P(_sz)], C.c_int32),
    "cvae_train_step": ([_P(CvaeShape), _vp, _vp, _vp, _P(Adam), _vp, _vp, _i64, _i32, _i32, _u64, _i64,
                         _u64, C.c_double, _vp, _sz, _vp, _vp, _vp], C.c_int32),
    "cvae_train_step_noalloc": ([_P(CvaeShape), _vp, _vp, _vp, _P(Adam), _vp, _vp, _i64, _i32, _i32, _u64, _i64,
                                 _u64, C.c_double, _vp, _vp, _vp], C.c_int32),
    "cvae_packed_bytes": ([], C.c_size_t),
    "cvae_pack": ([_P(CvaeShape), _vp, _vp, _i32, _vp, _i64, _vp, _sz, _vp], C.c_int32),
    "cvae_sample": ([_vp, _vp, _i64, _u64, _u64, _vp, _vp], C.c_int32),
    "sphere_trace_render_workspace_size": ([_P(Camera), _P(RenderDesc), _P(_sz)], C.c_int32),
    "sphere_trace_render": ([_P(Scene), _P(Camera), _P(Light), _P(Medium), _P(RenderDesc), _P(ImageOut), _vp,
                             _sz, _vp], C.c_int32),
    "ms_build_sdf_grid": ([_P(Scene), _i32, _vp, _vp], C.c_int32),
    "ms_mesh_bvh_size": ([_i32, _P(_sz)], C.c_int32),
    "ms_build_mesh_bvh": ([_vp, _i32, _vp, _sz, _vp, _P(_i32)], C.c_int32),
    "ms_image_stats_workspace_size": ([_i64, _P(_sz)], C.c_int32),
    "ms_image_stats": ([_vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp, _sz, _vp], C.c_int32),
}

_LIB = None


def lib():
    """Loads libmsst.so.  Raises if it has not been built: there is no fallback."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with paper_2011_03082_amd.build.build() "
                              "(the HIP library is required, there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            if not hasattr(L, name):
                continue  # reported by the export test; calling it raises AttributeError
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def check(status):
    if status != MS_OK:
        raise MsError(status, lib().ms_last_error().decode(errors="replace"))
    return status
