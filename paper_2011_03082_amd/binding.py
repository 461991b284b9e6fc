"""Thin Python binding of libmsst: argument marshalling only.

Functions named like the C entry points take torch device tensors and plain
numbers, fill the C descriptor structs and call the library on the current
torch stream.  The helpers at the bottom only allocate outputs and
workspaces and then call those functions, or write and read a model's
training state; every step of the computation runs in the HIP kernels.
"""
import ctypes as C
import json

import torch

from . import _abi
from ._abi import check, lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libmsst takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libmsst takes contiguous tensors")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def ms_abi_version():
    return lib().ms_abi_version()


def ms_last_error():
    return lib().ms_last_error().decode(errors="replace")


def ms_philox_fill(seed, tag, id0, n_ids, c0, n_draws, out, stream=None):
    check(lib().ms_philox_fill(seed, tag, id0, n_ids, c0, n_draws, _ptr(out), _stream(stream)))


# ---------------------------------------------------------------- walk
def walk_desc(n_photons, seed=0, photon_offset=0, mode=_abi.WALK_ANALOG, sigma_t=10.0, g=0.8, albedo=0.99,
              radius=1.0, st_range=(0.1, 200.0), g_range=(-0.9, 0.95), albedo_range=(0.9, 1.0),
              event_weighting=_abi.EVENT_ALBEDO_POWER, max_events=1 << 20, blocks_per_cu=0, focus_fraction=0.0,
              focus_st_range=(1.0, 1.0), focus_g_range=(0.0, 0.0)):
    return _abi.WalkDesc(seed, photon_offset, n_photons, mode, event_weighting, sigma_t, g, albedo, radius,
                         (C.c_double * 2)(*st_range), (C.c_double * 2)(*g_range),
                         (C.c_double * 2)(*albedo_range), max_events, blocks_per_cu, focus_fraction,
                         (C.c_double * 2)(*focus_st_range), (C.c_double * 2)(*focus_g_range))


WALK_FIELDS = ("params", "n_scatter", "event_index", "absorbed", "truncated", "exit_pos", "exit_dir",
               "exit_param", "event_pos", "event_dir", "counters")


def ms_random_walk_workspace_size(desc):
    n = C.c_size_t()
    check(lib().ms_random_walk_workspace_size(C.byref(desc), C.byref(n)))
    return n.value


def ms_random_walk(desc, out, workspace, stream=None):
    o = _abi.WalkOut(*[_ptr(out.get(k)) for k in WALK_FIELDS])
    check(lib().ms_random_walk(C.byref(desc), C.byref(o), _ptr(workspace), workspace.numel(),
                               _stream(stream)))


def alloc_walk_outputs(n, mode, device="cuda"):
    f = dict(device=device)
    out = {
        "params": torch.empty((3, n), dtype=torch.float32, **f),
        "n_scatter": torch.empty(n, dtype=torch.int32, **f),
        "absorbed": torch.empty(n, dtype=torch.uint8, **f),
        "truncated": torch.empty(n, dtype=torch.uint8, **f),
        "exit_pos": torch.empty((3, n), dtype=torch.float32, **f),
        "exit_dir": torch.empty((3, n), dtype=torch.float32, **f),
        "exit_param": torch.empty((3, n), dtype=torch.float32, **f),
        "counters": torch.zeros(4, dtype=torch.int64, **f),
    }
    if mode == _abi.WALK_TRAINING:
        out["event_index"] = torch.empty(n, dtype=torch.int32, **f)
        out["event_pos"] = torch.empty((3, n), dtype=torch.float32, **f)
        out["event_dir"] = torch.empty((3, n), dtype=torch.float32, **f)
    return out


def random_walk(n_photons, device="cuda", stream=None, **kw):
    """Allocates outputs and a workspace, then runs ms_random_walk."""
    desc = walk_desc(n_photons, **kw)
    out = alloc_walk_outputs(n_photons, desc.mode, device)
    ws = torch.empty(ms_random_walk_workspace_size(desc), dtype=torch.uint8, device=device)
    ms_random_walk(desc, out, ws, stream)
    return out


# ---------------------------------------------------------------- CVAE
STANDARD_SHAPES = {
    0: dict(model=0, p_in=2, p_out=1, latent=4, width=16, n_linear=3),
    1: dict(model=1, p_in=3, p_out=3, latent=4, width=16, n_linear=3),
    2: dict(model=2, p_in=7, p_out=6, latent=4, width=16, n_linear=3),
}


def cvae_shape(shape):
    if isinstance(shape, _abi.CvaeShape):
        return shape
    if isinstance(shape, int):
        shape = STANDARD_SHAPES[shape]
    return _abi.CvaeShape(shape["model"], shape["p_in"], shape["p_out"], shape["latent"], shape["width"],
                          shape["n_linear"])


def cvae_param_count(shape):
    n = C.c_size_t()
    check(lib().cvae_param_count(C.byref(cvae_shape(shape)), C.byref(n)))
    return n.value


def cvae_init(shape, seed, master, stream=None):
    check(lib().cvae_init(C.byref(cvae_shape(shape)), seed, _ptr(master), _stream(stream)))


def cvae_features(model, n, walk, seed, id_offset, stats, cond, target, rows=None, stream=None):
    n_records = walk["n_scatter"].numel()
    check(lib().cvae_features(model, n, _ptr(rows), n_records, _ptr(walk["params"]), _ptr(walk["n_scatter"]),
                              _ptr(walk.get("exit_param")), _ptr(walk.get("event_pos")), _ptr(walk.get("event_dir")),
                              seed, id_offset, _ptr(stats), _ptr(cond), _ptr(target), _stream(stream)))


def ms_select_rows_workspace_size(n):
    b = C.c_size_t()
    check(lib().ms_select_rows_workspace_size(n, C.byref(b)))
    return b.value


def ms_select_rows(n, n_scatter, event_index, min_scatter, min_event, rows, count, workspace, stream=None):
    check(lib().ms_select_rows(n, _ptr(n_scatter), _ptr(event_index), min_scatter, min_event, _ptr(rows), _ptr(count),
                               _ptr(workspace), workspace.numel(), _stream(stream)))


def select_rows(walk, min_scatter, min_event=0):
    """Indices (int64 device tensor) of walk records with N >= min_scatter and k >= min_event."""
    n = walk["n_scatter"].numel()
    rows = torch.empty(n, dtype=torch.int64, device=walk["n_scatter"].device)
    count = torch.zeros(1, dtype=torch.int64, device=rows.device)
    ws = torch.empty(ms_select_rows_workspace_size(n), dtype=torch.uint8, device=rows.device)
    ms_select_rows(n, walk["n_scatter"], walk.get("event_index") if min_event > 0 else None, min_scatter, min_event,
                   rows, count, ws)
    return rows[: int(count.item())]


def ms_column_moments_workspace_size(n, dim):
    b = C.c_size_t()
    check(lib().ms_column_moments_workspace_size(n, dim, C.byref(b)))
    return b.value


def ms_column_moments(x, n, dim, out, workspace, stream=None):
    check(lib().ms_column_moments(_ptr(x), n, dim, _ptr(out), _ptr(workspace), workspace.numel(), _stream(stream)))


def cvae_workspace_size(shape, batch):
    b = C.c_size_t()
    check(lib().cvae_workspace_size(C.byref(cvae_shape(shape)), batch, C.byref(b)))
    return b.value


def adam_params(step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    return _abi.Adam(lr, beta1, beta2, eps, weight_decay, step)


def cvae_train_step(shape, master, adam_m, adam_v, adam, cond, target, n_rows, batch, sample_rows, seed, step,
                    id_offset, workspace, loss=None, grad=None, stream=None, kl_weight=1.0):
    check(lib().cvae_train_step(C.byref(cvae_shape(shape)), _ptr(master), _ptr(adam_m), _ptr(adam_v),
                                None if adam is None else C.byref(adam), _ptr(cond), _ptr(target), n_rows, batch,
                                sample_rows, seed, step, id_offset, kl_weight, _ptr(workspace), workspace.numel(),
                                _ptr(loss), _ptr(grad), _stream(stream)))


def cvae_train_step_noalloc(shape, master, adam_m, adam_v, adam, cond, target, n_rows, batch, sample_rows, seed,
                            step, id_offset, loss=None, grad=None, stream=None, kl_weight=1.0):
    check(lib().cvae_train_step_noalloc(C.byref(cvae_shape(shape)), _ptr(master), _ptr(adam_m), _ptr(adam_v),
                                        None if adam is None else C.byref(adam), _ptr(cond), _ptr(target), n_rows,
                                        batch, sample_rows, seed, step, id_offset, kl_weight, _ptr(loss), _ptr(grad),
                                        _stream(stream)))


TRAINING_STATE_FORMAT = "msst-cvae-training-state-1"


def save_training_state(path, shape, master, adam_m, adam_v, step, stats=None, extra=None):
    """Writes one CVAE's training state to a safetensors file: the FP32 master
    weights, AdamW's first and second moments, the number of steps taken and
    optionally the FP64 standardisation constants [64] and a JSON-able dict
    `extra` (the training seed, schedule, ...).  The training step draws its
    rows and noise from counter-based streams keyed by (seed, step) and
    reduces its gradient in a fixed order, so continuing from the loaded
    state with the next step number reproduces an uninterrupted run bit for
    bit."""
    from safetensors.torch import save_file
    sh = cvae_shape(shape)
    n = cvae_param_count(sh)
    tensors = {}
    for name, t in (("master", master), ("adam_m", adam_m), ("adam_v", adam_v)):
        if t.dtype != torch.float32 or t.numel() != n:
            raise ValueError(f"{name}: expected {n} float32 values, got {t.numel()} {t.dtype}")
        tensors[name] = t.detach().reshape(-1).cpu().contiguous()
    if stats is not None:
        if stats.dtype != torch.float64 or stats.numel() != 64:
            raise ValueError("stats: expected 64 float64 standardisation constants")
        tensors["stats"] = stats.detach().reshape(-1).cpu().contiguous()
    if int(step) < 0:
        raise ValueError("step must be >= 0")
    shape_d = {k: int(getattr(sh, k)) for k, _ in _abi.CvaeShape._fields_}
    meta = {"format": TRAINING_STATE_FORMAT, "shape": json.dumps(shape_d), "step": str(int(step)),
            "extra": json.dumps({} if extra is None else extra)}
    save_file(tensors, str(path), metadata=meta)


def load_training_state(path, device="cuda"):
    """Reads a file written by save_training_state; returns dict(shape, master,
    adam_m, adam_v, step, stats (None if not saved), extra) with the tensors
    on `device`.  Raises ValueError for a file of another format or whose
    tensors do not match the stored shape."""
    from safetensors import safe_open
    with safe_open(str(path), framework="pt") as f:
        meta = f.metadata() or {}
        if meta.get("format") != TRAINING_STATE_FORMAT:
            raise ValueError(f"{path}: not a CVAE training state ({meta.get('format')!r})")
        shape = json.loads(meta["shape"])
        keys = set(f.keys())
        t = {k: f.get_tensor(k) for k in keys}
    n = cvae_param_count(shape)
    for name in ("master", "adam_m", "adam_v"):
        if name not in t or t[name].dtype != torch.float32 or t[name].numel() != n:
            raise ValueError(f"{path}: {name} does not hold {n} float32 values")
    stats = t.get("stats")
    if stats is not None and (stats.dtype != torch.float64 or stats.numel() != 64):
        raise ValueError(f"{path}: stats does not hold 64 float64 values")
    return dict(shape=shape, master=t["master"].to(device), adam_m=t["adam_m"].to(device),
                adam_v=t["adam_v"].to(device), step=int(meta["step"]),
                stats=None if stats is None else stats.to(device), extra=json.loads(meta.get("extra", "{}")))


def cvae_packed_bytes():
    return lib().cvae_packed_bytes()


def cvae_pack(shape, master, stats, precision, packed, stream=None, calib=None):
    """calib: optional device [n, p_in] raw calibration conditions (FP8
    activation scales)."""
    n_calib = 0 if calib is None else calib.shape[0]
    check(lib().cvae_pack(C.byref(cvae_shape(shape)), _ptr(master), _ptr(stats), precision, _ptr(calib), n_calib,
                          _ptr(packed), packed.numel() * packed.element_size(), _stream(stream)))


def cvae_sample(packed, cond, n, seed, id_offset, out, stream=None):
    check(lib().cvae_sample(_ptr(packed), _ptr(cond), n, seed, id_offset, _ptr(out), _stream(stream)))


# ---------------------------------------------------------------- rendering
def make_scene(prims, grid=None, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), res=0, mesh=None):
    """prims: device float32 tensor [n, 8] (or None with a mesh); grid:
    optional device int16 tensor [res^3]; mesh: (tris [n, 9], nodes, n_nodes)
    from build_mesh (device tensors)."""
    tris, nodes, n_nodes = mesh if mesh is not None else (None, None, 0)
    return _abi.Scene(_ptr(prims), 0 if prims is None else prims.shape[0], _ptr(grid),
                      res if grid is not None else 0, (C.c_float * 3)(*lo), (C.c_float * 3)(*hi), _ptr(tris),
                      0 if tris is None else tris.shape[0], _ptr(nodes), n_nodes)


def build_mesh(tris, device="cuda"):
    """BVH of a closed triangle mesh ([n, 9] float32 vertex triples) built on
    the host by ms_build_mesh_bvh; returns (reordered triangles, nodes,
    n_nodes) on the device."""
    import numpy as np
    t = np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 9)
    n = t.shape[0]
    nb = C.c_size_t()
    check(lib().ms_mesh_bvh_size(n, C.byref(nb)))
    nodes = np.zeros(nb.value, np.uint8)
    tsorted = np.zeros_like(t)
    nn = C.c_int32()
    check(lib().ms_build_mesh_bvh(t.ctypes.data, n, nodes.ctypes.data, nb.value, tsorted.ctypes.data, C.byref(nn)))
    return (torch.as_tensor(tsorted).to(device).contiguous(),
            torch.as_tensor(nodes[: nn.value * 32]).to(device).contiguous(), nn.value)


def make_camera(cam):
    return _abi.Camera((C.c_float * 3)(*cam["eye"]), (C.c_float * 3)(*cam["look_at"]), (C.c_float * 3)(*cam["up"]),
                       cam["vfov_deg"], cam["width"], cam["height"])


def make_light(light):
    return _abi.Light((C.c_float * 3)(*light["pos"]), light["intensity"])


def make_medium(med):
    return _abi.Medium(med["sigma_t"], med["g"], med["albedo"])


def render_desc(method, sampler=_abi.SAMPLER_CVAE, packed=(None, None, None), tau_min=0.1, st_max=200.0, spp=1,
                chunk=0, seed=0, sample_offset=0, max_events=1 << 20, blocks_per_cu=0, cvae_batch_min=0,
                nee_samples=1, flags=0, restart_min=0, max_wait=0, min_chain=0.0, nee_chain=0):
    ptrs = (C.c_void_p * 3)(*[None if p is None else p.data_ptr() for p in packed])
    return _abi.RenderDesc(method, sampler, ptrs, tau_min, st_max, spp, chunk, seed, sample_offset, max_events,
                           blocks_per_cu, cvae_batch_min, restart_min, max_wait, nee_samples, flags, min_chain,
                           nee_chain)


IMAGE_FIELDS = ("sum", "comp", "sumsq", "events", "steps", "counters")


def ms_build_sdf_grid(scene, res, grid, stream=None):
    check(lib().ms_build_sdf_grid(C.byref(scene), res, _ptr(grid), _stream(stream)))


def build_sdf_grid(prims, res, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), device="cuda", tris=None):
    """FP16 conservative distance grid (int16 device tensor of binary16 bits)
    of primitives, or of a closed triangle mesh (tris [n, 9])."""
    grid = torch.empty(res ** 3, dtype=torch.int16, device=device)
    if tris is not None:
        t = torch.as_tensor(tris, dtype=torch.float32).reshape(-1, 9).to(device).contiguous()
        ms_build_sdf_grid(make_scene(None, None, lo, hi, mesh=(t, None, 0)), res, grid)
        torch.cuda.synchronize()
        return grid
    prims = torch.as_tensor(prims, dtype=torch.float32).reshape(-1, 8).to(device).contiguous()
    ms_build_sdf_grid(make_scene(prims, None, lo, hi), res, grid)
    return grid


def sphere_trace_render_workspace_size(cam, desc):
    b = C.c_size_t()
    check(lib().sphere_trace_render_workspace_size(C.byref(cam), C.byref(desc), C.byref(b)))
    return b.value


def sphere_trace_render(scene, cam, light, medium, desc, out, workspace, stream=None):
    img = _abi.ImageOut(*[_ptr(out.get(k)) for k in IMAGE_FIELDS])
    check(lib().sphere_trace_render(C.byref(scene), C.byref(cam), C.byref(light), C.byref(medium), C.byref(desc),
                                    C.byref(img), _ptr(workspace), workspace.numel(), _stream(stream)))


def alloc_image(width, height, device="cuda"):
    n = width * height
    f = dict(device=device)
    return {"sum": torch.zeros(n, dtype=torch.float32, **f), "comp": torch.zeros(n, dtype=torch.float32, **f),
            "sumsq": torch.zeros(n, dtype=torch.float32, **f), "events": torch.zeros(n, dtype=torch.int32, **f),
            "steps": torch.zeros(n, dtype=torch.int32, **f), "counters": torch.zeros(4, dtype=torch.int64, **f)}


def ms_image_stats_workspace_size(n_pixels):
    b = C.c_size_t()
    check(lib().ms_image_stats_workspace_size(n_pixels, C.byref(b)))
    return b.value


def ms_image_stats(sum_, comp, sumsq, ref, n_pixels, spp, out, workspace, stream=None):
    check(lib().ms_image_stats(_ptr(sum_), _ptr(comp), _ptr(sumsq), _ptr(ref), n_pixels, spp, _ptr(out),
                               _ptr(workspace), workspace.numel(), _stream(stream)))


# ---------------------------------------------------------------- allocation helpers
class Renderer:
    """Holds a scene on the device and renders images through sphere_trace_render."""

    def __init__(self, prims, camera, light, grid=None, grid_lo=(-1, -1, -1), grid_hi=(1, 1, 1), device="cuda",
                 tris=None):
        self.prims = None if prims is None else torch.as_tensor(prims, dtype=torch.float32).reshape(-1, 8).to(
            device).contiguous()
        self.grid = None if grid is None else torch.as_tensor(grid).to(device).contiguous()
        res = 0 if grid is None else round(self.grid.numel() ** (1 / 3))
        self.mesh = None if tris is None else build_mesh(tris, device)
        self.scene = make_scene(self.prims, self.grid, grid_lo, grid_hi, res, mesh=self.mesh)
        self.camera = camera
        self.cam = make_camera(camera)
        self.light = make_light(light)
        self.device = device
        self._ws = None

    def workspace(self, desc):
        need = sphere_trace_render_workspace_size(self.cam, desc)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def render(self, medium, method, out=None, stream=None, **kw):
        desc = render_desc(method, **kw)
        if out is None:
            out = alloc_image(self.camera["width"], self.camera["height"], self.device)
        sphere_trace_render(self.scene, self.cam, self.light, make_medium(medium), desc, out, self.workspace(desc),
                            stream)
        return out

    def render_rgb(self, media, method, seed=0, stream=None, **kw):
        """RGB media: one medium (sigma_t, g, albedo) per colour channel.  Each
        channel is traced with its own coefficients and Philox key seed + c,
        so the three channels are independent estimates; the learned models
        are shared (their conditions carry sigma_t r and the albedo).
        Returns per-channel image planes stacked on a leading axis of 3."""
        if len(media) != 3:
            raise ValueError("render_rgb needs three media (R, G, B)")
        planes = [self.render(media[c], method, seed=seed + c, stream=stream, **kw) for c in range(3)]
        return {k: torch.stack([p[k] for p in planes]) for k in planes[0]}


def column_moments(x):
    """FP64 column mean / std of a [n, dim] device float32 tensor as a [64] stats half."""
    n, dim = x.shape
    out = torch.zeros(32, dtype=torch.float64, device=x.device)
    ws = torch.empty(ms_column_moments_workspace_size(n, dim), dtype=torch.uint8, device=x.device)
    ms_column_moments(x, n, dim, out, ws)
    return out


def make_stats(cond, target):
    """Standardisation constants [mean_c, std_c, mean_y, std_y] (16 each) on the device."""
    mc, my = column_moments(cond), column_moments(target)
    st = torch.zeros(64, dtype=torch.float64, device=cond.device)
    st[16:32] = 1.0
    st[48:64] = 1.0
    st[: cond.shape[1]] = mc[: cond.shape[1]]
    st[16:16 + cond.shape[1]] = mc[16:16 + cond.shape[1]]
    st[32:32 + target.shape[1]] = my[: target.shape[1]]
    st[48:48 + target.shape[1]] = my[16:16 + target.shape[1]]
    return st
