"""C-ABI contract of the renderer, the CVAE size queries and the mesh BVH on
the CPU: invalid descriptors are refused with MS_ERR_INVALID_ARGUMENT (or
WORKSPACE_TOO_SMALL) and a message, before anything touches a device.  Device
pointers here are placeholders that validation never dereferences."""
import ctypes as C

import numpy as np
import pytest

FAKE = 0x10000  # a 16-byte aligned placeholder address


@pytest.fixture(scope="module")
def M():
    import paper_2011_03082_amd as M
    M.lib()
    return M


def scene(M, **kw):
    s = M._abi.Scene()
    s.prims, s.n_prims = FAKE, 2
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def camera(M, **kw):
    c = M._abi.Camera((C.c_float * 3)(0, 0, 4), (C.c_float * 3)(0, 0, 0), (C.c_float * 3)(0, 1, 0), 40.0, 16, 16)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def status(M, sc=None, cam=None, med=None, desc=None, img=None, ws=FAKE, ws_bytes=1 << 30):
    sc = sc or scene(M)
    cam = cam or camera(M)
    light = M._abi.Light((C.c_float * 3)(2, 2, 2), 10.0)
    med = med or M._abi.Medium(10.0, 0.8, 0.99)
    desc = desc or M.render_desc(1, spp=4)
    if img is None:
        img = M._abi.ImageOut(FAKE, FAKE, FAKE, FAKE, FAKE, None)
    return M.lib().sphere_trace_render(C.byref(sc), C.byref(cam), C.byref(light), C.byref(med), C.byref(desc),
                                       C.byref(img), C.c_void_p(ws) if ws else None, ws_bytes, None)


def desc_with(M, **kw):
    base = dict(spp=4)
    base.update(kw)
    method = base.pop("method", 1)
    return M.render_desc(method, **base)


@pytest.mark.parametrize("case", [
    "method", "sampler", "spp0", "spp_big", "nee17", "flags", "tau", "tau0", "st_max", "restart", "batch", "bpc",
    "cvae_no_models",
])
def test_render_rejects_invalid_descriptor(M, case):
    d = {
        "method": dict(method=7), "sampler": dict(method=2, sampler=4), "spp0": dict(spp=0),
        "spp_big": dict(spp=(1 << 24) + 1), "nee17": dict(nee_samples=17), "flags": dict(flags=8),
        "tau": dict(tau_min=-1.0), "tau0": dict(tau_min=0.0), "st_max": dict(st_max=0.0), "restart": dict(restart_min=65),
        "batch": dict(cvae_batch_min=65), "bpc": dict(blocks_per_cu=65), "cvae_no_models": dict(method=2, sampler=0),
    }[case]
    assert status(M, desc=desc_with(M, **d)) == M._abi.MS_ERR_INVALID_ARGUMENT
    assert M.lib().ms_last_error().decode().startswith("sphere_trace_render")


@pytest.mark.parametrize("med", [(0.0, 0.8, 0.9), (10.0, 1.0, 0.9), (10.0, -1.0, 0.9), (10.0, 0.5, 0.0),
                                 (10.0, 0.5, 1.5)])
def test_render_rejects_invalid_medium(M, med):
    assert status(M, med=M._abi.Medium(*med)) == M._abi.MS_ERR_INVALID_ARGUMENT


def test_render_rejects_invalid_scene_camera_and_buffers(M):
    inv = M._abi.MS_ERR_INVALID_ARGUMENT
    assert status(M, sc=scene(M, n_prims=0)) == inv
    assert status(M, sc=scene(M, n_prims=257)) == inv
    assert status(M, sc=scene(M, prims=None)) == inv
    # a mesh needs its BVH and its distance grid
    assert status(M, sc=scene(M, n_tris=100, tris=FAKE)) == inv
    assert status(M, sc=scene(M, n_tris=100, tris=FAKE, bvh=FAKE, n_nodes=50)) == inv
    assert status(M, sc=scene(M, sdf_fp16=FAKE, res=0)) == inv
    assert status(M, cam=camera(M, width=0)) == inv
    assert status(M, cam=camera(M, vfov_deg=180.0)) == inv
    assert status(M, img=M._abi.ImageOut(None, FAKE, None, FAKE, FAKE, None)) == inv
    assert status(M, ws=0) == inv
    assert "workspace" in M.lib().ms_last_error().decode()
    assert status(M, ws_bytes=16) == M._abi.MS_ERR_WORKSPACE_TOO_SMALL


@pytest.mark.parametrize("shape", [
    dict(model=0, p_in=2, p_out=1, latent=4, width=33, n_linear=3),
    dict(model=0, p_in=2, p_out=1, latent=4, width=16, n_linear=5),
    dict(model=0, p_in=2, p_out=1, latent=4, width=16, n_linear=1),
    dict(model=2, p_in=7, p_out=6, latent=17, width=16, n_linear=3),
    dict(model=2, p_in=17, p_out=6, latent=4, width=16, n_linear=3),
    dict(model=3, p_in=2, p_out=1, latent=4, width=16, n_linear=3),
])
def test_cvae_rejects_unsupported_shapes(M, shape):
    n = C.c_size_t()
    st = M.lib().cvae_param_count(C.byref(M.cvae_shape(shape)), C.byref(n))
    assert st in (M._abi.MS_ERR_INVALID_ARGUMENT, M._abi.MS_ERR_UNSUPPORTED)
    assert M.lib().ms_last_error().decode()


@pytest.mark.parametrize("shape, stride", [
    (dict(model=2, p_in=7, p_out=6, latent=5, width=16, n_linear=3), 16),
    (dict(model=2, p_in=7, p_out=6, latent=9, width=16, n_linear=3), 32),
    (dict(model=2, p_in=7, p_out=6, latent=5, width=20, n_linear=4), 32),
    (dict(model=1, p_in=3, p_out=3, latent=9, width=8, n_linear=2), 32),
])
def test_cvae_param_count_follows_the_layer_stride(M, oracle, shape, stride):
    """2 n_linear layers of S x S weights and S biases, S = 32 once any
    width of the two networks exceeds 16 (2 x 9 encoder outputs, 20 hidden
    units), on both sides of the shared layout."""
    n = C.c_size_t()
    assert M.lib().cvae_param_count(C.byref(M.cvae_shape(shape)), C.byref(n)) == 0
    assert n.value == 2 * shape["n_linear"] * (stride * stride + stride)
    assert oracle.n_params(shape) == n.value
    assert oracle.layer_stride(shape) == stride


def test_mesh_bvh_rejects_invalid(M):
    L = M.lib()
    nb = C.c_size_t()
    assert L.ms_mesh_bvh_size(0, C.byref(nb)) == M._abi.MS_ERR_INVALID_ARGUMENT
    tris = np.zeros((4, 9), np.float32)
    tris[:, 3] = 1.0
    tris[:, 7] = 1.0
    tris[2, 4] = np.nan
    assert L.ms_mesh_bvh_size(4, C.byref(nb)) == 0
    nodes = np.zeros(nb.value, np.uint8)
    out = np.zeros_like(tris)
    nn = C.c_int32()
    assert L.ms_build_mesh_bvh(tris.ctypes.data, 4, nodes.ctypes.data, nb.value, out.ctypes.data,
                               C.byref(nn)) == M._abi.MS_ERR_INVALID_ARGUMENT
    tris[2, 4] = 0.0
    assert L.ms_build_mesh_bvh(tris.ctypes.data, 4, nodes.ctypes.data, 32, out.ctypes.data,
                               C.byref(nn)) == M._abi.MS_ERR_WORKSPACE_TOO_SMALL
    assert L.ms_build_mesh_bvh(tris.ctypes.data, 4, nodes.ctypes.data, nb.value, out.ctypes.data, C.byref(nn)) == 0
    assert 1 <= nn.value <= 8


def test_render_rejects_negative_min_chain(M):
    assert status(M, desc=desc_with(M, min_chain=-1.0)) == M._abi.MS_ERR_INVALID_ARGUMENT
    assert b"min_chain" in M.lib().ms_last_error()


def test_render_rejects_negative_nee_chain(M):
    assert status(M, desc=desc_with(M, nee_chain=-1)) == M._abi.MS_ERR_INVALID_ARGUMENT
    assert b"nee_chain" in M.lib().ms_last_error()


@pytest.mark.parametrize("w,h,spp", [(512, 512, 256), (256, 256, 256), (1024, 1024, 1024), (2048, 2048, 1024),
                                     (32, 32, 3), (7, 5, 5)])
def test_workspace_follows_the_default_samples_per_unit(M, w, h, spp):
    """The workspace holds one 16-byte record per work unit, the units being
    the pixels times ceil(spp / chunk) at the header's default chunk (the rule
    bench.default_chunk restates), after 256 bytes of counters."""
    import bench
    chunk = bench.default_chunk(w * h, spp)
    n_units = w * h * -(-spp // chunk)
    need = 256 + -(-n_units * 16 // 256) * 256
    assert M.sphere_trace_render_workspace_size(camera(M, width=w, height=h), M.render_desc(1, spp=spp)) == need
