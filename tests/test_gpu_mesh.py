"""Triangle-mesh bodies on the GPU against the FP64 oracle: the FP16 distance
grid built on the mesh, and path-by-path renders (plain tracing, sphere
tracing with exact in-sphere walks and with BF16 learned steps) through the
stackless BVH."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import announce
from test_gpu_render import CVAE, EXACT, LEARNED_REL, PLAIN, ST, compare_paths, f32_camera, f32_light, f32_medium, \
    models_for_test, pack_all

pytestmark = pytest.mark.gpu

LO, HI = (-1.2, -1.2, -1.2), (1.2, 1.2, 1.2)


@pytest.fixture(scope="module")
def blob():
    return W.mesh_blob(0, 3)


def test_mesh_grid_matches_oracle(msst, oracle, blob):
    announce("mesh sdf grid")
    res = 32
    g = msst.build_sdf_grid(None, res, LO, HI, tris=blob).cpu().numpy().view(np.uint16)
    o = oracle.Scene(None, tris=blob).build_grid(res, LO, HI)
    diff = np.abs(g.astype(np.int64) - o.astype(np.int64))
    gv, ov = g.view(np.float16).astype(np.float64), o.view(np.float16).astype(np.float64)
    print(f"exact {(diff == 0).mean():.5f}, max diff {diff.max()}, inside {(ov < 0).mean():.3f}")
    assert (diff == 0).mean() > 0.999 and diff.max() <= 1
    assert np.all(np.sign(gv) * np.sign(ov) >= 0)


@pytest.mark.parametrize("method,sampler", [(PLAIN, CVAE), (ST, EXACT), (ST, CVAE)])
def test_mesh_render_path_by_path(msst, oracle, blob, method, sampler):
    announce(f"mesh render method={method} sampler={sampler}")
    res = 64
    grid_g = msst.build_sdf_grid(None, res, LO, HI, tris=blob)
    grid_o = oracle.Scene(None, tris=blob).build_grid(res, LO, HI)
    cam, light = f32_camera(W.camera_mesh(40, 40)), f32_light(W.light_c4())
    med = f32_medium(W.medium_c4(20.0))
    opts = dict(spp=1, seed=31)
    kw_o = dict(method=oracle.METHOD_PLAIN_NEE if method == PLAIN else oracle.METHOD_ST)
    packed = (None, None, None)
    if method == ST:
        opts["tau_min"] = 2.0
        kw_o["sampler"] = oracle.SAMPLER_EXACT_WALK if sampler == EXACT else oracle.SAMPLER_CVAE
        if sampler == CVAE:
            models, src = models_for_test(oracle)
            packed = pack_all(msst, src, 1)
            opts.update(nee_samples=2, flags=1)
            kw_o.update(models=models, precision=oracle.PREC_BF16)
    r = msst.Renderer(None, cam, light, grid=grid_g, grid_lo=LO, grid_hi=HI, tris=blob)
    out = r.render(med, method=method, sampler=sampler, packed=packed, **opts)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    o = oracle.render(oracle.Scene(None, sdf_fp16=grid_o, lo=LO, hi=HI, tris=blob), cam, light, med, **kw_o, **opts)
    frac, _ = compare_paths(g, o, rel=LEARNED_REL)
    print(f"diverged {frac:.2e}; lit {(o['sum'] > 0).mean():.2f}, events {o['events'].sum()}, steps {o['steps'].sum()}")
    assert (o["sum"] > 0).mean() > 0.1
    assert frac < 2e-3
    if method == ST:
        assert o["steps"].sum() > 50
