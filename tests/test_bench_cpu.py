"""Host-side pieces of bench.py that run without a GPU: argument defaults,
the refusal of several GPUs, the measured-traffic reader and the image
moments helper."""
import os
import subprocess
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_defaults_match_the_documented_configuration(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.gpus, a.width, a.spp, a.ref_spp) == (1, 512, 256, 4096)
    assert a.tau_min == 10.0 and a.nee_samples == 1 and a.nee_flags == 1 and a.min_chain == 256.0
    assert a.train_samples == 1 << 22 and a.train_steps == 20000


def test_cost_rule_of_the_sphere_box_launches(monkeypatch):
    """The bench's CPU baseline applies the render kernel's cost rule: the
    unit sphere's centre (radius 0.999) bypasses 0.5 (0.999 sigma_t)^2 0.2
    collisions -- under 256 at sigma_t 10, 20 and 40 (160), above at 80 (638);
    under 64 only at 10 and 20."""
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert [bench.c4_tau(s, a) for s in (10.0, 20.0, 40.0, 80.0)] == [1e30, 1e30, 1e30, 10.0]
    a.min_chain = 64.0
    assert [bench.c4_tau(s, a) for s in (10.0, 20.0, 40.0, 80.0)] == [1e30, 1e30, 10.0, 10.0]
    a.min_chain = 0.0
    assert bench.c4_tau(20.0, a) == 10.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_reader_follows_the_kernel_sources():
    d = bench.render_source_digest()
    assert len(d) == 16 and d == bench.render_source_digest()
    t = bench.measured_traffic()
    assert t is None or t > 0


def test_image_moments():
    img = {"sum": torch.tensor([4.0, 2.0]), "comp": torch.tensor([0.0, 1e-7]),
           "sumsq": torch.tensor([8.0, 2.0])}
    mean, var = bench.image_moments(img, 4)
    np.testing.assert_allclose(mean.numpy(), [1.0, (2.0 + 1e-7) / 4], rtol=1e-7)
    assert var.min() >= 0


def test_subset_pixels_and_anchor_statistics():
    """The oracle anchor's pixel subset is the centre of every stride x
    stride block, and its matched-RMSE inputs are taken on those pixels
    only: the plain tracer's variance on the subset, and each image's error
    against the oracle with the oracle's own noise removed."""
    w = h = 32
    for stride in (8, 16):
        pix = bench.subset_pixels(w, h, stride)
        assert pix.size == (w // stride) * (h // stride)
        assert set((pix % w).tolist()) == set(range(stride // 2, w, stride))
        assert set((pix // w).tolist()) == set(range(stride // 2, h, stride))
    rng = np.random.default_rng(0)
    pix = bench.subset_pixels(w, h, 8)
    truth = rng.uniform(0.5, 1.0, w * h)
    n_o, n_r = 4096, 1024
    sub = dict(pix=pix, mean=truth[pix], var=np.full(pix.size, 0.04), spp=n_o, seconds=0.0)
    ref_var = np.full(w * h, 0.09)
    pt_var = np.where(np.arange(w * h) % 2 == 0, 1.0, 3.0)
    img = truth + 0.1  # an image off by 0.1 everywhere
    a = bench.anchor_stats(sub, truth, ref_var, n_r, {"x": img}, pt_var)
    # the subset's pixels are all even (centres at 4, 12, ...): variance 1, not the image mean 2
    assert a["pt_var_subset"] == 1.0
    np.testing.assert_allclose(a["rmse_x_vs_oracle"], np.sqrt(0.01 - 0.04 / n_o), rtol=1e-12)
    np.testing.assert_allclose(a["rmse_x_vs_reference_on_subset"], np.sqrt(0.01 - 0.09 / n_r), rtol=1e-12)
    assert a["pixels"] == pix.size and a["lit_pixels"] == pix.size
    assert a["z_rms"] == 0.0 and a["z_global"] == 0.0
    # a pixel whose variances are negligible (squares flushed to zero) but
    # whose means differ is left out of the z-test instead of dominating it
    ref2 = truth.copy()
    ref2[pix[0]] += 1e-20
    ref_var2 = ref_var.copy()
    ref_var2[pix[0]] = 0.0
    sub2 = dict(sub, var=sub["var"].copy())
    sub2["var"][0] = 1e-60
    a2 = bench.anchor_stats(sub2, ref2, ref_var2, n_r, {"x": img}, pt_var)
    assert a2["lit_pixels"] == pix.size - 1 and a2["z_max"] < 1.0


def test_default_samples_per_unit():
    """The header's rule for ms_render_desc.chunk = 0 at the shapes rendered:
    about 2^23 units of at most 64 samples, longer where that would leave more
    than 2^24 units, at least 2."""
    assert bench.default_chunk(512 * 512, 256) == 8
    assert bench.default_chunk(256 * 256, 256) == 2
    assert bench.default_chunk(1024 * 1024, 1024) == 64
    assert bench.default_chunk(2048 * 2048, 1024) == 256
    assert bench.default_chunk(32 * 32, 3) == 2
    assert bench.default_chunk(7, 1) == 1


def _project(cam, p):
    """Pixel index (row-major) whose centre ray is nearest to world point p."""
    eye = np.asarray(cam["eye"], float)
    f = np.asarray(cam["look_at"], float) - eye
    f /= np.linalg.norm(f)
    rt = np.cross(f, cam["up"])
    rt /= np.linalg.norm(rt)
    uv = np.cross(rt, f)
    th = np.tan(np.radians(cam["vfov_deg"]) / 2)
    w, h = cam["width"], cam["height"]
    v = np.asarray(p, float) - eye
    sx = (v @ rt) / (v @ f) / (th * w / h)
    sy = (v @ uv) / (v @ f) / th
    px, py = int((sx + 1) / 2 * w), int((1 - sy) / 2 * h)
    return py * w + px


def test_primary_hit_labels_of_a_lone_sphere_cover_its_silhouette():
    """The silhouette of a sphere of radius r seen from distance D subtends
    a half-angle asin(r / D): a disc of radius tan(asin(r / D)) / tan(vfov / 2)
    half-widths around the image centre."""
    import workloads as W
    w = 400
    cam = dict(eye=(0.0, 0.0, 5.0), look_at=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=30.0, width=w, height=w)
    lab = bench.primary_hit_labels(cam, W.scene_sphere(1.0))
    rad = np.tan(np.arcsin(1.0 / 5.0)) / np.tan(np.radians(15.0)) * (w / 2)
    assert set(np.unique(lab)) == {0, 1}
    assert abs((lab == 1).sum() / (np.pi * rad**2) - 1.0) < 0.01
    # a wider image of the same view keeps the pixel aspect (the disc stays round)
    cam2 = dict(cam, width=2 * w)
    lab2 = bench.primary_hit_labels(cam2, W.scene_sphere(1.0)).reshape(w, 2 * w)
    rows, cols = np.nonzero(lab2 == 1)
    assert abs((cols.max() - cols.min()) / (rows.max() - rows.min()) - 1.0) < 0.02


def test_primary_hit_labels_split_the_sphere_box_scene():
    import workloads as W
    cam = W.camera_c4(256, 256)
    lab = bench.primary_hit_labels(cam, W.scene_c4())
    # the arm's free end lies outside the sphere: its pixels see the box first
    assert lab[_project(cam, (1.9, 0.0, 0.4))] == 2
    assert lab[_project(cam, (1.6, 0.3, 0.4))] == 2
    # the front of the sphere is nearer than the box buried in it
    assert lab[_project(cam, (0.0, 0.0, 1.0))] == 1
    assert lab[_project(cam, (-0.6, 0.5, 0.6))] == 1
    # the corners of the view miss the body
    assert lab[0] == 0 and lab[-1] == 0
    n1, n2 = (lab == 1).sum(), (lab == 2).sum()
    assert n1 > 2 * n2 > 0


def test_region_counts_average_per_pixel_means():
    labels = np.array([0, 1, 1, 2, 2, 2])
    img = {"events": torch.tensor([9, 4, 8, 2, 2, 20], dtype=torch.int32),
           "steps": torch.tensor([0, 2, 0, 0, 2, 0], dtype=torch.int32)}
    r = bench.region_counts(img, labels, 2, {1: "sphere", 2: "box_arm", 3: "absent"})
    assert set(r) == {"sphere", "box_arm"}
    assert r["sphere"]["pixels"] == 2 and r["sphere"]["events_per_path"] == 3.0 and r["sphere"]["steps_per_path"] == 0.5
    assert r["box_arm"]["events_per_path"] == 4.0 and r["box_arm"]["events_max"] == 10.0
