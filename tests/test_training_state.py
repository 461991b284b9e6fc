"""Save and load of a CVAE's training state (master weights, AdamW moments,
step, standardisation constants): host-side file format and its checks.
The resume-equals-uninterrupted check runs on the GPU in test_gpu_cvae."""
import json

import numpy as np
import pytest
import torch


@pytest.fixture(scope="module")
def M():
    import paper_2011_03082_amd as M
    M.lib()
    return M


def _state(M, model, seed=0):
    rng = np.random.default_rng(seed)
    n = M.cvae_param_count(model)
    t = lambda: torch.as_tensor(rng.normal(size=n).astype(np.float32))  # noqa: E731
    stats = torch.as_tensor(rng.normal(size=64))
    return t(), t(), t().abs(), stats


@pytest.mark.parametrize("model", [0, 1, 2])
def test_round_trip_is_bitwise(M, tmp_path, model):
    master, m, v, stats = _state(M, model, model)
    path = tmp_path / f"m{model}.safetensors"
    M.save_training_state(path, model, master, m, v, 1234, stats=stats, extra={"seed": 7, "lr": [2e-3, 6e-4]})
    st = M.load_training_state(path, device="cpu")
    assert st["shape"] == M.STANDARD_SHAPES[model]
    assert st["step"] == 1234 and st["extra"] == {"seed": 7, "lr": [2e-3, 6e-4]}
    for k, ref in (("master", master), ("adam_m", m), ("adam_v", v), ("stats", stats)):
        assert st[k].dtype == ref.dtype and torch.equal(st[k].view(torch.int8), ref.view(torch.int8)), k


def test_round_trip_of_a_table1_shape_without_stats(M, tmp_path):
    shape = dict(model=2, p_in=7, p_out=6, latent=9, width=20, n_linear=3)
    n = M.cvae_param_count(shape)
    master = torch.arange(n, dtype=torch.float32) * 0.5
    path = tmp_path / "t1.safetensors"
    M.save_training_state(path, shape, master, torch.zeros(n), torch.ones(n), 0)
    st = M.load_training_state(path, device="cpu")
    assert st["shape"] == shape and st["stats"] is None and st["step"] == 0 and st["extra"] == {}
    assert torch.equal(st["master"], master) and torch.equal(st["adam_v"], torch.ones(n))


def test_rejects_mismatched_tensors(M, tmp_path):
    master, m, v, stats = _state(M, 0)
    p = tmp_path / "x.safetensors"
    with pytest.raises(ValueError, match="adam_m"):
        M.save_training_state(p, 0, master, m[:-1], v, 1)
    with pytest.raises(ValueError, match="master"):
        M.save_training_state(p, 0, master.double(), m, v, 1)
    with pytest.raises(ValueError, match="stats"):
        M.save_training_state(p, 0, master, m, v, 1, stats=stats.float())
    with pytest.raises(ValueError, match="step"):
        M.save_training_state(p, 0, master, m, v, -1)
    # a state saved for one shape does not load as another's
    M.save_training_state(p, 0, master, m, v, 3)
    from safetensors import safe_open
    from safetensors.torch import save_file
    with safe_open(str(p), framework="pt") as f:
        meta, t = f.metadata(), {k: f.get_tensor(k) for k in f.keys()}
    meta["shape"] = json.dumps(M.STANDARD_SHAPES[0] | {"width": 20})
    save_file(t, str(tmp_path / "y.safetensors"), metadata=meta)
    with pytest.raises(ValueError, match="master"):
        M.load_training_state(tmp_path / "y.safetensors", device="cpu")


def test_rejects_a_foreign_file(M, tmp_path):
    from safetensors.torch import save_file
    save_file({"master": torch.zeros(4)}, str(tmp_path / "f.safetensors"))
    with pytest.raises(ValueError, match="not a CVAE training state"):
        M.load_training_state(tmp_path / "f.safetensors", device="cpu")
