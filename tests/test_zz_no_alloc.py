"""cvae_train_step_noalloc (the training step that allocates nothing; its
partials live in the library's static device scratch) against
cvae_train_step with a caller workspace: the same kernels on the same
inputs, so weights, AdamW moments, loss and gradient must agree bitwise --
on two calls in a row, the second with a smaller batch and another model,
which reuses the scratch the first call left behind."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import announce

pytestmark = pytest.mark.gpu


def _state(msst, oracle, model, seed):
    shape = W.SHAPE_LIST[model]
    master = torch.as_tensor(oracle.cvae_init(shape, seed).astype(np.float32)).cuda()
    n = master.numel()
    return dict(shape=model, master=master, m=torch.zeros(n, device="cuda"), v=torch.zeros(n, device="cuda"),
                loss=torch.zeros(3, dtype=torch.float64, device="cuda"), grad=torch.zeros(n, device="cuda"))


def _copy(st):
    return {k: (v.clone() if torch.is_tensor(v) else v) for k, v in st.items()}


def test_noalloc_step_matches_workspace_step(msst, oracle):
    rng = np.random.default_rng(11)
    # (model, batch, rows): the second call is smaller than the first
    calls = [(2, 4096, 20000), (0, 1024, 3000)]
    for i, (model, batch, n_rows) in enumerate(calls):
        announce(f"noalloc train step call {i}: model={model} batch={batch} rows={n_rows}")
        p_in, p_out = [(2, 1), (3, 3), (7, 6)][model]
        cond = torch.as_tensor(rng.normal(size=(n_rows, p_in)).astype(np.float32)).cuda()
        target = torch.as_tensor(rng.normal(size=(n_rows, p_out)).astype(np.float32)).cuda()
        ref = _state(msst, oracle, model, 40 + i)
        new = _copy(ref)
        ws = torch.empty(msst.cvae_workspace_size(model, batch), dtype=torch.uint8, device="cuda")
        for step in (1, 2, 3):
            adam = msst.adam_params(step, lr=1e-3)
            msst.cvae_train_step(model, ref["master"], ref["m"], ref["v"], adam, cond, target, n_rows, batch, 1, 7,
                                 step, 0, ws, ref["loss"], ref["grad"], kl_weight=0.5)
            msst.cvae_train_step_noalloc(model, new["master"], new["m"], new["v"], adam, cond, target, n_rows, batch,
                                         1, 7, step, 0, new["loss"], new["grad"], kl_weight=0.5)
            torch.cuda.synchronize()
            for k in ("master", "m", "v", "loss", "grad"):
                a, b = ref[k].cpu().numpy(), new[k].cpu().numpy()
                assert np.array_equal(a, b), (i, step, k, np.abs(a - b).max())
        assert np.isfinite(new["loss"].cpu().numpy()).all()
        del ws
