"""The training step that allocates nothing (dolinc_mlp_train_step_static)
against dolinc_mlp_train_step, through the C ABI: two steps in a row, the
second on a smaller (ragged) batch, parameters and losses equal bit for bit
(the same partial grid in a different buffer); no device memory taken by
the calls; sizes beyond the maximum and calls before the parameters are set
are refused."""
import numpy as np
import pytest

from oracle import indicator as OI
from synth import mesh as M

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    Xh = OI.bf16_round(rng.normal(size=(n, 24)).clip(-8, 8)).astype(np.float32)
    Xb = np.zeros((n, 32), dtype=np.uint16)
    Xb[:, :24] = (Xh.view(np.uint32) >> 16).astype(np.uint16)
    X = torch.from_numpy(Xb.view(np.int16)).cuda()
    y = torch.from_numpy(rng.random(n).astype(np.float32)).cuda()
    return X, y


def test_static_training_step_equals_the_allocating_one():
    import torch

    from paper_2404_08952_amd import Solver
    from paper_2404_08952_amd import binding as B
    mesh = M.periodic_3d(4, jitter=0.2, seed=3)
    kw = dict(pde="euler", scheme="USR3", flux="rusanov", blend="learned")
    a = Solver(mesh, **kw)
    b = Solver(mesh, **kw)
    # refused before the parameters are set
    X0, y0 = _batch(64, 0)
    with pytest.raises(B.DolincError) as e:
        b.mlp_train_step_static(X0, y0, 1e-3)
    assert e.value.status == B.ESTATE
    p0 = OI.xavier_init(11).astype(np.float32)
    a.mlp_set(p0)
    b.mlp_set(p0)
    loss_b = torch.zeros(1, dtype=torch.float32, device="cuda")
    for n, seed in ((40000, 1), (7001, 2)):
        X, y = _batch(n, seed)
        la = a.mlp_train_step(X, y, 2e-3)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        b.mlp_train_step_static(X, y, 2e-3, loss_b)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        np.testing.assert_array_equal(b.mlp_get(), a.mlp_get())
        assert la.item() == loss_b.item()
        assert np.isfinite(loss_b.item())
    # a later step moves the parameters (the step is taken, not skipped)
    X, y = _batch(5000, 3)
    before = b.mlp_get()
    b.mlp_train_step_static(X, y, 2e-3)
    assert np.abs(b.mlp_get() - before).max() > 0
    # beyond the maximum batch: refused, nothing enqueued
    Xbig, ybig = _batch(B.MLP_STATIC_MAX_ROWS + 1, 4)
    after = b.mlp_get()
    with pytest.raises(B.DolincError) as e:
        b.mlp_train_step_static(Xbig, ybig, 2e-3)
    assert e.value.status == B.EINVAL
    np.testing.assert_array_equal(b.mlp_get(), after)
    a.close()
    b.close()
