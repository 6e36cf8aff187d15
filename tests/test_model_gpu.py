"""The model object through the C ABI: save / load round trip with identical
logits and refined results, one-call training steps equal to the separate
gradient + Adam calls, and the grid check."""
import os

import numpy as np
import pytest

import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import learn, synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctx():
    c = ssg.Context(0)
    yield c
    c.close()


def _trained_params():
    return np.load(os.path.join(HERE, "paper_2111_07396_amd", "weights", "encoder_c5.npy"),
                   allow_pickle=False).astype(np.float32)


def test_model_save_load_gives_identical_logits(ctx, tmp_path):
    import torch
    cat, grid = synth.catalog_mixed(n_obj=300)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    model = ssg.Model.create(ctx, grid, _trained_params())
    path = str(tmp_path / "enc.ssm")
    model.save(path)
    loaded = ssg.Model.load(ctx, path)
    g, step, _ = loaded.info()
    assert g == tuple(grid) and step == 0
    p0, p1 = model.params(), loaded.params()
    torch.cuda.synchronize()
    assert torch.equal(p0, p1)
    _, l0, _ = ctx.enc_forward(dc, grid, p0)
    _, l1, _ = ctx.enc_forward(dc, grid, p1)
    torch.cuda.synchronize()
    assert torch.equal(l0.view(torch.int32), l1.view(torch.int32))
    r0 = model.best_period(ctx, ssg.SS_METHOD_SS, dc, grid, gamma=1.0, top_k=16, margin=0,
                           full_below=80)
    r1 = loaded.best_period(ctx, ssg.SS_METHOD_SS, dc, grid, gamma=1.0, top_k=16, margin=0,
                            full_below=80)
    torch.cuda.synchronize()
    assert torch.equal(r0[0], r1[0]) and torch.equal(r0[2], r1[2])
    with pytest.raises(ssg.SSError):
        model.best_period(ctx, ssg.SS_METHOD_SS, dc, (grid[0], grid[1], grid[2] + 1), gamma=1.0)
    model.close()
    loaded.close()


def test_train_step_equals_gradient_plus_adam(ctx, tmp_path):
    import torch
    cat, grid = synth.catalog_mixed(n_obj=256)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    rng = np.random.default_rng(3)
    lab = torch.tensor(rng.integers(0, ssg.ENC_BINS, cat.n_obj), dtype=torch.int32,
                       device="cuda")
    p0 = learn.init_params(5).astype(np.float32)
    model = ssg.Model.create(ctx, grid, p0)
    p = torch.tensor(p0, device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    for step in range(1, 4):
        b = learn.view(dc, 64 * (step - 1), 64 * step + 40)
        lb = lab[64 * (step - 1):64 * step + 40]
        loss_m = model.train_step(ctx, b, lb, 2e-3)
        g, loss_r, _ = ctx.enc_train_grad(b, grid, p, lb)
        ssg.adam_step(p, g, m, v, step, 2e-3)
        torch.cuda.synchronize()
        assert torch.equal(loss_m, loss_r)
        assert torch.equal(model.params(), p)
    assert model.info()[1] == 3
    # the optimizer state survives a save / load: the next step is the same
    path = str(tmp_path / "mid.ssm")
    model.save(path)
    again = ssg.Model.load(ctx, path)
    b = learn.view(dc, 0, 128)
    model.train_step(ctx, b, lab[:128], 2e-3)
    again.train_step(ctx, b, lab[:128], 2e-3)
    torch.cuda.synchronize()
    assert torch.equal(model.params(), again.params())
    model.close()
    again.close()
