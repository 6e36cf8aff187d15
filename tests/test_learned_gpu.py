"""GPU parity of the learned proposal, through the C ABI.

- Encoder forward (BF16 matrix-core per-point layers, FP32 head) and the
  training gradient, per tensor, in relative Frobenius norm:
  (a) against the FP64 reference with the same operands rounded to BF16:
      <= 2e-3 (what is left is FP32 accumulation order and the FP32
      features, each ~1e-6, plus ReLU gates that flip for pre-activations
      within an FP32 rounding of zero);
  (b) against the plain FP64 definition: <= 2 x the error that the BF16
      operand rounding alone causes (measured by (a)'s reference) + 2e-3.
      BF16 keeps 8 significant bits (2^-9 relative per operand); the first
      layer's weight gradient sums point terms of both signs, so its
      relative error grows with the cancellation (a few percent here).
- Adam against its definition (FP32 vs FP64: 1e-5 relative).
- Refine against the FP64 refine reference on the same seeded logits: best
  index bit-exact (unless the reference's two best powers over the refined
  set differ by less than 1e-4 (1 - P)), power within 1e-4 (1 - P).
"""
import numpy as np
import pytest

import oracle
from oracle import encoder as enc
from oracle import refine as ref
import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu
FROB_EMUL = 2e-3


def _check(gpu, pure, emul, what):
    budget = _frob(emul, pure)
    e_emul, e_pure = _frob(gpu, emul), _frob(gpu, pure)
    assert e_emul <= FROB_EMUL, (what, e_emul)
    assert e_pure <= 2 * budget + FROB_EMUL, (what, e_pure, budget)


@pytest.fixture(scope="module")
def ctx():
    c = ssg.Context(0)
    yield c
    c.close()


def _frob(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _catalog(seed, n_obj, lens=(20, 300)):
    return synth.make_catalog(seed, n_obj, lens, 1000.0, (0.1, 100.0), 0.05)


def _params(seed):
    p = enc.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    parts = enc.unpack(p)
    parts["w1"][enc.ONE_SLOT] = rng.normal(0, 0.3, enc.H1)  # nonzero first-layer bias
    parts["b2"] = rng.normal(0, 0.3, enc.H2)
    parts["b3"] = rng.normal(0, 0.1, enc.BINS)
    return enc.pack(parts)


def _feats(cat, band):
    out = []
    for o in range(cat.n_obj):
        a, b = cat.offsets[o], cat.offsets[o + 1]
        out.append(enc.features(cat.t[a:b], cat.y[a:b], cat.e[a:b], band[0], band[1]))
    return out


def test_encoder_forward_matches_reference(ctx):
    import torch
    cat = _catalog(21, 24)
    grid = (0.05, 20.0, 50000)
    params = _params(1)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    pt = torch.tensor(params, dtype=torch.float32, device="cuda")
    emb, logits, st = ctx.enc_forward(dc, grid, pt)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    feats = _feats(cat, grid)
    ref_logits, (ref_emb, _) = enc.forward(params, feats)
    emu_logits, (emu_emb, _) = enc.forward(params, feats, bf16=True)
    e, lg = emb.cpu().numpy(), logits.cpu().numpy()
    _check(e, ref_emb, emu_emb, "emb")
    _check(lg, ref_logits, emu_logits, "logits")
    # per object, too (lengths 20..300 cover one to ten 32-point tiles)
    for o in range(cat.n_obj):
        _check(e[o], ref_emb[o], emu_emb[o], f"emb[{o}]")


def test_encoder_skips_bad_objects(ctx):
    import torch
    cat = _catalog(22, 6)
    cat.e[cat.offsets[2]] = -1.0  # object 2: bad error bar
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    params = _params(2)
    pt = torch.tensor(params, dtype=torch.float32, device="cuda")
    emb, logits, st = ctx.enc_forward(dc, (0.1, 10.0, 2000), pt)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[2] == ssg.OBJ_BAD_ERR and (np.delete(st, 2) == 0).all()
    assert (emb.cpu().numpy()[2] == 0).all()
    np.testing.assert_allclose(logits.cpu().numpy()[2], enc.unpack(params)["b3"], rtol=1e-6)


def test_training_gradient_matches_reference(ctx):
    import torch
    cat = _catalog(23, 40)
    grid = (0.05, 20.0, 50000)
    params = _params(3)
    labels = np.random.default_rng(5).integers(0, enc.BINS, cat.n_obj)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    pt = torch.tensor(params, dtype=torch.float32, device="cuda")
    lt = torch.tensor(labels, dtype=torch.int32, device="cuda")
    grad, loss, st = ctx.enc_train_grad(dc, grid, pt, lt)
    torch.cuda.synchronize()
    feats = _feats(cat, grid)
    ref_loss, ref_grad = enc.loss_and_grad(params, feats, labels)
    emu_loss, emu_grad = enc.loss_and_grad(params, feats, labels, bf16=True)
    assert abs(loss.item() - emu_loss) <= 1e-4 * abs(emu_loss)
    assert abs(loss.item() - ref_loss) <= 2 * abs(emu_loss - ref_loss) + 1e-4 * abs(ref_loss)
    g = enc.unpack(grad.cpu().numpy().astype(np.float64))
    r, m = enc.unpack(ref_grad), enc.unpack(emu_grad)
    for name, _ in enc.SHAPES:
        _check(g[name], r[name], m[name], name)
    assert (g["w1"][enc.ONE_SLOT + 1:] == 0).all()
    # deterministic: a second call gives the same bits
    grad2, loss2, _ = ctx.enc_train_grad(dc, grid, pt, lt)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2) and torch.equal(loss, loss2)


def test_adam_step_matches_definition():
    import torch
    rng = np.random.default_rng(9)
    n = 1000
    p, g = rng.normal(size=n), rng.normal(size=n)
    m, v = rng.normal(size=n) * 0.1, rng.random(n) * 0.1
    tp, tg, tm, tv = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (p, g, m, v))
    ssg.adam_step(tp, tg, tm, tv, 7, 1e-3)
    torch.cuda.synchronize()
    rp, rm, rv = enc.adam_step(p, g, m, v, 7, 1e-3)
    np.testing.assert_allclose(tm.cpu().numpy(), rm, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(tv.cpu().numpy(), rv, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(tp.cpu().numpy(), rp, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP])
@pytest.mark.parametrize("top_k,margin,full_below", [(16, 1, 0), (3, 0, 0), (40, 2, 0),
                                                     (4, 1, 120)])
def test_refine_matches_reference(ctx, method, top_k, margin, full_below):
    import torch
    cat = synth.make_catalog(31, 12, (40, 260), 1000.0, (0.2, 10.0), 0.05)
    cat.y[cat.offsets[4]:cat.offsets[5]] = 15.0  # object 4: constant magnitudes
    grid = (0.1, 10.0, 3000)
    logits = np.random.default_rng(7).normal(size=(cat.n_obj, ref.BINS)).astype(np.float32)
    logits[1, 100:110] = 5.0  # equal logits: lower bins first
    bi_o, bp_o = ref.refine_best(method, cat.offsets, cat.t, cat.y, cat.e, grid,
                                 logits.astype(np.float64), top_k, margin, full_below=full_below)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    lt = torch.tensor(logits, device="cuda")
    bi, bp, bw, st = ctx.refine_best_period(method, dc, grid, lt, top_k, margin, full_below)
    torch.cuda.synchronize()
    bi, bw, st = bi.cpu().numpy(), bw.cpu().numpy(), st.cpu().numpy()
    assert st[4] == ssg.OBJ_CONST_MAG and bi[4] == -1 and np.isnan(bw[4])
    table = ref.bin_table(*grid)
    for o in range(cat.n_obj):
        if o == 4:
            continue
        if bi_o[o] < 0:  # every selected bin is narrower than the grid step: nothing to search
            assert bi[o] == -1 and np.isnan(bw[o]), o
            continue
        if bi[o] != bi_o[o]:
            ks = ref.refine_set(logits[o].astype(np.float64), top_k, margin, table)
            if cat.offsets[o + 1] - cat.offsets[o] < full_below:
                ks = np.arange(grid[2])
            a, b = cat.offsets[o], cat.offsets[o + 1]
            pg, _ = oracle.periodogram(method, np.array([0, b - a]), cat.t[a:b], cat.y[a:b],
                                       cat.e[a:b], *grid, ks=ks)
            top = np.sort(pg[0])[::-1]
            assert top[0] - top[1] < 1e-4 * (1 - top[0]), (o, bi[o], bi_o[o])
        assert abs(bw[o] - bp_o[o]) <= 1e-4 * (1 - bp_o[o]) + 1e-12


def test_refine_everything_equals_full_grid(ctx):
    """top_k = 1024 selects the whole grid: the refine result is the full one."""
    import torch
    cat = synth.make_catalog(32, 20, (30, 400), 1000.0, (0.2, 10.0), 0.05)
    grid = (0.1, 10.0, 2500)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    lt = torch.zeros((cat.n_obj, ref.BINS), dtype=torch.float32, device="cuda")
    for method in (oracle.SS, oracle.SSSP):
        full = ctx.ss_best_period(method, dc, grid)
        part = ctx.refine_best_period(method, dc, grid, lt, ref.BINS, 0)
        torch.cuda.synchronize()
        assert torch.equal(full[0], part[0]) and torch.equal(full[2], part[2])


def test_learned_call_equals_forward_then_refine(ctx):
    import torch
    cat = _catalog(33, 30, (20, 500))
    grid = (0.05, 20.0, 20000)
    pt = torch.tensor(_params(4), dtype=torch.float32, device="cuda")
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    _, logits, _ = ctx.enc_forward(dc, grid, pt)
    a = ctx.refine_best_period(0, dc, grid, logits, 16, 1)
    b = ctx.learned_best_period(0, dc, grid, pt, 0.0, 16, 1)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_bin_scores_match_reference(ctx):
    import torch
    cat = synth.make_catalog(34, 10, (20, 400), 1000.0, (0.2, 10.0), 0.05)
    cat.e[cat.offsets[3]] = 0.0  # object 3: bad error bar
    grid = (0.1, 10.0, 3000)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    sc, st = ctx.bin_scores(dc, grid)
    torch.cuda.synchronize()
    sc = sc.cpu().numpy().astype(np.float64)
    assert st.cpu().numpy()[3] == ssg.OBJ_BAD_ERR
    for o in range(cat.n_obj):
        a, b = cat.offsets[o], cat.offsets[o + 1]
        r = ref.bin_scores(cat.t[a:b], cat.y[a:b], cat.e[a:b], grid)
        # FP32 sums of at most 400 terms: relative error well under 1e-4
        np.testing.assert_allclose(sc[o], r, rtol=1e-4, atol=2e-6, err_msg=str(o))


def test_score_proposal_equals_refine_on_scores(ctx):
    """gamma x scores with no encoder selects exactly the top bins of the scores."""
    import torch
    cat = synth.make_catalog(35, 16, (30, 300), 1000.0, (0.2, 10.0), 0.05)
    grid = (0.1, 10.0, 4000)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    sc, _ = ctx.bin_scores(dc, grid)
    for method in (0, 1):
        a = ctx.refine_best_period(method, dc, grid, sc, 8, 1)
        b = ctx.learned_best_period(method, dc, grid, None, 1.0, 8, 1)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y)
