"""The phase-dispersion finder computed from the trial kernel's own fold and
sort, against the FP64 oracle, through the C ABI.  Bar: |dscore| <= 1e-9 at
every frequency where no point lies within 1e-9 of a phase-bin edge (there the
fold's last bits decide the bin and either side is correct, the same reading
as for sort ties); FP32c within 1e-5.  The method's own periodogram from the
same call meets the FP64 parity bar."""
import numpy as np
import pytest

import oracle
import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth
from tests.test_parity_gpu import _assert_pgram_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = ssg.Context(0)
    yield c
    c.close()


def _catalog():
    lens = [5, 17, 64, 65, 100, 200, 257, 400, 700]
    cats = [synth.make_catalog(3000 + i, 1, n, 500.0, (0.3, 5.0), 0.05, shapes=(i % 3,))
            for i, n in enumerate(lens)]
    offs = np.concatenate([[0], np.cumsum([c.offsets[-1] for c in cats])]).astype(np.int64)
    t = np.concatenate([c.t for c in cats])
    y = np.concatenate([c.y for c in cats])
    e = np.concatenate([c.e for c in cats])
    e[offs[1]] = -1.0  # object 1: bad error bar
    return offs, t, y, e


def _edge_mask(offs, t, y, e, grid, n_bins):
    """True where some point of the object is within 1e-9 of a bin edge."""
    fmin, fmax, nf = grid
    mask = np.zeros((len(offs) - 1, nf), dtype=bool)
    for o in range(len(offs) - 1):
        a, b = offs[o], offs[o + 1]
        st, tt, w, ybar, chi0 = oracle.prep(t[a:b], y[a:b], e[a:b])
        if st != 0:
            continue
        B = oracle.pdm_bins(b - a, n_bins)
        for k in range(nf):
            z = oracle.fold(tt, oracle.freq(fmin, fmax, nf, k)) * B
            # the earliest point has phase exactly 0 at every frequency: not an edge case
            mask[o, k] = np.any((np.abs(z - np.rint(z)) < 1e-9) & (z != 0.0))
    return mask


@pytest.mark.parametrize("method,n_bins", [(0, 0), (1, 7), (2, 0)])
def test_pdm_matches_oracle(ctx, method, n_bins):
    import torch
    offs, t, y, e = _catalog()
    grid = (0.2, 3.3, 97)
    dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
    pg, pd, st = ctx.pdm_periodogram(method, dc, grid, n_bins)
    torch.cuda.synchronize()
    pm, _ = oracle.periodogram(method, offs, t, y, e, *grid)
    _assert_pgram_close(pg.cpu().numpy(), pm, what=f"method {method} beside the second finder")
    pd = pd.cpu().numpy()
    po = oracle.pdm_periodogram(offs, t, y, e, *grid, n_bins=n_bins)
    assert st.cpu().numpy()[1] == ssg.OBJ_BAD_ERR
    assert np.isnan(pd[1]).all() and np.isnan(po[1]).all()
    edge = _edge_mask(offs, t, y, e, grid, n_bins)
    ok = np.isfinite(po) & ~edge
    assert np.all(np.abs(pd[ok] - po[ok]) <= 1e-9), float(np.max(np.abs(pd[ok] - po[ok])))
    assert ok.sum() >= 0.99 * np.isfinite(po).sum()


def test_pdm_fp32c(ctx):
    import torch
    offs, t, y, e = _catalog()
    grid = (0.2, 3.3, 61)
    dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
    pg, pd, st = ctx.pdm_periodogram(0, dc, grid, 0, ssg.Params(precision=ssg.SS_FP32C))
    torch.cuda.synchronize()
    pd = pd.cpu().numpy().astype(np.float64)
    po = oracle.pdm_periodogram(offs, t, y, e, *grid)
    ok = np.isfinite(po) & ~_edge_mask(offs, t, y, e, grid, 0)
    assert np.all(np.abs(pd[ok] - po[ok]) <= 1e-5)
