"""spmm_run_static -- spmm_run without device allocation (its scratch in a
static device array) -- against spmm_run through the C ABI: identical
results on consecutive calls, the second on a smaller input, and the
stated preconditions."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth

pytestmark = pytest.mark.gpu


def _run(fn, h, X, k):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Yd = torch.full((h.n_rows, k), float("nan"), device="cuda")
    fn(h, Xd, Yd)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


def test_static_scratch_matches_spmm_run_on_consecutive_calls():
    big = synth.rmat_csr(15, 16, seed=41)
    small = synth.rmat_csr(12, 8, seed=42)
    hb = pk.spmm_build_tiles(*big, keep_order=True, item_nnz=500)     # many split rows: partial slots used
    hs = pk.spmm_build_tiles(*small, keep_order=True, item_nnz=200)
    assert pk.spmm_get_stats(hb)["n_parts"] > pk.spmm_get_stats(hs)["n_parts"] > 0
    cases = [(hb, big, 8), (hs, small, 3), (hb, big, 33), (hs, small, 1)]
    for h, (rp, col), k in cases:
        _run(pk.spmm_run, h, synth.uniform(rp.shape[0] - 1, k, seed=1), k)   # puts the tiles on the device
    for i, (h, (rp, col), k) in enumerate(cases):
        n = rp.shape[0] - 1
        Xu = synth.uniform(n, k, seed=2 + i)
        assert np.array_equal(_run(pk.spmm_run_static, h, Xu, k), _run(pk.spmm_run, h, Xu, k)), i
        Xi = synth.int07(n, k, seed=9 + i)
        assert np.array_equal(_run(pk.spmm_run_static, h, Xi, k).astype(np.float64),
                              oracle.spmm(rp, col, None, Xi)), i
    hb.close()
    hs.close()


def test_static_scratch_preconditions():
    import torch
    rp, col = synth.rmat_csr(11, 8, seed=43)
    n = rp.shape[0] - 1
    X = torch.from_numpy(synth.uniform(n, 4, seed=2)).cuda()
    Y = torch.empty((n, 4), device="cuda")
    h = pk.spmm_build_tiles(rp, col)                                       # relabelled columns
    pk.spmm_run(h, X, Y)
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_run_static(h, X, Y)
    assert ei.value.status == pk.SPMM_EUNSUPPORTED
    h.close()
    h = pk.spmm_build_tiles(rp, col, keep_order=True)
    with pytest.raises(pk.SpmmError) as ei:                                # tiles not on the device yet
        pk.spmm_run_static(h, X, Y)
    assert ei.value.status == pk.SPMM_ESTATE
    h.close()
    # a handle whose split rows need more than the 16 MiB of scratch
    rows, width = 6000, 200
    cols = np.sort((np.arange(rows)[:, None] * 7 + np.arange(width)[None, :] * 37) % 8192, axis=1)
    rp2 = np.arange(rows + 1, dtype=np.int64) * width
    h = pk.spmm_build_tiles(rp2, cols.astype(np.int32).ravel(), n_cols=8192, keep_order=True, item_nnz=16)
    X2 = torch.from_numpy(synth.uniform(8192, 4, seed=3)).cuda()
    Y2 = torch.empty((rows, 4), device="cuda")
    pk.spmm_run(h, X2, Y2)
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_run_static(h, X2, Y2)
    assert ei.value.status == pk.SPMM_EINVAL
    torch.cuda.synchronize()
    h.close()
