"""Parity at the benchmark's full size, in the configuration bench.py times.

The directed R-MAT graph of scale 25, edge factor 44 (33,554,432 vertices,
1,431,381,365 non-zeros) with the default build; the oracle computes sampled
output rows one by one: the 64 highest-degree rows (R-MAT's hubs are rows
0-63) and 64 evenly spread blocks of consecutive rows.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth

from gpu_util import dev

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[fullsize {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def full():
    rp, col = synth.rmat_csr(25, 44, seed=synth.SEED_GRAPH, progress=log)
    n = rp.shape[0] - 1
    assert col.shape[0] == 1431381365
    deg = np.diff(rp)
    assert 7 * int(deg.max()) < 2 ** 24          # integer X stays exact in FP32
    B = 2048
    starts = np.linspace(64, n - B, 64).astype(np.int64)
    sel = np.unique(np.concatenate([np.arange(64)] + [np.arange(s, s + B) for s in starts]))
    h = pk.spmm_build_tiles(rp, col, validate=False)
    log(f"built: {pk.spmm_get_stats(h)['n_items']} items; {sel.size} sampled rows, {int(deg[sel].sum())} nnz")
    yield rp, col, n, sel, h
    h.close()


def _sampled(h, n, X, sel, **kw):
    import torch
    Xd = torch.from_numpy(X).to(dev())
    Yd = torch.empty((n, X.shape[1]), dtype=torch.float32, device=dev())
    pk.spmm_run(h, Xd, Yd, **kw)
    rows = Yd[torch.from_numpy(sel).to(dev())].cpu().numpy()
    del Xd, Yd
    return rows


@pytest.mark.parametrize("k", [1, 4, 32])
def test_fp32_sampled_rows(full, k):
    rp, col, n, sel, h = full
    X = synth.uniform(n, k, seed=synth.SEED_X)
    got = _sampled(h, n, X, sel)
    err = oracle.frob_rel_err(got, oracle.spmm_sel(rp, col, None, X, sel))
    log(f"k={k}: relative Frobenius {err:.3g}")
    assert err <= 1e-6


def test_integer_sampled_rows_exact(full):
    rp, col, n, sel, h = full
    X = synth.int07(n, 4, seed=3)
    got = _sampled(h, n, X, sel)
    assert np.array_equal(got.astype(np.float64), oracle.spmm_sel(rp, col, None, X, sel))


def test_learned_selection_sampled_rows(full):
    from paper_1602_02864_amd.selector_train import WEIGHTS
    rp, col, n, sel, _ = full
    h = pk.spmm_build_tiles(rp, col, validate=False)
    pk.spmm_select_learned(h, np.load(WEIGHTS, allow_pickle=False), 1)
    X = synth.int07(n, 1, seed=4)
    got = _sampled(h, n, X, sel)
    h.close()
    assert np.array_equal(got.astype(np.float64), oracle.spmm_sel(rp, col, None, X, sel))


def test_streamed_equals_in_hbm(full):
    import torch
    rp, col, n, sel, h = full
    hs = pk.spmm_build_tiles(rp, col, validate=False, place=pk.SPMM_PLACE_PINNED_HOST)
    X = torch.from_numpy(synth.uniform(n, 4, seed=synth.SEED_X)).to(dev())
    Yd = torch.empty((n, 4), device=dev())
    Ys = torch.empty((n, 4), device=dev())
    pk.spmm_run(h, X, Yd)
    pk.spmm_stream_run(hs, X, Ys, copy=torch.cuda.Stream(dev()))
    torch.cuda.synchronize()
    assert torch.equal(Yd, Ys)
    hs.close()
