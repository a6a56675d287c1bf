"""Rows without entries of a row-relabelled handle are not tiled; the
library zero-fills them, on a side stream concurrently with the SpMM when
there are many (spmm.h, spmm_run).  Both paths against the oracle, with Y
pre-filled with NaN, over back-to-back calls."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [1, 32])
def test_empty_rows_zero_filled_back_to_back(k):
    import torch
    rp, col = synth.rmat_csr(22, 4, seed=31)
    n = rp.shape[0] - 1
    empty = np.diff(rp) == 0
    # k = 32 takes the side-stream fill (>= 2^26 zero values), k = 1 the
    # fill after the SpMM on the caller's stream
    assert (int(empty.sum()) * 32 >= 1 << 26) and (int(empty.sum()) * 1 < 1 << 26)
    h = pk.spmm_build_tiles(rp, col)
    Xs = [synth.uniform(n, k, seed=s) for s in (4, 5, 6)]
    Ys = [torch.full((n, k), float("nan"), dtype=torch.float32, device=dev()) for _ in Xs]
    for X, Y in zip(Xs, Ys):
        pk.spmm_run(h, torch.from_numpy(X).to(dev()), Y)      # no synchronisation between calls
    torch.cuda.synchronize()
    for X, Y in zip(Xs, Ys):
        got = Y.cpu().numpy()
        assert (got[empty] == 0.0).all()
        ref = oracle.spmm(rp, col, None, X.astype(np.float64))
        assert oracle.frob_rel_err(got, ref) <= 1e-6
    h.close()
