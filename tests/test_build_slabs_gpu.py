"""A handle built slab-wise (spmm_build_begin / append_rows / end) against
the oracle on the GPU: integer X exact, FP32 X within 1e-6, in HBM and
streamed."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth
from gpu_util import run_spmm

pytestmark = pytest.mark.gpu


def _slab_build(rp, col, val, block, **opts):
    n = rp.shape[0] - 1
    h = pk.spmm_build_begin(n, **opts)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        a, b = rp[r0], rp[r1]
        pk.spmm_build_append_rows(h, r0, rp[r0:r1 + 1] - a, col[a:b], None if val is None else val[a:b])
    pk.spmm_build_end(h)
    return h


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("block", [1000, 1 << 20])
def test_slab_built_handle_matches_oracle(weighted, block):
    rp, col = synth.rmat_csr(15, 16, seed=8)
    n = rp.shape[0] - 1
    val = synth.lognormal_weights(rp, col, seed=3) if weighted else None
    h = _slab_build(rp, col, val, block, item_nnz=2000)
    for k in (1, 4, 33):
        Xi = synth.int07(n, k, seed=2)
        Y = run_spmm(h, Xi)
        ref = oracle.spmm(rp, col, val, Xi)
        if weighted:
            assert oracle.frob_rel_err(Y, ref) <= 1e-6
        else:
            assert np.array_equal(Y.astype(np.float64), ref)
        Xu = synth.uniform(n, k, seed=3)
        assert oracle.frob_rel_err(run_spmm(h, Xu), oracle.spmm(rp, col, val, Xu)) <= 1e-6
    h.close()


def test_slab_built_streamed_equals_in_hbm():
    import torch
    rp, col = synth.rmat_csr(15, 16, seed=9)
    n = rp.shape[0] - 1
    hd = _slab_build(rp, col, None, 3000)
    hs = _slab_build(rp, col, None, 3000, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=256)
    X = torch.from_numpy(synth.uniform(n, 8, seed=2)).cuda()
    Yd = torch.empty((n, 8), device="cuda")
    Ys = torch.empty((n, 8), device="cuda")
    pk.spmm_run(hd, X, Yd)
    pk.spmm_stream_run(hs, X, Ys, copy=torch.cuda.Stream())
    torch.cuda.synchronize()
    assert torch.equal(Yd, Ys)
    hd.close()
    hs.close()
