"""The untiled CSR format (V-csr, the baseline of the format comparison)
against the oracle: integer X exact, FP32 X within 1e-6, for column counts
that exercise every launch width and the row classes (lane groups,
wavefronts, split rows); PageRank through it."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth
from gpu_util import run_spmm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("keep", [False, True])
def test_csr_format_matches_oracle(keep):
    rp, col = synth.rmat_csr(16, 16, seed=1, symmetrize=True)
    n = rp.shape[0] - 1
    assert np.diff(rp).max() > 8192          # some rows are split into pieces
    h = pk.spmm_build_tiles(rp, col, format=pk.SPMM_FORMAT_CSR, keep_order=keep)
    for k in (1, 2, 3, 4, 8, 17, 32, 33, 64):
        Xi = synth.int07(n, k, seed=2)
        assert np.array_equal(run_spmm(h, Xi).astype(np.float64), oracle.spmm(rp, col, None, Xi)), k
        Xu = synth.uniform(n, k, seed=3)
        assert oracle.frob_rel_err(run_spmm(h, Xu, ldy=k + 1)[:, :k], oracle.spmm(rp, col, None, Xu)) <= 1e-6, k
    with pytest.raises(pk.SpmmError) as ei:
        run_spmm(h, oracle.bf16_quantize(synth.uniform(n, 4, seed=3)), dtype=pk.SPMM_X_BF16)
    assert ei.value.status == pk.SPMM_EUNSUPPORTED
    h.close()


def test_pagerank_on_csr_format():
    import torch
    rp, col = synth.rmat_csr(14, 8, seed=2, symmetrize=True)
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col, format=pk.SPMM_FORMAT_CSR)
    pr = torch.empty(n, device="cuda")
    pk.spmm_pagerank(h, pr, iters=30)
    torch.cuda.synchronize()
    ref, _ = oracle.pagerank(rp, col, n, iters=30, symmetric=True)
    got = pr.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).sum() / np.abs(ref).sum() <= 1e-5
    h.close()
