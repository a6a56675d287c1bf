"""PageRank (Section 4.1) and NMF (Section 4.3) on the GPU against the FP64
oracle.  Bars: PageRank relative L1 <= 1e-5 after 30 iterations (FP32
vectors, FP64 reductions), sum PR = 1 within 1e-5; NMF relative Frobenius
<= 1e-4 on W and H after 10 iterations (proposed bar)."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth
from gpu_util import transpose_csr

pytestmark = pytest.mark.gpu


def _pr_gpu(h, n, iters=30, flags=0, init=None):
    import torch
    pr = torch.empty(n, dtype=torch.float32, device="cuda")
    if init is not None:
        pr.copy_(torch.from_numpy(init))
    res = pk.spmm_pagerank(h, pr, iters=iters, flags=flags)
    return pr.cpu().numpy().astype(np.float64), res


def _rel_l1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


@pytest.mark.parametrize("scale", [12, 16])
def test_pagerank_symmetric_matches_oracle(scale):
    rp, col = synth.rmat_csr(scale, 16, seed=1, symmetrize=True)
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col)
    pr, res = _pr_gpu(h, n)
    ref, rref = oracle.pagerank(rp, col, n, iters=30, symmetric=True)
    assert _rel_l1(pr, ref) <= 1e-5
    assert abs(pr.sum() - 1.0) <= 1e-5
    assert np.all(np.abs(res - rref) <= 1e-6 + 1e-3 * rref)
    pr2, res2 = _pr_gpu(h, n, flags=pk.SPMM_PR_NO_GRAPH)
    assert np.array_equal(pr, pr2) and np.array_equal(res, res2)   # graph == eager launches


def test_pagerank_directed_uses_transpose():
    rp, col = synth.rmat_csr(14, 8, seed=2)
    n = rp.shape[0] - 1
    t_ptr, t_col, _ = transpose_csr(rp, col, None, n)
    h = pk.spmm_build_tiles(t_ptr, t_col)   # row u = in-neighbours of u
    pr, _ = _pr_gpu(h, n)
    ref, _ = oracle.pagerank(rp, col, n, iters=30)
    assert _rel_l1(pr, ref) <= 1e-5
    # paper-literal mode (no dangling redistribution) and a given start vector
    init = synth.uniform(n, 1, seed=7)[:, 0].astype(np.float32)
    init /= init.sum()
    pr3, _ = _pr_gpu(h, n, iters=5, flags=pk.SPMM_PR_NO_REDISTRIBUTE | pk.SPMM_PR_INIT_GIVEN, init=init)
    deg = np.diff(rp).astype(np.float64)
    ref3 = init.astype(np.float64)
    for _ in range(5):
        x = np.where(deg > 0, ref3 / np.maximum(deg, 1), 0.0)
        ref3 = 0.15 / n + 0.85 * oracle.spmv_t(rp, col, None, x, n)
    assert _rel_l1(pr3, ref3) <= 1e-5


@pytest.mark.parametrize("symmetric", [True, False])
def test_nmf_matches_oracle(symmetric):
    rp, col = synth.rmat_csr(12, 8, seed=1, symmetrize=symmetric)
    n = rp.shape[0] - 1
    r = 16
    W0 = synth.uniform(n, r, seed=synth.SEED_W)
    H0 = synth.uniform(n, r, seed=synth.SEED_H)
    hA = pk.spmm_build_tiles(rp, col)
    if symmetric:
        hAT, AT = hA, None
    else:
        AT = transpose_csr(rp, col, None, n)
        hAT = pk.spmm_build_tiles(AT[0], AT[1])
    import torch
    W = torch.from_numpy(W0.copy()).cuda()
    H = torch.from_numpy(H0.copy()).cuda()
    pk.spmm_nmf(hA, hAT, W, H, iters=10, eps=1e-9)
    torch.cuda.synchronize()
    Wr, Hr = oracle.nmf(rp, col, None, W0, H0, iters=10, eps=1e-9, AT=AT)
    assert oracle.frob_rel_err(W.cpu().numpy(), Wr) <= 1e-4
    assert oracle.frob_rel_err(H.cpu().numpy(), Hr) <= 1e-4
    assert W.min().item() >= 0 and H.min().item() >= 0


def test_nmf_calls_are_asynchronous_and_chain():
    """spmm_nmf returns once its work is queued (workspace kept on the
    handle): two 5-iteration calls queued back to back, with a wider rank in
    between that regrows the workspace, equal one 10-iteration call bit for
    bit."""
    import torch
    rp, col = synth.rmat_csr(12, 8, seed=4, symmetrize=True)
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col)
    W0 = synth.uniform(n, 8, seed=synth.SEED_W)
    H0 = synth.uniform(n, 8, seed=synth.SEED_H)
    W1, H1 = torch.from_numpy(W0.copy()).cuda(), torch.from_numpy(H0.copy()).cuda()
    pk.spmm_nmf(h, h, W1, H1, iters=10)
    W2, H2 = torch.from_numpy(W0.copy()).cuda(), torch.from_numpy(H0.copy()).cuda()
    pk.spmm_nmf(h, h, W2, H2, iters=5)
    Wb = torch.from_numpy(synth.uniform(n, 16, seed=7)).cuda()
    Hb = torch.from_numpy(synth.uniform(n, 16, seed=8)).cuda()
    pk.spmm_nmf(h, h, Wb, Hb, iters=2)
    pk.spmm_nmf(h, h, W2, H2, iters=5)
    torch.cuda.synchronize()
    assert torch.equal(W1, W2) and torch.equal(H1, H2)
    h.close()


def test_directed_apps_with_transposed_handle():
    """PageRank and NMF on a directed graph with A^T tiled by the library
    (build option transpose) instead of a caller-side transpose."""
    import torch
    rp, col = synth.rmat_csr(14, 8, seed=2)
    n = rp.shape[0] - 1
    hT = pk.spmm_build_tiles(rp, col, transpose=True)      # row u = in-neighbours of u
    pr, _ = _pr_gpu(hT, n)
    ref, _ = oracle.pagerank(rp, col, n, iters=30)
    assert _rel_l1(pr, ref) <= 1e-5 and abs(pr.sum() - 1.0) <= 1e-5
    hA = pk.spmm_build_tiles(rp, col)
    W0 = synth.uniform(n, 8, seed=synth.SEED_W)
    H0 = synth.uniform(n, 8, seed=synth.SEED_H)
    W = torch.from_numpy(W0).cuda()
    H = torch.from_numpy(H0).cuda()
    pk.spmm_nmf(hA, hT, W, H, iters=10)
    torch.cuda.synchronize()
    AT = transpose_csr(rp, col, None, n)
    Wr, Hr = oracle.nmf(rp, col, None, W0, H0, iters=10, eps=1e-9, AT=AT)
    assert oracle.frob_rel_err(W.cpu().numpy(), Wr) <= 1e-4
    assert oracle.frob_rel_err(H.cpu().numpy(), Hr) <= 1e-4
    hT.close()
    hA.close()
