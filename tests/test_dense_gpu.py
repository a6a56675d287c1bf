"""Tall-skinny dense products of the eigensolver through the C ABI, against
FP64 products of the same FP32 inputs: C = A^T B (FP64 result, sums in a
fixed order) and W = alpha W + beta A C (FP64 sums, one rounding to FP32)."""
import numpy as np
import pytest

import paper_1602_02864_amd as pk
import synth

from gpu_util import dev

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


@pytest.mark.parametrize("n,p,q,lda,ldb", [(0, 3, 2, 3, 2), (1, 1, 1, 1, 1), (1000, 5, 3, 7, 4),
                                            (70001, 36, 2, 52, 2), (9000, 300, 3, 301, 3),
                                            (12345, 64, 16, 64, 16), (5000, 512, 2, 520, 2),
                                            (3000, 128, 16, 130, 16)])
def test_tn_matches_fp64(n, p, q, lda, ldb):
    import torch
    A = synth.uniform(n, lda, seed=1) - 0.5
    B = synth.uniform(n, ldb, seed=2) - 0.5
    Ad, Bd = _dev(A), _dev(B)
    C = torch.full((p, q), float("nan"), dtype=torch.float64, device=dev())
    work = torch.empty(pk.spmm_dense_tn_workspace(n, p, q) // 8, dtype=torch.float64, device=dev())
    pk.spmm_dense_tn(Ad, Bd, C, work, p=p, q=q)
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    ref = A[:, :p].astype(np.float64).T @ B[:, :q].astype(np.float64)
    bound = np.abs(A[:, :p]).astype(np.float64).T @ np.abs(B[:, :q]).astype(np.float64)
    assert np.all(np.abs(got - ref) <= 1e-13 * bound + 1e-300)
    C2 = torch.zeros_like(C)
    pk.spmm_dense_tn(Ad, Bd, C2, work, p=p, q=q)
    torch.cuda.synchronize()
    assert torch.equal(C, C2)                       # same bits every call


@pytest.mark.parametrize("n,p,q,lda,ldw,alpha,beta", [(0, 2, 2, 2, 2, 0.0, 1.0), (1, 1, 1, 1, 1, 1.0, -1.0),
                                                      (1000, 5, 3, 7, 4, 1.0, -1.0), (70001, 40, 2, 41, 2, 0.0, 1.0),
                                                      (3000, 100, 56, 104, 60, 0.0, 1.0),
                                                      (2500, 33, 70, 40, 70, 0.5, 2.0)])
def test_nn_matches_fp64(n, p, q, lda, ldw, alpha, beta):
    import torch
    A = synth.uniform(n, lda, seed=3) - 0.5
    Cm = (synth.uniform(p, q, seed=4) - 0.5).astype(np.float64)
    W0 = synth.uniform(n, ldw, seed=5)
    if alpha == 0.0:
        W0[:, :q] = np.nan                          # not read when alpha = 0
    Wd = _dev(W0)
    pk.spmm_dense_nn(_dev(A), _dev(Cm), Wd, alpha=alpha, beta=beta, p=p, q=q)
    torch.cuda.synchronize()
    got = Wd.cpu().numpy()
    ref = beta * (A[:, :p].astype(np.float64) @ Cm)
    if alpha != 0.0:
        ref = ref + alpha * W0[:, :q].astype(np.float64)
    scale = np.abs(beta) * (np.abs(A[:, :p]).astype(np.float64) @ np.abs(Cm))
    if alpha != 0.0:
        scale = scale + abs(alpha) * np.abs(W0[:, :q])
    assert np.all(np.abs(got[:, :q] - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-13 * scale + 1e-300)
    assert np.array_equal(got[:, q:], W0[:, q:], equal_nan=True)     # columns past q untouched


def test_argument_errors():
    import torch
    A = torch.zeros((10, 4), device=dev())
    C = torch.zeros((4, 4), dtype=torch.float64, device=dev())
    work = torch.empty(pk.spmm_dense_tn_workspace(10, 4, 4) // 8, dtype=torch.float64, device=dev())
    for kw in (dict(p=0), dict(q=17), dict(p=5)):
        with pytest.raises(pk.SpmmError):
            pk.spmm_dense_tn(A, A, C, work, **kw)
    with pytest.raises(pk.SpmmError):
        pk.spmm_dense_tn(A, A, C, work[:10])
    W = torch.zeros((10, 2), device=dev())
    with pytest.raises(pk.SpmmError):
        pk.spmm_dense_nn(A, C, W, q=3)                 # ldw < q
