"""The SpMM's stated arithmetic (spmm.h, spmm_run): exact fixed-point sums
on a per-column grid, and NaN columns for non-finite X.

The expected values here come from the documented rule, computed on the
CPU, not from the FP64 oracle: the point is the rule's edge (products far
below a column's bound round to the grid, possibly to zero), which no
relative-error bar against the oracle can see."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth
from gpu_util import run_spmm

pytestmark = pytest.mark.gpu


def _perm_csr(n, seed):
    p = synth.draws(synth.stream_key(seed, 13), 0, n).argsort().astype(np.int32)
    return np.arange(n + 1, dtype=np.int64), p


def test_products_round_to_the_column_grid():
    """A permutation matrix (largest row L1 norm 1) and a column whose
    largest |x| is 1: the grid is 2^-60 (2^e = 2 is the smallest power of two
    above 1, f = 61 - 1).  Every Y entry is its x rounded to that grid, ties
    to even -- 2^-62 vanishes, 3 * 2^-62 becomes 2^-60."""
    n = 4096
    rp, col = _perm_csr(n, 3)
    X = synth.uniform(n, 2, seed=4)
    tiny = np.array([2.0 ** -60, 2.0 ** -61, 3 * 2.0 ** -62, 2.0 ** -62, 2.0 ** -70, 5 * 2.0 ** -61,
                     -(2.0 ** -61), -3 * 2.0 ** -62, 1.0 + 2.0 ** -23, 1.0], np.float64)
    X[: tiny.size, 0] = tiny.astype(np.float32)
    X[:, 0] = np.minimum(X[:, 0], 1.0)
    X[:, 1] *= 1e-30                          # a column of tiny values keeps its own grid
    X = X.astype(np.float32)
    h = pk.spmm_build_tiles(rp, col)
    Y = run_spmm(h, X)
    h.close()
    x = X[col].astype(np.float64)              # row r holds x[col[r]]
    m = np.abs(X.astype(np.float64)).max(axis=0)
    e = np.frexp(m)[1]                         # m < 2^e
    f = 61 - e
    want = (np.rint(x * 2.0 ** f) * 2.0 ** -f).astype(np.float32)
    assert np.array_equal(Y, want)
    # the first column: exactly the listed outcomes
    r_of = np.empty(n, np.int64)
    r_of[col] = np.arange(n)
    got = Y[r_of[: tiny.size], 0].astype(np.float64)
    g = 2.0 ** -60
    assert list(got) == [g, 0.0, g, 0.0, 0.0, 2 * g, 0.0, -g, 1.0, 1.0]


@pytest.mark.parametrize("dt", ["f32", "bf16", "fp8"])
def test_non_finite_x_gives_nan_columns(dt):
    rp, col = synth.rmat_csr(12, 8, seed=5)
    n = rp.shape[0] - 1
    X = synth.uniform(n, 4, seed=2)
    has_entries = np.diff(rp) > 0
    hit = int(col[rp[np.flatnonzero(has_entries)[0]]])     # a column some row reads
    if dt == "f32":
        X[hit, 1] = np.inf
        X[(hit + 1) % n, 2] = np.nan
        Xq, kw = X, {}
        deq = X.astype(np.float64)
    elif dt == "bf16":
        Xq = (X.view(np.uint32) >> 16).astype(np.uint16)
        Xq[hit, 1] = 0x7F80                                 # +inf
        Xq[(hit + 1) % n, 2] = 0x7FC0                       # NaN
        kw = {"dtype": pk.SPMM_X_BF16}
        deq = oracle.bf16_decode(Xq.ravel()).reshape(n, 4).astype(np.float64)
    else:
        Xq = oracle.e4m3_encode(X.ravel()).reshape(n, 4)
        Xq[hit, 1] = 0x7F                                   # NaN code
        Xq[(hit + 1) % n, 2] = 0xFF                         # NaN code
        kw = {"dtype": pk.SPMM_X_FP8_E4M3, "col_scale": np.ones(4, np.float32)}
        deq = oracle.e4m3_decode(Xq.ravel()).reshape(n, 4).astype(np.float64)
    h = pk.spmm_build_tiles(rp, col)
    Y = run_spmm(h, Xq, **kw)
    h.close()
    ref = oracle.spmm(rp, col, None, np.nan_to_num(deq, nan=0.0, posinf=0.0))
    for j in (0, 3):
        assert oracle.frob_rel_err(Y[:, j:j + 1], ref[:, j:j + 1]) <= 1e-6
    for j in (1, 2):
        assert np.isnan(Y[has_entries, j]).all(), j
        assert (Y[~has_entries, j] == 0.0).all(), j
