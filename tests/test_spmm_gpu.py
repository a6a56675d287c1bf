"""GPU parity of Y = A X against the FP64 oracle, through the C ABI.

Bar (matching rules): bit-exact for binary A with integer X in {0..7}
(every partial sum is an integer below 2^24, so any summation order gives
the same bits); relative Frobenius error <= 1e-6 for FP32 X."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth
from gpu_util import dev, run_spmm

pytestmark = pytest.mark.gpu

KS = [1, 2, 3, 4, 5, 8, 16, 17, 32, 33, 64]


@pytest.fixture(scope="module")
def graph():
    rp, col = synth.rmat_csr(16, 16, seed=synth.SEED_GRAPH)   # small config: scale 16, ef 16
    assert 7 * np.diff(rp).max() < 2 ** 24
    return rp, col


@pytest.mark.parametrize("variant", range(pk.SPMM_NUM_VARIANTS))
def test_integer_x_bit_exact(graph, variant):
    rp, col = graph
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col, fixed_variant=variant)
    for k in KS:
        X = synth.int07(n, k, seed=2)
        Y = run_spmm(h, X)
        ref = oracle.spmm(rp, col, None, X)
        assert np.array_equal(Y.astype(np.float64), ref), (variant, k)


@pytest.mark.parametrize("variant", range(pk.SPMM_NUM_VARIANTS))
def test_fp32_within_1e6(graph, variant):
    rp, col = graph
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col, fixed_variant=variant)
    for k in KS:
        X = synth.uniform(n, k, seed=2)
        err = oracle.frob_rel_err(run_spmm(h, X), oracle.spmm(rp, col, None, X))
        assert err <= 1e-6, (variant, k, err)


GEOMS = [dict(tile_rows=16, tile_cols=256, item_nnz=100),      # many splits, tiny tiles
         dict(tile_rows=1, tile_cols=1 << 16),                 # one row per tile row
         dict(tile_rows=64, tile_cols=64, item_nnz=1),         # one unit per item
         dict(tile_rows=4096, tile_cols=1024, item_nnz=64),    # tall tile rows, tiny items
         dict(tile_rows=300, tile_cols=8192, item_nnz=5000),   # ragged tile rows
         dict(max_kc=32),
         dict(keep_order=True, tile_rows=64),
         dict(x_stage_kib=128),                                # X rows staged in LDS (k <= 8)
         dict(x_stage_kib=4)]                                  # 1024 staged rows at k = 1 only


@pytest.mark.parametrize("geom", GEOMS)
def test_geometries_integer_exact(graph, geom):
    rp, col = graph
    n = rp.shape[0] - 1
    for variant in range(pk.SPMM_NUM_VARIANTS):
        h = pk.spmm_build_tiles(rp, col, fixed_variant=variant, **geom)
        for k in (1, 4, 32, 48):
            X = synth.int07(n, k, seed=3)
            assert np.array_equal(run_spmm(h, X).astype(np.float64), oracle.spmm(rp, col, None, X)), \
                (geom, variant, k)
        h.close()


def test_weighted_rectangular_ragged():
    n_rows, n_cols = 5000, 70001
    d = synth.draws(synth.stream_key(9, 12), 0, n_rows * 9)
    rows = np.repeat(np.arange(n_rows), 9)
    cols = (d % np.uint64(n_cols)).astype(np.int64)
    pairs = np.unique(rows * n_cols + cols)
    r, c = pairs // n_cols, pairs % n_cols
    rp = np.zeros(n_rows + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp)
    col = c.astype(np.int32)
    val = synth.lognormal_weights(rp, col, seed=3)
    for variant in range(pk.SPMM_NUM_VARIANTS):
        h = pk.spmm_build_tiles(rp, col, val, n_cols=n_cols, tile_rows=77, fixed_variant=variant,
                                item_nnz=999)
        for k in (1, 6, 16):
            X = synth.uniform(n_cols, k, seed=4)
            err = oracle.frob_rel_err(run_spmm(h, X), oracle.spmm(rp, col, val, X))
            assert err <= 1e-6, (variant, k, err)
        h.close()


def test_strided_x_and_y(graph):
    rp, col = graph
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col)
    Xfull = synth.int07(n, 13, seed=5)
    import torch
    Xd = torch.from_numpy(Xfull).cuda()
    Yd = torch.full((n, 11), -7.0, device="cuda")
    pk.spmm_run(h, Xd[:, 2:], Yd[:, 1:], k=9, ldx=13, ldy=11)   # misaligned column offsets
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    ref = oracle.spmm(rp, col, None, Xfull[:, 2:11])
    assert np.array_equal(Y[:, 1:10].astype(np.float64), ref)
    assert np.all(Y[:, 0] == -7.0) and np.all(Y[:, 10] == -7.0)


def test_empty_rows_overwritten_and_empty_matrix():
    rp, col = synth.rmat_csr(14, 4, seed=1)
    n = rp.shape[0] - 1
    assert (np.diff(rp) == 0).any()
    h = pk.spmm_build_tiles(rp, col)
    Y = run_spmm(h, synth.uniform(n, 4, seed=1), fill=float("nan"))
    assert not np.isnan(Y).any()
    assert np.all(Y[np.diff(rp) == 0] == 0)
    rp0 = np.zeros(1001, np.int64)
    h0 = pk.spmm_build_tiles(rp0, np.zeros(0, np.int32))
    assert np.all(run_spmm(h0, synth.uniform(1000, 3, seed=1)) == 0)


def test_repeat_runs_bit_identical(graph):
    rp, col = graph
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col, item_nnz=2000)
    X = synth.uniform(n, 8, seed=6)
    a = run_spmm(h, X)
    b = run_spmm(h, X)
    assert np.array_equal(a, b)


def test_hub_rows_fp32_accuracy():
    """Symmetrised scale-18 graph: hub rows of several thousand entries."""
    rp, col = synth.rmat_csr(18, 16, seed=1, symmetrize=True)
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col)
    X = synth.uniform(n, 4, seed=2)
    Y = run_spmm(h, X)
    ref = oracle.spmm(rp, col, None, X)
    assert oracle.frob_rel_err(Y, ref) <= 1e-6
    top = np.argsort(np.diff(rp))[-50:]
    assert oracle.frob_rel_err(Y[top], ref[top]) <= 1e-6


def test_kernel_timing_counts_runs(graph):
    import torch
    rp, col = graph
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col)
    X = torch.from_numpy(synth.uniform(n, 4, seed=2)).to(dev())
    Y = torch.empty((n, 4), device=dev())
    pk.spmm_run(h, X, Y)
    pk.spmm_timing_begin(h)
    for _ in range(3):
        pk.spmm_run(h, X, Y)
    ms, runs = pk.spmm_timing_end(h)
    assert runs == 3 and ms > 0.0
    pk.spmm_run(h, X, Y)            # after the window: not recorded
    pk.spmm_timing_begin(h)
    assert pk.spmm_timing_end(h) == (0.0, 0)
    h.close()


def test_read_probe_reads_without_writing():
    import torch
    buf = torch.ones(1 << 20, dtype=torch.float32, device=dev())
    sink = torch.full((1,), 7.0, device=dev())
    pk.spmm_read_probe(buf, sink)
    pk.spmm_read_probe(buf[:5], sink, nbytes=16)   # a partial buffer
    torch.cuda.synchronize()
    assert sink.item() == 7.0
