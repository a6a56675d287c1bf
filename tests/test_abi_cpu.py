"""CPU checks of the C ABI: every declared symbol is exported, argument
errors are reported, and the host-side tile encoding round-trips exactly
(decoded with the kernels' indexing).  No GPU is touched here."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth


def test_library_exports_every_header_symbol():
    L = pk.load_library()
    names = pk.header_functions()
    assert "spmm_run" in names and "spmm_build_tiles" in names
    for n in names:
        assert hasattr(L, n), n


def _err(fn, *a, **kw):
    with pytest.raises(pk.SpmmError) as ei:
        fn(*a, **kw)
    return ei.value


def test_build_rejects_bad_options_and_csr():
    rp, col = synth.small_random_csr(20, 0.2, 1)
    assert _err(pk.spmm_build_tiles, rp, col, tile_rows=5000).status == pk.SPMM_EINVAL
    assert _err(pk.spmm_build_tiles, rp, col, tile_cols=1000).status == pk.SPMM_EINVAL
    assert _err(pk.spmm_build_tiles, rp, col, fixed_variant=9).status == pk.SPMM_EINVAL
    bad = col.copy()
    bad[0] = 25
    e = _err(pk.spmm_build_tiles, rp, bad)
    assert e.status == pk.SPMM_EINVAL and "range" in pk.spmm_last_error()
    uns = col.copy()
    r = int(np.argmax(np.diff(rp) >= 2))
    uns[rp[r]], uns[rp[r] + 1] = uns[rp[r] + 1], uns[rp[r]]
    assert _err(pk.spmm_build_tiles, rp, uns).status == pk.SPMM_EINVAL
    pk.spmm_build_tiles(rp, uns, validate=False).close()   # unsorted allowed without validation
    rp2 = rp.copy()
    rp2[3] = rp2[4] + 1
    assert _err(pk.spmm_build_tiles, rp2, col).status == pk.SPMM_EINVAL


def test_null_handle_and_args():
    L = pk.load_library()
    assert L.spmm_run(None, None, 4, 4, 0, None, None, 4, None) == pk.SPMM_EINVAL
    assert L.spmm_get_stats(None, None) == pk.SPMM_EINVAL
    L.spmm_destroy(None)


def test_run_argument_checks_before_device():
    rp, col = synth.small_random_csr(20, 0.2, 1)
    h = pk.spmm_build_tiles(rp, col)
    L = pk.load_library()
    fake = 1 << 20
    for k, ldx, ldy, dt, sc in [(0, 4, 4, 0, None), (65, 65, 65, 0, None), (4, 3, 4, 0, None),
                                (4, 4, 2, 0, None), (4, 4, 4, 7, None), (4, 4, 4, 2, None),
                                (4, 4, 4, 0, fake)]:
        assert L.spmm_run(h.ptr, fake, k, ldx, dt, sc, fake, ldy, None) == pk.SPMM_EINVAL
    assert L.spmm_run(h.ptr, None, 4, 4, 0, None, fake, 4, None) == pk.SPMM_EINVAL
    h.close()


GEOMS = [dict(), dict(tile_rows=16, tile_cols=32), dict(tile_rows=1, tile_cols=1),
         dict(tile_rows=100, tile_cols=256, item_nnz=64), dict(tile_rows=4096, tile_cols=65536, item_nnz=1)]


@pytest.mark.parametrize("keep_order", [False, True])
@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("variant", range(pk.SPMM_NUM_VARIANTS))
def test_encode_decode_roundtrip(geom, variant, keep_order):
    rp, col = synth.rmat_csr(11, 8, seed=3)
    h = pk.spmm_build_tiles(rp, col, fixed_variant=variant, keep_order=keep_order, **geom)
    drp, dcol = pk.spmm_decode_tiles(h, col.shape[0])
    assert np.array_equal(drp, rp) and np.array_equal(dcol, col)
    st = pk.spmm_get_stats(h)
    assert st["nnz"] == col.shape[0]
    assert sum(st["variant_nnz"]) == col.shape[0]
    assert st["variant_nnz"][variant] == col.shape[0]
    h.close()


def test_encode_decode_weighted_rectangular_ragged():
    n_rows, n_cols = 1000, 3001
    d = synth.draws(synth.stream_key(9, 12), 0, n_rows * 6)
    rows = np.repeat(np.arange(n_rows), 6)
    cols = (d % np.uint64(n_cols)).astype(np.int64)
    pairs = np.unique(rows * n_cols + cols)
    r, c = pairs // n_cols, pairs % n_cols
    rp = np.zeros(n_rows + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp)
    col = c.astype(np.int32)
    val = synth.uniform(col.shape[0], 1, seed=3)[:, 0]
    for v in range(pk.SPMM_NUM_VARIANTS):
        h = pk.spmm_build_tiles(rp, col, val, n_cols=n_cols, tile_rows=37, tile_cols=512,
                                fixed_variant=v, item_nnz=300)
        drp, dcol, dval = pk.spmm_decode_tiles(h, col.shape[0], weighted=True)
        assert np.array_equal(drp, rp) and np.array_equal(dcol, col) and np.array_equal(dval, val)
        h.close()


def test_empty_matrix_and_empty_rows():
    rp = np.zeros(11, np.int64)
    h = pk.spmm_build_tiles(rp, np.zeros(0, np.int32))
    st = pk.spmm_get_stats(h)
    assert st["nnz"] == 0 and st["n_tiles"] == 0
    drp, dcol = pk.spmm_decode_tiles(h, 0)
    assert np.array_equal(drp, rp)
    h.close()
    h = pk.spmm_build_tiles(np.zeros(1, np.int64), np.zeros(0, np.int32))
    h.close()


def test_tile_stats_match_definition():
    rp, col = synth.rmat_csr(12, 8, seed=2)
    n = 1 << 12
    h, w = 64, 128
    rows = np.repeat(np.arange(n), np.diff(rp))
    indeg = np.bincount(col, minlength=n)
    rank = np.empty(n, np.int64)
    rank[np.lexsort((np.arange(n), -indeg))] = np.arange(n)   # by (-in-degree, id)
    outdeg = np.diff(rp)
    rrank = np.empty(n, np.int64)
    rrank[np.lexsort((np.arange(n), -outdeg))] = np.arange(n)  # by (-out-degree, id)
    for keep, r, c in ((True, rows, col.astype(np.int64)), (False, rrank[rows], rank[col])):
        hd = pk.spmm_build_tiles(rp, col, tile_rows=h, tile_cols=w, keep_order=keep)
        st = pk.spmm_get_stats(hd)
        tiles = (r // h) * (n // w) + c // w
        assert st["n_tiles"] == np.unique(tiles).size
        assert st["sum_nnr"] == np.unique(tiles * n + r).size
        assert st["sum_nnc"] == np.unique(tiles * n + c).size
        hd.close()


@pytest.mark.parametrize("t", [1, 7, 64, 16384])
def test_model_tiles_and_paper_formula(t):
    rp, col = synth.rmat_csr(12, 8, seed=4, symmetrize=True)
    n = 1 << 12
    T, R, C = pk.spmm_model_tiles(rp, col, t)
    rows = np.repeat(np.arange(n), np.diff(rp))
    nstrip = (n + t - 1) // t
    tile = (rows // t) * nstrip + col // t
    assert T == np.unique(tile).size
    assert R == np.unique(tile * n + rows).size
    assert C == np.unique(tile * n + col).size
    # S_SCSR / S_DCSC within the paper's bound when nnr ~ nnc (symmetric A)
    r = oracle.scsr_bytes(R, col.shape[0], 0) / oracle.dcsc_bytes(C, col.shape[0], 0)
    assert 0.4 <= r < 1.0 or R != C


def test_timing_window_without_runs():
    rp, col = synth.small_random_csr(50, 0.1, 3)
    h = pk.spmm_build_tiles(rp, col)
    pk.spmm_timing_begin(h)
    assert pk.spmm_timing_end(h) == (0.0, 0)
    assert pk.spmm_timing_end(h) == (0.0, 0)   # ending again: still empty
    h.close()
    L = pk.load_library()
    assert L.spmm_timing_begin(None) == pk.SPMM_EINVAL
    assert L.spmm_timing_end(None, None, None) == pk.SPMM_EINVAL


def test_read_probe_rejects_bad_arguments():
    L = pk.load_library()
    assert L.spmm_read_probe(None, 16, None, None) == pk.SPMM_EINVAL
    assert L.spmm_read_probe(16, 15, 16, None) == pk.SPMM_EINVAL     # not a multiple of 16
    assert L.spmm_read_probe(8, 16, 16, None) == pk.SPMM_EINVAL      # misaligned


def _transpose_ref(rp, col, val, n_cols):
    rows = np.repeat(np.arange(rp.shape[0] - 1, dtype=np.int64), np.diff(rp))
    order = np.lexsort((rows, col.astype(np.int64)))
    tp = np.concatenate([[0], np.cumsum(np.bincount(col, minlength=n_cols))]).astype(np.int64)
    return tp, rows[order].astype(np.int32), None if val is None else val[order]


@pytest.mark.parametrize("weighted", [False, True])
def test_transposed_build_decodes_to_the_transpose(weighted):
    rng = np.random.default_rng(3)
    n, m = 700, 1300                                  # rectangular: A is n x m
    dense = (rng.random((n, m)) < 0.01)
    rp = np.concatenate([[0], np.cumsum(dense.sum(1))]).astype(np.int64)
    col = np.nonzero(dense)[1].astype(np.int32)
    val = rng.random(col.shape[0]).astype(np.float32) + 0.5 if weighted else None
    h = pk.spmm_build_tiles(rp, col, val, n_cols=m, transpose=True, tile_rows=32, tile_cols=256)
    assert (h.n_rows, h.n_cols) == (m, n)
    st = pk.spmm_get_stats(h)
    assert (st["n_rows"], st["n_cols"], st["nnz"]) == (m, n, col.shape[0])
    tp, tc, tv = _transpose_ref(rp, col, val, m)
    got = pk.spmm_decode_tiles(h, col.shape[0], weighted=weighted)
    assert np.array_equal(got[0], tp) and np.array_equal(got[1], tc)
    if weighted:
        assert np.array_equal(got[2], tv)
    h.close()
    # the R-MAT graph: the transpose of the transpose is the graph
    rp2, col2 = synth.rmat_csr(12, 8, seed=6)
    ht = pk.spmm_build_tiles(rp2, col2, transpose=True)
    trp, tcol = pk.spmm_decode_tiles(ht, col2.shape[0])
    htt = pk.spmm_build_tiles(trp, tcol, transpose=True)
    rrp, rcol = pk.spmm_decode_tiles(htt, col2.shape[0])
    assert np.array_equal(rrp, rp2) and np.array_equal(rcol, col2)
    ht.close()
    htt.close()


def test_transposed_build_checks_input():
    rp, col = synth.small_random_csr(20, 0.2, 1)
    bad = col.copy()
    bad[0] = 25
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_build_tiles(rp, bad, transpose=True)
    assert ei.value.status == pk.SPMM_EINVAL


def test_row_order_by_degree_and_empty_rows_untiled():
    """Default build: tile rows take the rows by descending out-degree and
    rows without entries are not tiled (they are zero-filled at run time);
    keep_row_order (or keep_order) tiles every row in the given order.  Both
    decode back to the input CSR."""
    rp, col = synth.rmat_csr(13, 4, seed=3)
    n = rp.shape[0] - 1
    live = int(np.count_nonzero(np.diff(rp)))
    assert live < n
    h = 32
    for opts, slabs in ((dict(), -(-live // h)), (dict(keep_row_order=True), -(-n // h)),
                        (dict(keep_order=True), -(-n // h))):
        hd = pk.spmm_build_tiles(rp, col, tile_rows=h, **opts)
        assert pk.spmm_get_stats(hd)["n_slabs"] == slabs, opts
        drp, dcol = pk.spmm_decode_tiles(hd, col.shape[0])
        assert np.array_equal(drp, rp) and np.array_equal(dcol, col), opts
        hd.close()


def test_csr_format_round_trip_and_limits():
    """The untiled CSR store (V-csr baseline) decodes to the input; it takes
    binary matrices in HBM only."""
    rp, col = synth.rmat_csr(13, 16, seed=12)
    for keep in (False, True):
        h = pk.spmm_build_tiles(rp, col, format=pk.SPMM_FORMAT_CSR, keep_order=keep)
        drp, dcol = pk.spmm_decode_tiles(h, col.shape[0])
        assert np.array_equal(drp, rp) and np.array_equal(dcol, col)
        assert pk.spmm_get_stats(h)["nnz"] == col.shape[0]
        h.close()
    val = np.ones(col.shape[0], np.float32)
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_build_tiles(rp, col, val, format=pk.SPMM_FORMAT_CSR)
    assert ei.value.status == pk.SPMM_EUNSUPPORTED
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_build_tiles(rp, col, format=pk.SPMM_FORMAT_CSR, place=pk.SPMM_PLACE_PINNED_HOST)
    assert ei.value.status == pk.SPMM_EUNSUPPORTED
