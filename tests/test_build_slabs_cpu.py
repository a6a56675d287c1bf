"""Slab-wise build (spmm_build_begin / append_rows / end): the tile store
built from blocks of rows decodes to the input CSR, matches a one-shot build
of the same row and column order, and the call order is enforced."""
import ctypes

import numpy as np
import pytest

import paper_1602_02864_amd as pk
import synth


def _blocks(rp, col, val, sizes):
    """Yield (row0, local row_ptr, cols, vals) for consecutive row blocks."""
    n = rp.shape[0] - 1
    r0, i = 0, 0
    while r0 < n:
        nr = min(sizes[i % len(sizes)], n - r0)
        a, b = rp[r0], rp[r0 + nr]
        yield r0, rp[r0:r0 + nr + 1] - a, col[a:b], None if val is None else val[a:b]
        r0 += nr
        i += 1


def _slab_build(rp, col, val, sizes, **opts):
    n = rp.shape[0] - 1
    h = pk.spmm_build_begin(n, **opts)
    for r0, lrp, c, v in _blocks(rp, col, val, sizes):
        pk.spmm_build_append_rows(h, r0, lrp, c, v)
    pk.spmm_build_end(h)
    return h


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("sizes", [[1000], [777, 1, 64, 5000], [1 << 20]])
def test_slab_build_decodes_to_input(weighted, sizes):
    rp, col = synth.rmat_csr(13, 8, seed=21)
    val = synth.lognormal_weights(rp, col, seed=3) if weighted else None
    for opts in (dict(), dict(keep_row_order=True), dict(tile_rows=7, item_nnz=50)):
        h = _slab_build(rp, col, val, sizes, **opts)
        out = pk.spmm_decode_tiles(h, col.shape[0], weighted=weighted)
        assert np.array_equal(out[0], rp) and np.array_equal(out[1], col), opts
        if weighted:
            assert np.array_equal(out[2], val)
        st = pk.spmm_get_stats(h)
        assert st["nnz"] == col.shape[0]
        h.close()


def test_slab_build_in_given_order_equals_one_shot():
    """With rows and columns in the given order the tiling does not depend
    on how the rows were cut into blocks."""
    rp, col = synth.rmat_csr(13, 8, seed=22)
    one = pk.spmm_build_tiles(rp, col, keep_order=True)
    ref = pk.spmm_get_stats(one)
    for sizes in ([100], [33, 4000], [1 << 20]):
        h = _slab_build(rp, col, None, sizes, keep_row_order=True)
        st = pk.spmm_get_stats(h)
        for key in ("n_tiles", "n_slabs", "sum_nnr", "sum_nnc", "n_items", "n_parts", "blob_bytes"):
            assert st[key] == ref[key], (sizes, key)
        h.close()
    one.close()


def test_slab_build_orders_rows_by_degree_within_blocks():
    """The default slab-wise build tiles only rows with entries, by
    descending degree within each block: a block holding the whole matrix
    gives the one-shot build's row tiling (same tile statistics when the
    columns keep their order in both)."""
    rp, col = synth.rmat_csr(12, 8, seed=23)
    h = _slab_build(rp, col, None, [1 << 20])
    one = pk.spmm_build_tiles(rp, col, keep_row_order=False, keep_order=False)
    live = int(np.count_nonzero(np.diff(rp)))
    st = pk.spmm_get_stats(h)
    assert st["n_slabs"] == -(-live // 32)
    assert pk.spmm_get_stats(one)["n_slabs"] == st["n_slabs"]
    h.close()
    one.close()


def test_slab_build_call_order_enforced():
    rp, col = synth.rmat_csr(10, 8, seed=24)
    n = rp.shape[0] - 1
    h = pk.spmm_build_begin(n)
    blocks = list(_blocks(rp, col, None, [300]))
    pk.spmm_build_append_rows(h, *blocks[0][:3])
    with pytest.raises(pk.SpmmError) as ei:          # skips a block
        pk.spmm_build_append_rows(h, *blocks[2][:3])
    assert ei.value.status == pk.SPMM_EINVAL
    with pytest.raises(pk.SpmmError) as ei:          # rows missing
        pk.spmm_build_end(h)
    assert ei.value.status == pk.SPMM_ESTATE
    with pytest.raises(pk.SpmmError) as ei:          # not usable before the end
        pk.spmm_get_stats(h)
    assert ei.value.status == pk.SPMM_ESTATE
    for b in blocks[1:]:
        pk.spmm_build_append_rows(h, *b[:3])
    pk.spmm_build_end(h)
    with pytest.raises(pk.SpmmError) as ei:          # already ended
        pk.spmm_build_end(h)
    assert ei.value.status == pk.SPMM_ESTATE
    drp, dcol = pk.spmm_decode_tiles(h, col.shape[0])
    assert np.array_equal(drp, rp) and np.array_equal(dcol, col)
    h.close()
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_build_begin(n, transpose=True)
    assert ei.value.status == pk.SPMM_EUNSUPPORTED


def test_slab_build_keeps_no_tile_store():
    """Each block is encoded as it is cut and its tiles are dropped: every
    tile carries fixed_variant (HYBRID by default), and the per-tile
    selectors refuse the handle."""
    rp, col = synth.rmat_csr(12, 8, seed=25)
    for fv, want in ((-1, pk.SPMM_VAR_HYBRID), (pk.SPMM_VAR_COO, pk.SPMM_VAR_COO)):
        h = _slab_build(rp, col, None, [500, 3000], fixed_variant=fv)
        st = pk.spmm_get_stats(h)
        assert st["variant_tiles"][want] == st["n_tiles"] > 0
        for call in (lambda: pk.spmm_tile_features(h, 4), lambda: pk.spmm_get_variants(h),
                     lambda: pk.spmm_select_learned(h, np.zeros(pk.SPMM_MLP_PARAMS, np.float32), 4)):
            with pytest.raises(pk.SpmmError) as ei:
                call()
            assert ei.value.status == pk.SPMM_EUNSUPPORTED
        drp, dcol = pk.spmm_decode_tiles(h, col.shape[0])
        assert np.array_equal(drp, rp) and np.array_equal(dcol, col)
        h.close()
