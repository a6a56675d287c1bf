"""CPU checks of the selection entry points that run on the host: tile
features against their definition, per-tile variants (set, get, re-encode,
decode), the He-uniform initial weights, and argument errors reported
before any device work."""
import numpy as np
import pytest

import paper_1602_02864_amd as pk
import synth


def _tile_table(rp, col, n, h, w):
    """Per tile (slab, strip): nnz, nnr, nnc, longest row, single-entry rows."""
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    c = col.astype(np.int64)
    nstrip = (n + w - 1) // w
    tile = (rows // h) * nstrip + c // w
    out = {}
    for t in np.unique(tile):
        sel = tile == t
        r = rows[sel]
        _, cnt = np.unique(r, return_counts=True)
        out[int(t)] = (int(sel.sum()), cnt.size, np.unique(c[sel]).size, int(cnt.max()), int((cnt == 1).sum()))
    return out


def _features(nnz, nnr, nnc, mx, single, k, xbytes):
    f32 = np.float32
    mean = f32(nnz) / f32(max(1, nnr))
    return np.array([np.log2(f32(1 + nnz)), np.log2(f32(1 + nnr)), np.log2(f32(1 + nnc)),
                     np.log2(f32(1 + mx)), f32(single) / f32(max(1, nnr)),
                     np.log2(f32(mx) / max(mean, f32(1))), np.log2(f32(k)), np.log2(f32(xbytes))],
                    dtype=np.float32)


@pytest.mark.parametrize("k,dt,xb", [(1, pk.SPMM_X_F32, 4), (16, pk.SPMM_X_BF16, 2), (64, pk.SPMM_X_FP8_E4M3, 1)])
def test_tile_features_match_definition(k, dt, xb):
    rp, col = synth.rmat_csr(11, 8, seed=3)
    n = 1 << 11
    h, w = 64, 256
    hd = pk.spmm_build_tiles(rp, col, tile_rows=h, tile_cols=w, keep_order=True)
    got = pk.spmm_tile_features(hd, k, dt)
    ref = np.stack([_features(*v, k, xb) for v in _tile_table(rp, col, n, h, w).values()])
    assert got.shape == ref.shape
    # tiles are compared as multisets of feature rows (same content, any order)
    g = got[np.lexsort(got.T[::-1])]
    r = ref[np.lexsort(ref.T[::-1])]
    np.testing.assert_allclose(g, r, rtol=2e-6, atol=2e-6)
    hd.close()


def test_set_variants_reencodes_same_matrix():
    rp, col = synth.rmat_csr(11, 8, seed=5)
    vals = synth.lognormal_weights(rp, col, seed=synth.SEED_WEIGHT)
    hd = pk.spmm_build_tiles(rp, col, vals, tile_rows=64, tile_cols=512)
    T = pk.spmm_get_stats(hd)["n_tiles"]
    assert np.all(pk.spmm_get_variants(hd) == pk.SPMM_VAR_HYBRID)
    v = (synth.int07(T, 1, seed=9)[:, 0].astype(np.int64) % pk.SPMM_NUM_VARIANTS).astype(np.uint8)
    pk.spmm_set_variants(hd, v)
    assert np.array_equal(pk.spmm_get_variants(hd), v)
    st = pk.spmm_get_stats(hd)
    assert st["variant_tiles"] == list(np.bincount(v, minlength=pk.SPMM_NUM_VARIANTS))
    drp, dcol, dval = pk.spmm_decode_tiles(hd, col.shape[0], weighted=True)
    assert np.array_equal(drp, rp) and np.array_equal(dcol, col) and np.array_equal(dval, vals)
    hd.close()


def test_set_variants_rejects_bad_values():
    rp, col = synth.small_random_csr(100, 0.05, 1)
    hd = pk.spmm_build_tiles(rp, col)
    T = pk.spmm_get_stats(hd)["n_tiles"]
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_set_variants(hd, np.full(T, pk.SPMM_NUM_VARIANTS, np.uint8))
    assert ei.value.status == pk.SPMM_EINVAL
    with pytest.raises(ValueError):
        pk.spmm_set_variants(hd, np.zeros(T + 1, np.uint8))
    hd.close()


def test_mlp_init_is_he_uniform():
    p = pk.spmm_mlp_init(11)
    assert p.shape == (pk.SPMM_MLP_PARAMS,) and pk.SPMM_MLP_PARAMS == 4996
    assert np.array_equal(p, pk.spmm_mlp_init(11))
    assert not np.array_equal(p, pk.spmm_mlp_init(12))
    H, F, V = pk.SPMM_MLP_HIDDEN, pk.SPMM_NUM_FEATURES, pk.SPMM_NUM_VARIANTS
    layers = [(pk.SPMM_MLP_OFF_W1, F, H), (pk.SPMM_MLP_OFF_W2, H, H), (pk.SPMM_MLP_OFF_W3, H, V)]
    for off, fi, fo in layers:
        w = p[off:off + fi * fo].astype(np.float64)
        lim = np.sqrt(6.0 / fi)
        assert np.all(np.abs(w) <= lim) and np.abs(w).max() > 0.9 * lim
        # U(-lim, lim): mean 0, variance lim^2 / 3 (4 standard errors)
        assert abs(w.mean()) < 4 * lim / np.sqrt(3 * w.size)
        assert abs(w.var() / (lim * lim / 3) - 1) < 4 * np.sqrt(0.8 / w.size)
    for off, n in [(pk.SPMM_MLP_OFF_B1, H), (pk.SPMM_MLP_OFF_B2, H), (pk.SPMM_MLP_OFF_B3, V)]:
        assert np.all(p[off:off + n] == 0)


def test_selection_argument_errors():
    rp, col = synth.small_random_csr(100, 0.05, 1)
    hd = pk.spmm_build_tiles(rp, col)
    for fn, args in [(pk.spmm_tile_features, (hd, 0)), (pk.spmm_tile_features, (hd, 65)),
                     (pk.spmm_tile_features, (hd, 4, 7))]:
        with pytest.raises(pk.SpmmError) as ei:
            fn(*args)
        assert ei.value.status == pk.SPMM_EINVAL
    hp = pk.spmm_build_tiles(rp, col, place=pk.SPMM_PLACE_PINNED_HOST)
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_autotune(hp, 4)
    assert ei.value.status == pk.SPMM_ESTATE
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_selector_collect(hp, 4)
    assert ei.value.status == pk.SPMM_ESTATE
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_selector_train(np.zeros((0, 8), np.float32), np.zeros((0, 4), np.float32))
    assert ei.value.status == pk.SPMM_EINVAL
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_mlp_adam(1, 1, 1, 1, 0)
    assert ei.value.status == pk.SPMM_EINVAL
    hd.close()
    hp.close()


def test_training_calibration_and_margin():
    """The training script's host arithmetic: calibrated bucket times of
    each variant sum to its whole-SpMM time, and the margin moves only
    HYBRID's output bias, by -log(1 + margin)."""
    from paper_1602_02864_amd.selector_train import B3_OFFSET, calibration, with_margin
    rng = np.random.default_rng(3)
    b = rng.integers(0, 5, 1000)
    ns = rng.uniform(10.0, 500.0, (5, pk.SPMM_NUM_VARIANTS))
    whole = np.array([3.0, 5.0, 2.5, 9.0])
    c = calibration(b, ns, whole)
    assert np.allclose((ns[b] * c[None, :]).sum(axis=0) * 1e-6, whole, rtol=1e-12)
    assert B3_OFFSET == pk.SPMM_MLP_OFF_B3
    p = pk.spmm_mlp_init(11)
    q = with_margin(p, 0.2)
    d = np.flatnonzero(q != p)
    assert list(d) == [pk.SPMM_MLP_OFF_B3 + pk.SPMM_VAR_HYBRID]
    assert np.isclose(q[d[0]] - p[d[0]], -np.log1p(0.2), rtol=1e-6)
