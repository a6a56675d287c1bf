"""Streamed (semi-external) SpMM: the tile payload lives in pinned host
memory and is copied per group of work items into a device ring.  Same
kernels and work items as the in-HBM path, so results must be bit-identical
to spmm_run on a device-placed handle built with the same options."""
import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth

pytestmark = pytest.mark.gpu


def _stream_y(h, X, fill=float("nan")):
    import torch
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.full((h.n_rows, X.shape[1]), fill, device="cuda")
    comp = torch.cuda.Stream()
    copy = torch.cuda.Stream()
    comp.wait_stream(torch.cuda.current_stream())
    pk.spmm_stream_run(h, Xd, Yd, compute=comp, copy=copy)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


def _dev_y(h, X):
    import torch
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.full((h.n_rows, X.shape[1]), float("nan"), device="cuda")
    pk.spmm_run(h, Xd, Yd)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


@pytest.mark.parametrize("opts", [dict(stream_kib=64, ring_depth=2),
                                  dict(stream_kib=256, ring_depth=3, item_nnz=2000),
                                  dict(stream_kib=1 << 20, ring_depth=2)])
def test_stream_matches_device_bit_exact(opts):
    rp, col = synth.rmat_csr(16, 16, seed=1)
    n = rp.shape[0] - 1
    hs = pk.spmm_build_tiles(rp, col, place=pk.SPMM_PLACE_PINNED_HOST, **opts)
    hd = pk.spmm_build_tiles(rp, col, **opts)
    for k in (1, 4, 48):
        Xi = synth.int07(n, k, seed=2)
        Ys = _stream_y(hs, Xi)
        assert np.array_equal(Ys.astype(np.float64), oracle.spmm(rp, col, None, Xi))
        Xu = synth.uniform(n, k, seed=3)
        assert np.array_equal(_stream_y(hs, Xu), _dev_y(hd, Xu))
    # running twice reuses the ring and the split-row counters
    Xu = synth.uniform(n, 4, seed=4)
    assert np.array_equal(_stream_y(hs, Xu), _stream_y(hs, Xu))


def test_stream_weighted_and_wrong_placement():
    rp, col = synth.rmat_csr(14, 8, seed=5, symmetrize=True)
    n = rp.shape[0] - 1
    val = synth.lognormal_weights(rp, col, seed=3)
    hs = pk.spmm_build_tiles(rp, col, val, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=32, ring_depth=2)
    X = synth.uniform(n, 8, seed=2)
    assert oracle.frob_rel_err(_stream_y(hs, X), oracle.spmm(rp, col, val, X)) <= 1e-6
    import torch
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_run(hs, torch.from_numpy(X).cuda(), torch.empty((n, 8), device="cuda"))
    assert ei.value.status == pk.SPMM_ESTATE


@pytest.mark.parametrize("weighted", [False, True])
def test_host_resident_column_blocks_equal_in_hbm(weighted):
    """X and Y in pinned host memory, columns in blocks: identical to the
    in-HBM product for every block width (A re-streamed per block)."""
    import torch
    rp, col = synth.rmat_csr(14, 12, seed=9)
    n = rp.shape[0] - 1
    val = synth.lognormal_weights(rp, col, seed=synth.SEED_WEIGHT) if weighted else None
    hd = pk.spmm_build_tiles(rp, col, val)
    hs = pk.spmm_build_tiles(rp, col, val, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=64)
    k = 7
    Xh = torch.from_numpy(synth.uniform(n, 9, seed=2)).pin_memory()[:, 1:1 + k]   # strided host view
    ref = torch.empty((n, k), device="cuda")
    pk.spmm_run(hd, Xh.cuda(), ref)
    torch.cuda.synchronize()
    ref = ref.cpu()
    for cb in (1, 3, 7):
        Yh = torch.full((n, k + 2), float("nan")).pin_memory()
        pk.spmm_stream_run_host(hs, Xh, Yh[:, :k], cb)
        assert torch.equal(Yh[:, :k], ref), cb
        assert torch.isnan(Yh[:, k:]).all()      # columns beyond k untouched
        # blocked layout: each block of columns contiguous, blocks back to back
        blocks = [(c0, min(cb, k - c0)) for c0 in range(0, k, cb)]
        Xb = torch.cat([Xh[:, c0:c0 + w].reshape(-1) for c0, w in blocks]).pin_memory()
        Yb = torch.full((n * k,), float("nan")).pin_memory()
        pk.spmm_stream_run_host(hs, Xb, Yb, cb, k=k, blocked=True)
        off = 0
        for c0, w in blocks:
            assert torch.equal(Yb[off:off + n * w].reshape(n, w), ref[:, c0:c0 + w]), (cb, c0)
            off += n * w
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_stream_run_host(hd, Xh, Yh[:, :k], 2)
    assert ei.value.status == pk.SPMM_ESTATE
    with pytest.raises(pk.SpmmError):
        pk.spmm_stream_run_host(hs, Xh, Yh[:, :k], 8)     # more columns per block than k
    hd.close()
    hs.close()


@pytest.mark.parametrize("weighted", [False, True])
def test_host_resident_column_blocks_match_oracle(weighted):
    """X and Y in pinned host memory, processed in column blocks, against the
    oracle: integer X exact, FP32 X within 1e-6 (relative Frobenius)."""
    import torch
    rp, col = synth.rmat_csr(14, 12, seed=9)
    n = rp.shape[0] - 1
    val = synth.lognormal_weights(rp, col, seed=synth.SEED_WEIGHT) if weighted else None
    hs = pk.spmm_build_tiles(rp, col, val, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=64, item_nnz=500)
    k = 6
    for X, exact in ((synth.int07(n, k, seed=2), not weighted), (synth.uniform(n, k, seed=2), False)):
        ref = oracle.spmm(rp, col, val, X)
        Xh = torch.from_numpy(X).pin_memory()
        for cb in (1, 4, 6):
            Yh = torch.full((n, k), float("nan")).pin_memory()
            pk.spmm_stream_run_host(hs, Xh, Yh, cb)
            Y = Yh.numpy()
            if exact:
                assert np.array_equal(Y.astype(np.float64), ref), cb
            else:
                assert oracle.frob_rel_err(Y, ref) <= 1e-6, cb
    hs.close()


@pytest.mark.parametrize("weighted", [False, True])
def test_y_streamed_to_host(weighted):
    """A streamed from pinned host memory and Y streamed back to pinned host
    memory by tile-row groups: exact against the oracle for integer X on a
    binary A, within 1e-6 otherwise, bit-identical to the in-HBM product, and
    untouched outside the k columns of a strided Y."""
    import torch
    rp, col = synth.rmat_csr(15, 16, seed=11)
    n = rp.shape[0] - 1
    val = synth.lognormal_weights(rp, col, seed=synth.SEED_WEIGHT) if weighted else None
    opts = dict(keep_row_order=True, item_nnz=3000)
    hd = pk.spmm_build_tiles(rp, col, val, **opts)
    hs = pk.spmm_build_tiles(rp, col, val, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=64, ring_depth=2, **opts)
    comp, copy, out = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    for k in (1, 4, 33):
        for X, exact in ((synth.int07(n, k, seed=2), not weighted), (synth.uniform(n, k, seed=3), False)):
            Xd = torch.from_numpy(X).cuda()
            comp.wait_stream(torch.cuda.current_stream())
            Yh = torch.full((n, k + 2), float("nan")).pin_memory()
            pk.spmm_stream_run_yhost(hs, Xd, Yh[:, :k], compute=comp, copy=copy, out=out)
            Yc = torch.full((n, k), float("nan")).pin_memory()              # contiguous rows
            pk.spmm_stream_run_yhost(hs, Xd, Yc, compute=comp, copy=copy, out=out)
            out.synchronize()
            Y = Yh[:, :k].numpy()
            assert torch.isnan(Yh[:, k:]).all()
            assert np.array_equal(Yc.numpy(), Y)
            ref = oracle.spmm(rp, col, val, X)
            if exact:
                assert np.array_equal(Y.astype(np.float64), ref), k
            else:
                assert oracle.frob_rel_err(Y, ref) <= 1e-6, k
            assert np.array_equal(Y, _dev_y(hd, X)), k
    # calls queued back to back reuse the A and Y slots
    Xd = torch.from_numpy(synth.uniform(n, 4, seed=5)).cuda()
    ref = _dev_y(hd, synth.uniform(n, 4, seed=5))
    comp.wait_stream(torch.cuda.current_stream())
    outs = [torch.empty((n, 4)).pin_memory() for _ in range(3)]
    for Yo in outs:
        pk.spmm_stream_run_yhost(hs, Xd, Yo, compute=comp, copy=copy, out=out)
    out.synchronize()
    for Yo in outs:
        assert np.array_equal(Yo.numpy(), ref)
    hd.close()
    hs.close()
    # rows in degree order do not form one Y range per group
    hr = pk.spmm_build_tiles(rp, col, val, place=pk.SPMM_PLACE_PINNED_HOST)
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_stream_run_yhost(hr, Xd, torch.empty((n, 4)).pin_memory(), compute=comp, copy=copy, out=out)
    assert ei.value.status == pk.SPMM_EUNSUPPORTED
    hr.close()


def test_back_to_back_streamed_calls_identical():
    """Consecutive streamed calls, enqueued without host synchronisation,
    reuse the ring slots: each call's first copies must wait for the previous
    call's last kernels (the ordering tests/test_stream_plan_cpu.py checks on
    the CPU).  Every call's result must match the in-HBM product."""
    import torch
    rp, col = synth.rmat_csr(15, 16, seed=10)
    n = rp.shape[0] - 1
    hd = pk.spmm_build_tiles(rp, col)
    hs = pk.spmm_build_tiles(rp, col, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=32, ring_depth=2)
    X = torch.from_numpy(synth.uniform(n, 4, seed=2)).cuda()
    ref = torch.empty((n, 4), device="cuda")
    pk.spmm_run(hd, X, ref)
    copy = torch.cuda.Stream()
    outs = [torch.empty((n, 4), device="cuda") for _ in range(4)]
    for Y in outs:
        pk.spmm_stream_run(hs, X, Y, copy=copy)
    torch.cuda.synchronize()
    for Y in outs:
        assert torch.equal(Y, ref)
    hd.close()
    hs.close()


@pytest.mark.parametrize("clustered", [True, False])
def test_sbm_graphs_exact_in_hbm_and_streamed(clustered):
    """Stochastic-block-model inputs of the clustering study, with the given
    column order kept and with the default relabelling: integer X exact
    against the oracle, streamed Y identical to in-HBM Y."""
    rp, col = synth.sbm_csr(1 << 14, 64, 1 << 19, 0.9, clustered=clustered, seed=6)
    n = rp.shape[0] - 1
    X = synth.int07(n, 4, seed=7)
    ref = oracle.spmm(rp, col, None, X)
    for keep in (True, False):
        hd = pk.spmm_build_tiles(rp, col, keep_order=keep)
        hs = pk.spmm_build_tiles(rp, col, keep_order=keep, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=64)
        Yd = _dev_y(hd, X)
        assert np.array_equal(Yd.astype(np.float64), ref), keep
        assert np.array_equal(_stream_y(hs, X), Yd), keep
        hd.close()
        hs.close()
