"""Train the per-tile cost model on timings of generated graphs.

    python -m paper_1602_02864_amd.selector_train [--out DIR] [--quick]

Data: R-MAT graphs (a/b/c/d = .57/.19/.19/.05) at scales 18-25 with graph
seeds 11-15, 18, 19, 21 and 23, directed and symmetrised, edge factors 8-44 --
never seed 1 (the benchmark graphs) or 17 (the held-out graphs).  Each graph is tiled with the library's
default geometry (32-row tile rows, 65536-column strips).  For every graph,
column count k and X type, spmm_selector_collect times each variant on
every bucket of similar tiles; a training row is one tile: its 8 features
and, per variant, the log of its bucket's nanoseconds per tile.  At most
``--per-bucket`` tiles of a bucket are kept per collection, so large
buckets of tiny tiles do not crowd out the rare large tiles that carry most
of the time.

Training runs on the GPU (spmm_selector_train: minibatch Adam on the MSE).
A held-out graph (seed 17) measures the result: per (k, type), the time the
learned choice costs over the per-bucket optimum of the exhaustive timing
(the regret), next to the regret of each fixed variant; and whole SpMM runs
on it with each fixed variant, the autotuner and the learned choice.

Bucket timings see each bucket alone, repeated to fill the GPU; inside a
whole SpMM the variants' costs shift (other tiles share the caches and the
memory system).  Two corrections follow.  Calibration: for every graph and
setting, each fixed variant's whole SpMM is timed, and that variant's
bucket times are scaled by one factor so that they sum to the measured
time (the labels keep each bucket's relative cost within the variant).
Margin: the shipped weights keep the build default (HYBRID) unless another
variant is predicted at least a margin faster (folded into the output bias
of HYBRID); of the candidate --margins, the one whose learned choice gives
the fastest whole SpMMs (summed over k = 1..32) on the largest training
graph is shipped.

Writes DIR/selector_weights.npy (float32[SPMM_MLP_PARAMS]) and
DIR/selector_train.json (data, loss trace, held-out regrets).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1602_02864_amd as pk  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.npy")

# (scale, edge factor, graph seed, symmetrise)
TRAIN_GRAPHS = [(18, 16, 18, False), (19, 8, 19, True), (20, 16, 11, False), (21, 44, 12, False),
                (22, 8, 13, True), (21, 28, 14, True), (22, 44, 15, False), (24, 24, 21, False),
                (25, 44, 23, False)]
HELD_OUT = (22, 32, 17, False)
QUICK_GRAPHS = [(16, 16, 11, False), (17, 8, 13, True)]
QUICK_HELD_OUT = (17, 16, 17, False)
# (k, X type) pairs timed per graph
RUNS = [(1, pk.SPMM_X_F32), (4, pk.SPMM_X_F32), (16, pk.SPMM_X_F32), (32, pk.SPMM_X_F32),
        (64, pk.SPMM_X_F32), (16, pk.SPMM_X_BF16), (16, pk.SPMM_X_FP8_E4M3)]
DT_NAMES = {pk.SPMM_X_F32: "f32", pk.SPMM_X_BF16: "bf16", pk.SPMM_X_FP8_E4M3: "fp8"}


def log(msg: str) -> None:
    print(f"[selector {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def graph(scale, ef, seed, sym):
    import synth
    return synth.rmat_csr(scale, ef, seed=seed, symmetrize=sym)


def collect_rows(h, k, dt, per_bucket, rng):
    """Features of (at most per_bucket) tiles per bucket, with their buckets'
    ns per tile for every variant."""
    b, ns = pk.spmm_selector_collect(h, k, dt)
    f = pk.spmm_tile_features(h, k, dt)
    keep = []
    for q in range(ns.shape[0]):
        idx = np.flatnonzero(b == q)
        if idx.size > per_bucket:
            idx = rng.choice(idx, per_bucket, replace=False)
        keep.append(idx)
    keep = np.concatenate(keep) if keep else np.zeros(0, np.int64)
    return f[keep], ns[b[keep]], b, ns


def _x_input(X, dt):
    """X (device FP32) in the X type dt: the tensor and its column scales."""
    import torch
    if dt == pk.SPMM_X_F32:
        return X, None
    if dt == pk.SPMM_X_BF16:
        Xq = torch.empty(X.shape, dtype=torch.bfloat16, device=X.device)
        pk.spmm_quantize_x(X, Xq, dt)
        return Xq, None
    Xq = torch.empty(X.shape, dtype=torch.uint8, device=X.device)
    cs = torch.empty(X.shape[1], dtype=torch.float32, device=X.device)
    pk.spmm_quantize_x(X, Xq, dt, col_scale=cs)
    return Xq, cs


def _timed(h, X, Y, dt, cs, reps):
    """Mean ms of one SpMM over reps launches after a warm-up."""
    import torch
    pk.spmm_run(h, X, Y, dtype=dt, col_scale=cs)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        pk.spmm_run(h, X, Y, dtype=dt, col_scale=cs)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def whole_times(h, settings, reps=10):
    """ms of a whole SpMM with every tile in variant v, for each (k, X type)
    setting and variant: float64[len(settings), V].  The handle's variants
    are left as HYBRID."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    st = pk.spmm_get_stats(h)
    T, n, m = st["n_tiles"], st["n_rows"], st["n_cols"]
    xs = {}
    for k, dt in settings:
        if k not in xs:
            xs[k] = torch.from_numpy(synth.uniform(m, k, seed=2)).to(dev)
    out = np.zeros((len(settings), pk.SPMM_NUM_VARIANTS))
    for v in range(pk.SPMM_NUM_VARIANTS):
        pk.spmm_set_variants(h, np.full(T, v, np.uint8))
        for i, (k, dt) in enumerate(settings):
            Xin, cs = _x_input(xs[k], dt)
            Y = torch.empty((n, k), device=dev)
            out[i, v] = _timed(h, Xin, Y, dt, cs, reps)
            del Xin, Y
    pk.spmm_set_variants(h, np.full(T, pk.SPMM_VAR_HYBRID, np.uint8))
    return out


def calibration(b, ns, whole_ms):
    """Per-variant factor that scales the bucket times of one (graph,
    setting) to the variant's measured whole-SpMM time: the summed bucket
    time of every tile in variant v is sum_t ns[b[t], v]."""
    pred_ns = ns[b].sum(axis=0).astype(np.float64)
    return whole_ms * 1e6 / np.maximum(pred_ns, 1e-9)


def regrets(h, params, k, dt, keep=None):
    """Time over the per-bucket optimum: learned choice and each fixed variant."""
    b, ns = pk.spmm_selector_collect(h, k, dt)
    f = pk.spmm_tile_features(h, k, dt)
    if keep is not None:
        # distinct (features, bucket) rows with their tile counts
        u, inv, cnt = np.unique(np.concatenate([f, b[:, None].astype(np.float32)], axis=1), axis=0,
                                return_inverse=True, return_counts=True)
        keep[f"k{k}_{DT_NAMES[dt]}"] = (u, cnt, ns)
    import torch
    dev = torch.device("cuda:0")
    ch = torch.empty(f.shape[0], dtype=torch.uint8, device=dev)
    pk.spmm_mlp_predict(torch.from_numpy(params).to(dev), torch.from_numpy(f).to(dev), None, ch)
    torch.cuda.synchronize()
    c = ch.cpu().numpy().astype(np.int64)
    best = ns.min(axis=1)[b].sum()
    out = {"learned": float(ns[b, c].sum() / best - 1.0)}
    for v, name in enumerate(pk.VARIANT_NAMES):
        out[name] = float(ns[b, v].sum() / best - 1.0)
    return out


B3_OFFSET = 8 * 64 + 64 + 64 * 64 + 64 + 64 * pk.SPMM_NUM_VARIANTS   # output-layer bias (spmm.h layout)
FULL_KS = (1, 2, 4, 8, 16, 32)


def with_margin(params, margin):
    """The weights with HYBRID favoured by the margin: a tile leaves HYBRID
    only where another variant is predicted >= (1 + margin) times faster."""
    p = params.astype(np.float32).copy()
    p[B3_OFFSET + pk.SPMM_VAR_HYBRID] -= np.float32(np.log1p(margin))
    return p


def margin_sweep(h, params, margins, reps=10):
    """Whole-SpMM ms summed over FULL_KS (FP32 X) on handle h: every tile
    HYBRID, and the learned choice at each margin."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    st = pk.spmm_get_stats(h)
    T, n, m = st["n_tiles"], st["n_rows"], st["n_cols"]
    xs = {k: torch.from_numpy(synth.uniform(m, k, seed=2)).to(dev) for k in FULL_KS}
    ys = {k: torch.empty((n, k), device=dev) for k in FULL_KS}
    tot = {"hybrid": 0.0, **{str(mg): 0.0 for mg in margins}}
    pk.spmm_set_variants(h, np.full(T, pk.SPMM_VAR_HYBRID, np.uint8))
    for k in FULL_KS:
        tot["hybrid"] += _timed(h, xs[k], ys[k], pk.SPMM_X_F32, None, reps)
    ch = torch.empty(T, dtype=torch.uint8, device=dev)
    for k in FULL_KS:
        f = torch.from_numpy(pk.spmm_tile_features(h, k)).to(dev)
        for mg in margins:
            pk.spmm_mlp_predict(torch.from_numpy(with_margin(params, mg)).to(dev), f, None, ch)
            torch.cuda.synchronize()
            pk.spmm_set_variants(h, ch.cpu().numpy())
            tot[str(mg)] += _timed(h, xs[k], ys[k], pk.SPMM_X_F32, None, reps)
        del f
    return {a: round(v, 4) for a, v in tot.items()}


def full_runs(g, params, reps=20):
    """Whole-SpMM times on graph g (ms, FP32 X) for each fixed variant, the
    exhaustive autotuner and the learned choice, per k and summed."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    rp, col = graph(*g)
    n = rp.shape[0] - 1
    h = pk.spmm_build_tiles(rp, col, validate=False)
    T = pk.spmm_get_stats(h)["n_tiles"]
    pd = torch.from_numpy(params).to(dev)

    def t(X, Y):
        pk.spmm_run(h, X, Y)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            pk.spmm_run(h, X, Y)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    per_k = {}
    for k in FULL_KS:
        X = torch.from_numpy(synth.uniform(n, k, seed=2)).to(dev)
        Y = torch.empty((n, k), device=dev)
        row = {}
        for v, name in enumerate(pk.VARIANT_NAMES):
            pk.spmm_set_variants(h, np.full(T, v, np.uint8))
            row[name] = t(X, Y)
        pk.spmm_autotune(h, k)
        row["autotune"] = t(X, Y)
        f = torch.from_numpy(pk.spmm_tile_features(h, k)).to(dev)
        ch = torch.empty(f.shape[0], dtype=torch.uint8, device=dev)
        pk.spmm_mlp_predict(pd, f, None, ch)
        torch.cuda.synchronize()
        pk.spmm_set_variants(h, ch.cpu().numpy())
        row["learned"] = t(X, Y)
        per_k[str(k)] = {a: round(v, 4) for a, v in row.items()}
    h.close()
    names = list(per_k[str(FULL_KS[0])])
    return {"graph": list(g), "per_k": per_k,
            "sum_ms": {a: round(sum(per_k[str(k)][a] for k in FULL_KS), 4) for a in names}}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=os.path.dirname(WEIGHTS))
    ap.add_argument("--quick", action="store_true", help="small graphs (a functional run)")
    ap.add_argument("--per-bucket", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=1200)
    ap.add_argument("--margins", default="0.05,0.1,0.2,0.3",
                    help="candidate margins: keep the build default (HYBRID) unless another variant is predicted "
                         "at least this much faster (folded into the output bias of the shipped weights); with "
                         "several, the one with the fastest whole SpMMs on the largest training graph is shipped")
    ap.add_argument("--no-calibrate", dest="calibrate", action="store_false",
                    help="train on the raw bucket timings (no scaling to whole-SpMM times)")
    ap.add_argument("--dump", action="store_true",
                    help="also write the training rows and held-out timing tables (.npz)")
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.init()
    rng = np.random.default_rng(args.seed)
    graphs = QUICK_GRAPHS if args.quick else TRAIN_GRAPHS
    held = QUICK_HELD_OUT if args.quick else HELD_OUT
    F, Y, meta = [], [], []
    for g in graphs:
        t0 = time.perf_counter()
        rp, col = graph(*g)
        h = pk.spmm_build_tiles(rp, col, validate=False)
        T = pk.spmm_get_stats(h)["n_tiles"]
        got = []
        for k, dt in RUNS:
            f, nsr, b, ns = collect_rows(h, k, dt, args.per_bucket, rng)
            got.append((f, nsr, b, ns))
            log(f"graph {g} k={k} {DT_NAMES[dt]}: {ns.shape[0]} buckets, {f.shape[0]} rows")
        # in-context calibration: each variant's bucket times of this graph
        # and setting are scaled to sum to its measured whole-SpMM time
        whole = whole_times(h, RUNS) if args.calibrate else None
        for i, ((k, dt), (f, nsr, b, ns)) in enumerate(zip(RUNS, got)):
            c = calibration(b, ns, whole[i]) if whole is not None else np.ones(pk.SPMM_NUM_VARIANTS)
            F.append(f)
            Y.append(np.log(np.maximum(nsr * c[None, :], 1e-3)).astype(np.float32))
            meta.append({"graph": g, "k": k, "x": DT_NAMES[dt], "tiles": T, "buckets": int(ns.shape[0]),
                         "rows": int(f.shape[0]), "whole_ms": None if whole is None else [round(x, 4) for x in whole[i]],
                         "calibration": [round(float(x), 4) for x in c]})
            if whole is not None:
                log(f"graph {g} k={k} {DT_NAMES[dt]}: whole ms " + ", ".join(
                    f"{nm}={t:.3f}" for nm, t in zip(pk.VARIANT_NAMES, whole[i])) +
                    "; calibration " + ", ".join(f"{x:.3f}" for x in c))
        if g == graphs[-1]:
            h_last = h          # the largest training graph: kept for the margin choice
        else:
            h.close()
        log(f"graph {g} done in {time.perf_counter() - t0:.1f}s")
    F = np.concatenate(F)
    Y = np.concatenate(Y)
    log(f"training on {F.shape[0]} rows")
    t0 = time.perf_counter()
    params, trace = pk.spmm_selector_train(F, Y, epochs=args.epochs, batch=1024, lr=1e-3, seed=args.seed)
    t_train = time.perf_counter() - t0
    log(f"trained in {t_train:.1f}s: loss {trace[0]:.4f} -> {trace[-1]:.4f}")
    rp, col = graph(*held)
    h = pk.spmm_build_tiles(rp, col, validate=False)
    held_res = []
    held_tables = {} if args.dump else None
    for k, dt in RUNS:
        r = regrets(h, params, k, dt, held_tables)
        held_res.append({"k": k, "x": DT_NAMES[dt], "regret": r})
        log(f"held-out k={k} {DT_NAMES[dt]}: " + ", ".join(f"{a}={v * 100:.1f}%" for a, v in r.items()))
    h.close()
    # the margin: chosen by whole SpMM runs on the largest training graph
    margins = [float(x) for x in args.margins.split(",") if x.strip()]
    sweep = None
    if len(margins) > 1:
        sweep = margin_sweep(h_last, params, margins)
        margin = min(margins, key=lambda mg: (sweep[str(mg)], -mg))
        log(f"margin sweep on {graphs[-1]} (ms, sum over k): " + ", ".join(f"{a}={v:.3f}" for a, v in sweep.items()) +
            f" -> margin {margin}")
    else:
        margin = margins[0] if margins else 0.0
    h_last.close()
    shipped = with_margin(params, margin)
    full = full_runs(held, shipped)
    log("held-out full SpMM runs (ms, sum over k): " + ", ".join(f"{a}={v:.3f}" for a, v in full["sum_ms"].items()))
    os.makedirs(args.out, exist_ok=True)
    np.save(os.path.join(args.out, "selector_weights.npy"), shipped)
    with open(os.path.join(args.out, "selector_train.json"), "w") as fh:
        json.dump({"graphs": [list(g) for g in graphs], "held_out": list(held), "runs": meta,
                   "rows": int(F.shape[0]), "epochs": args.epochs, "seed": args.seed,
                   "train_s": round(t_train, 2), "loss_trace": [float(x) for x in trace],
                   "held_out_regret": held_res, "default_margin": margin, "margin_sweep": sweep,
                   "calibrated": bool(args.calibrate),
                   "held_out_full_runs": full}, fh, indent=1)
    if args.dump:
        np.savez_compressed(os.path.join(args.out, "selector_rows.npz"), feat=F, target=Y)
        np.savez_compressed(os.path.join(args.out, "selector_heldout.npz"),
                            **{f"{name}_{part}": arr for name, (u, cnt, ns) in held_tables.items()
                               for part, arr in (("featbucket", u), ("count", cnt), ("ns", ns))})
    log(f"wrote {args.out}/selector_weights.npy")
    return 0


if __name__ == "__main__":
    sys.exit(main())
