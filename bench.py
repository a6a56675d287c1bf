#!/usr/bin/env python3
"""SpMM benchmark on one MI355X.

Workload: directed R-MAT graph, scale 25 (33,554,432 vertices), edge factor 44
(1.476e9 samples, ~1.43e9 stored non-zeros after removing duplicates and
self-loops), a/b/c/d = .57/.19/.19/.05, binary A; X is FP32 uniform[0,1)
(seed 2) with k in {1, 2, 4, 8, 16, 32}.  One step = one SpMM Y = A X for
every k of the sweep; the reported value is the aggregate GFLOP/s of a step,
2 * nnz * sum(k) / step time, with X, Y and the tiles resident in HBM.

Tile variants: "learned" (default) lets the trained cost model pick each
tile's variant for each k (one resident handle per distinct assignment, all
built before the timed region); "plain" keeps the build default for every
tile.  The plain step is timed as well and reported beside the learned one.
The format comparison (on by default, --no-compare skips it) times every
fixed variant, the exhaustive autotuner and the learned choice per k on the
same tiles, the untiled CSR baseline (V-csr), and the original row and
column order.

Printed (one JSON line on stdout): the metric, the roofline of the dominant
kernel under the paper-tile byte model (16K x 16K tiles: A as SCSR, each
tile reading the X rows of its non-empty columns once, each Y row written
once), the HBM traffic of that kernel from committed counter runs when they
were taken on the current kernel source, and the CPU oracle timed on a
bounded sample of rows, whose results also give a sampled full-size parity
check of the GPU output.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
KERNEL_SRC = os.path.join(ROOT, "paper_1602_02864_amd", "csrc", "spmm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_spmm_items_rmat-s25-ef44.txt")


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def model_bytes(T: int, R: int, C: int, nnz: int, n: int, k: int, xbytes: int = 4) -> dict:
    """Paper-tile byte model for one SpMM (Section 3.2 sizes, 16K tiles)."""
    b_a = 2 * R + 2 * nnz + 8 * T
    b_x = C * k * xbytes
    b_y = n * k * 4
    return {"A": b_a, "X": b_x, "Y": b_y, "total": b_a + b_x + b_y,
            "floor": b_a + n * k * xbytes + b_y}


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kc: int):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on this kernel source and column chunk."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            vals[a.strip()] = b.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash() or vals.get("kc") != str(kc):
        return None
    try:
        return int(float(vals["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def time_step(runs, steps, warmup, stream):
    """runs: list of (k, callable).  Returns (ms per step, {k: ms per SpMM})."""
    import numpy as np
    import torch
    for _ in range(max(warmup, 1)):
        for _, fn in runs:
            fn()
    torch.cuda.synchronize()
    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)] for k, _ in runs}
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for s in range(steps):
        for k, fn in runs:
            a, b = ev[k][s]
            a.record(stream)
            fn()
            b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_k = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k]])) for k, _ in runs}
    return wall * 1e3 / steps, ms_k


def attainable_read_gbs(gib=16, reps=5):
    """Read rate of a plain streaming-read kernel over gib GiB (the HBM rate a
    simple kernel attains on this GPU, beside the 8 TB/s nominal)."""
    import torch

    import paper_1602_02864_amd as pk
    buf = torch.ones(gib << 28, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    pk.spmm_read_probe(buf, sink)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        pk.spmm_read_probe(buf, sink)
    b.record()
    torch.cuda.synchronize()
    del buf
    return (gib << 30) * reps / (a.elapsed_time(b) * 1e-3) / 1e9


def time_one(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=None,
                    help="graph scale (25 for spmm/stream, 26 for precision/apps)")
    ap.add_argument("--edge-factor", type=float, default=None,
                    help="edge factor (44 for spmm/stream, 28 for precision/apps)")
    ap.add_argument("--ks", default="1,2,4,8,16,32")
    ap.add_argument("--select", choices=["learned", "plain"], default="learned")
    ap.add_argument("--weights", default=None, help="cost-model weights (.npy)")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the format comparison (fixed variants, autotuner, learned, V-csr)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--tile-cols", type=int, default=0)
    ap.add_argument("--item-nnz", type=int, default=0)
    ap.add_argument("--max-kc", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time for the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-gib", type=int, default=0,
                    help="run a plain device copy of this many GiB first (counter calibration)")
    ap.add_argument("--mode", default="spmm",
                    help="spmm (default) | stream | semiext | colblocks | apps_directed | precision | apps | eigs | dense | sbm "
                         "(comma-separated)")
    ap.add_argument("--stream-kib", type=int, default=0, help="streamed mode: bytes per transfer group")
    ap.add_argument("--ring-depth", type=int, default=0, help="streamed mode: device ring slots")
    ap.add_argument("--slab-rows", type=int, default=1 << 22,
                    help="semiext mode: rows per block of the slab-wise build")
    ap.add_argument("--eig-blocks", default="1,2,4,8,16", help="eigs mode: block sizes")
    ap.add_argument("--nev", type=int, default=8, help="eigs mode: eigenpairs wanted")
    ap.add_argument("--eig-tol", type=float, default=1e-5, help="eigs mode: relative residual tolerance")
    ap.add_argument("--no-sem", action="store_true", help="eigs mode: skip the semi-external runs")
    ap.add_argument("--sbm-scale", type=int, default=24, help="sbm mode: log2 of the vertex count")
    args = ap.parse_args()
    modes = args.mode.split(",")
    if args.gpus == 1 and modes != ["spmm"]:
        return run_other_modes(args, modes)

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import paper_1602_02864_amd as pk
    import synth
    from paper_1602_02864_amd.selector_train import WEIGHTS

    ks = [int(x) for x in args.ks.split(",")]
    args.scale = 25 if args.scale is None else args.scale
    args.edge_factor = 44.0 if args.edge_factor is None else args.edge_factor
    dev = torch.device("cuda:0")
    torch.cuda.init()
    if args.copy_gib > 0:
        # a plain copy kernel of known size: reads and writes copy_gib GiB
        ca = torch.empty(args.copy_gib << 28, dtype=torch.float32, device=dev).fill_(1.0)
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        torch.cuda.synchronize()
        del ca, cb
        log(f"calibration copy of {args.copy_gib} GiB done")
    params = None
    if args.select == "learned" or args.compare:
        wpath = args.weights or WEIGHTS
        if not os.path.exists(wpath):
            raise SystemExit(f"{wpath} is missing: train it with python -m paper_1602_02864_amd.selector_train")
        params = np.load(wpath, allow_pickle=False).astype(np.float32)

    t0 = time.perf_counter()
    rp, col = synth.rmat_csr(args.scale, args.edge_factor, seed=synth.SEED_GRAPH, progress=log)
    n = rp.shape[0] - 1
    nnz = int(col.shape[0])
    t_gen = time.perf_counter() - t0
    log(f"graph: n={n} nnz={nnz} ({t_gen:.1f}s)")

    t0 = time.perf_counter()
    T, R, C = pk.spmm_model_tiles(rp, col, 16384)
    t_model = time.perf_counter() - t0
    log(f"byte model (16K tiles): tiles={T} sum_nnr={R} sum_nnc={C} ({t_model:.1f}s)")

    def build():
        return pk.spmm_build_tiles(rp, col, tile_rows=args.tile_rows, tile_cols=args.tile_cols,
                                   item_nnz=args.item_nnz, max_kc=args.max_kc, validate=False)

    t0 = time.perf_counter()
    h_plain = build()
    t_build = time.perf_counter() - t0
    st = pk.spmm_get_stats(h_plain)
    max_kc = args.max_kc or 32
    log(f"tiles built in {t_build:.1f}s: tiles={st['n_tiles']} items={st['n_items']} "
        f"parts={st['n_parts']} blob={st['blob_bytes'] / nnz:.2f} B/nnz")

    # learned selection: one handle per distinct per-tile assignment
    handle_of = {k: h_plain for k in ks}
    select_info = {"mode": args.select}
    handles = [h_plain]
    t_select = 0.0
    if args.select == "learned":
        t0 = time.perf_counter()
        pd = torch.from_numpy(params).to(dev)
        assign = {}
        for k in ks:
            f = torch.from_numpy(pk.spmm_tile_features(h_plain, k)).to(dev)
            ch = torch.empty(f.shape[0], dtype=torch.uint8, device=dev)
            pk.spmm_mlp_predict(pd, f, None, ch)
            torch.cuda.synchronize()
            assign[k] = ch.cpu().numpy()
        groups = []
        for k in ks:
            for g in groups:
                if np.array_equal(assign[g[0]], assign[k]):
                    g.append(k)
                    break
            else:
                groups.append([k])
        plain_v = pk.spmm_get_variants(h_plain)
        for g in groups:
            v = assign[g[0]]
            if np.array_equal(v, plain_v):
                hg = h_plain
            else:
                hg = build()
                pk.spmm_set_variants(hg, v)
                handles.append(hg)
            for k in g:
                handle_of[k] = hg
        t_select = time.perf_counter() - t0
        select_info.update({
            "handles": len(handles), "groups": groups, "select_s": round(t_select, 1),
            "tiles_per_variant": {str(k): np.bincount(assign[k], minlength=pk.SPMM_NUM_VARIANTS).tolist()
                                  for k in ks}})
        log(f"learned selection in {t_select:.1f}s: groups {groups}")

    Xs, Ys = {}, {}
    for k in ks:
        Xs[k] = torch.from_numpy(synth.uniform(n, k, seed=synth.SEED_X)).to(dev)
        Ys[k] = torch.empty((n, k), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log("X/Y resident; first calls upload the tiles")

    stream = torch.cuda.current_stream(dev)

    def runs_for(hmap):
        return [(k, (lambda k=k: pk.spmm_run(hmap[k], Xs[k], Ys[k], stream=stream))) for k in ks]

    plain_ms_step, plain_ms_k = time_step(runs_for({k: h_plain for k in ks}), args.steps, args.warmup, stream)
    log("plain: " + ", ".join(f"k={k}: {plain_ms_k[k]:.3f} ms" for k in ks))
    if args.select == "learned":
        ms_step, ms_k = time_step(runs_for(handle_of), args.steps, args.warmup, stream)
        log("learned: " + ", ".join(f"k={k}: {ms_k[k]:.3f} ms" for k in ks))
    else:
        ms_step, ms_k = plain_ms_step, plain_ms_k

    # SpMM-kernel time alone (HIP events around the SpMM launches of each
    # run, on the run's stream), per k, over `steps` further runs
    kernel_ms = {}
    hmap = handle_of if args.select == "learned" else {k: h_plain for k in ks}
    for k in ks:
        pk.spmm_timing_begin(hmap[k])
        for _ in range(args.steps):
            pk.spmm_run(hmap[k], Xs[k], Ys[k], stream=stream)
        tot, runs = pk.spmm_timing_end(hmap[k])
        kernel_ms[k] = tot / max(runs, 1)
    log("kernel only: " + ", ".join(f"k={k}: {kernel_ms[k]:.3f} ms" for k in ks))

    flop_step = sum(2.0 * nnz * k for k in ks)
    value = flop_step / (ms_step * 1e-3) / 1e9
    plain_value = flop_step / (plain_ms_step * 1e-3) / 1e9

    per_k = {}
    for k in ks:
        mb = model_bytes(T, R, C, nnz, n, k)
        launches = -(-k // max_kc)
        per_k[str(k)] = {
            "ms": round(ms_k[k], 4),
            "kernel_ms": round(kernel_ms[k], 4),
            "plain_ms": round(plain_ms_k[k], 4),
            "gflops": round(2.0 * nnz * k / (ms_k[k] * 1e-3) / 1e9, 2),
            "model_gb": round(mb["total"] / 1e9, 4),
            "model_frac": round(mb["total"] / (ms_k[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "floor_frac": round(mb["floor"] / (ms_k[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launches": launches,
        }
    kdom = max(ks, key=lambda k: kernel_ms[k])
    mb = model_bytes(T, R, C, nnz, n, kdom)
    launches = per_k[str(kdom)]["launches"]
    # per launch: the whole A, this launch's share of the X columns and of Y
    kc = -(-kdom // launches)
    launch_bytes = mb["A"] + C * kc * 4 + n * kc * 4
    launch_ms = kernel_ms[kdom] / launches
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    read_gbs = attainable_read_gbs()
    log(f"attainable streaming read: {read_gbs:.0f} GB/s")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kc),
                "kernel": f"spmm_items k={kdom} (kc={kc}, {launches} launch(es) per SpMM; "
                          f"duration from HIP events around the launches)",
                "bytes_per_launch": int(launch_bytes), "ms_per_launch": round(launch_ms, 4),
                "kernel_source_sha256_16": kernel_source_hash(),
                "attainable_read_gbs": round(read_gbs, 1),
                "frac_of_attainable": round(achieved / read_gbs, 4)}

    compare = None
    if args.compare:
        compare = {"plain": {str(k): round(plain_ms_k[k], 4) for k in ks}}
        hc = h_plain
        for v, name in enumerate(pk.VARIANT_NAMES):
            pk.spmm_set_variants(hc, np.full(st["n_tiles"], v, np.uint8))
            compare[f"fixed_{name}"] = {str(k): round(time_one(
                lambda k=k: pk.spmm_run(hc, Xs[k], Ys[k], stream=stream)), 4) for k in ks}
            log(f"fixed {name}: {compare[f'fixed_{name}']}")
        compare["autotune"], compare["autotune_s"] = {}, {}
        for k in ks:
            t0 = time.perf_counter()
            pk.spmm_autotune(hc, k)
            compare["autotune_s"][str(k)] = round(time.perf_counter() - t0, 1)
            compare["autotune"][str(k)] = round(time_one(lambda: pk.spmm_run(hc, Xs[k], Ys[k], stream=stream)), 4)
            log(f"autotune k={k}: {compare['autotune'][str(k)]} ms ({compare['autotune_s'][str(k)]}s)")
        # the untiled CSR baseline (V-csr): rows by length, columns in
        # in-degree order, FP32 register sums
        t0 = time.perf_counter()
        hv = pk.spmm_build_tiles(rp, col, validate=False, format=pk.SPMM_FORMAT_CSR)
        compare["csr_build_s"] = round(time.perf_counter() - t0, 1)
        compare["v_csr"] = {str(k): round(time_one(
            lambda k=k: pk.spmm_run(hv, Xs[k], Ys[k], stream=stream)), 4) for k in ks}
        log(f"V-csr: {compare['v_csr']}")
        hv.close()
        # the same CSR kernels over the original column order: the first step
        # of the optimisation ladder (rows balanced by length, no locality)
        hv = pk.spmm_build_tiles(rp, col, validate=False, format=pk.SPMM_FORMAT_CSR, keep_order=True)
        compare["ablation_v_csr_original_columns"] = {str(k): round(time_one(
            lambda k=k: pk.spmm_run(hv, Xs[k], Ys[k], stream=stream)), 4) for k in ks}
        log(f"V-csr, original column order: {compare['ablation_v_csr_original_columns']}")
        hv.close()
        # ablations: tiles over the original row order, and over the original
        # row and column order (no relabelling at all)
        for name, opt in (("ablation_original_row_order", dict(keep_row_order=True)),
                          ("ablation_original_order", dict(keep_order=True))):
            hk = pk.spmm_build_tiles(rp, col, tile_rows=args.tile_rows, tile_cols=args.tile_cols,
                                     item_nnz=args.item_nnz, max_kc=args.max_kc, validate=False, **opt)
            compare[name] = {str(k): round(time_one(
                lambda k=k: pk.spmm_run(hk, Xs[k], Ys[k], stream=stream)), 4) for k in ks}
            log(f"{name}: {compare[name]}")
            hk.close()
        compare["learned"] = {}
        for k in ks:
            pk.spmm_select_learned(hc, params, k)
            compare["learned"][str(k)] = round(time_one(lambda: pk.spmm_run(hc, Xs[k], Ys[k], stream=stream)), 4)
        log(f"learned (same protocol): {compare['learned']}")
        tot = {m: sum(d.values()) for m, d in compare.items() if isinstance(d, dict) and not m.endswith("_s")}
        compare["sweep_gflops"] = {m: round(flop_step / (t * 1e-3) / 1e9, 1) for m, t in tot.items()}
        best_fixed = min(t for m, t in tot.items() if m.startswith("fixed_"))
        compare["learned_over_autotune"] = round(tot["learned"] / tot["autotune"], 4)
        compare["learned_over_best_fixed"] = round(tot["learned"] / best_fixed, 4)
        compare["learned_over_v_csr"] = round(tot["learned"] / tot["v_csr"], 4)
        # re-select for the parity check below (Y of the last comparison run)
        for k in ks:
            pk.spmm_run(handle_of[k], Xs[k], Ys[k], stream=stream)
        torch.cuda.synchronize()

    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle
        # Bounded sample: rows 0-63 (the R-MAT hubs) plus 64 evenly spread
        # blocks of B consecutive rows, B sized from a probe so that the
        # single-threaded oracle runs about --cpu-seconds over the k sweep.
        deg = np.diff(rp)
        Xh = {k: Xs[k].cpu().numpy() for k in ks}

        def sample(B):
            starts = np.linspace(64, max(64, n - B), 64).astype(np.int64)
            blocks = [np.arange(s0, min(n, s0 + B)) for s0 in starts]
            return np.unique(np.concatenate([np.arange(min(64, n))] + blocks))

        probe = sample(16)
        c0 = time.perf_counter()
        oracle.spmm_sel(rp, col, None, Xh[ks[-1]], probe)
        rate = float(deg[probe].sum()) * ks[-1] / max(time.perf_counter() - c0, 1e-6)
        target_nnz = rate * args.cpu_seconds / sum(ks)
        hub_nnz = float(deg[:64].sum())
        B = int(max(16, (target_nnz - hub_nnz) / (64 * max(deg.mean(), 1.0))))
        sel = sample(min(B, max(16, (n - 64) // 64)))
        sel_nnz = int(deg[sel].sum())
        t_cpu = 0.0
        errs = {}
        for k in ks:
            c0 = time.perf_counter()
            ref = oracle.spmm_sel(rp, col, None, Xh[k], sel)
            t_cpu += time.perf_counter() - c0
            got = Ys[k][torch.from_numpy(sel).to(dev)].cpu().numpy()
            errs[str(k)] = oracle.frob_rel_err(got, ref)
        cpu_gflops = sum(2.0 * sel_nnz * k for k in ks) / t_cpu / 1e9
        # second leg: the same loop with the rows spread over the host's
        # threads (OpenMP); rows are independent, so Y is the same bits
        t_omp = 0.0
        threads = 1
        for k in ks:
            c0 = time.perf_counter()
            ref_omp, threads = oracle.spmm_sel_omp(rp, col, None, Xh[k], sel)
            t_omp += time.perf_counter() - c0
            got = Ys[k][torch.from_numpy(sel).to(dev)].cpu().numpy()
            errs[str(k)] = max(errs[str(k)], oracle.frob_rel_err(got, ref_omp))
        omp_gflops = sum(2.0 * sel_nnz * k for k in ks) / t_omp / 1e9
        host = host_info()
        cpu = {"value": round(cpu_gflops, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"{sel.size} rows ({sel_nnz} nnz: rows 0-63 plus spread blocks), "
                         f"k sweep {ks}, FP64 single-threaded CSR loop, {t_cpu:.1f}s",
               "threaded": {"value": round(omp_gflops, 3), "unit": "GFLOP/s", "cores": threads,
                            "kind": "oracle, OpenMP over rows", "seconds": round(t_omp, 2)},
               **host}
        parity = {"rows": int(sel.size), "max_rel_frob_err": max(errs.values()), "per_k": errs,
                  "tolerance": 1e-6, "ok": max(errs.values()) <= 1e-6}
        log(f"cpu oracle {cpu_gflops:.2f} GFLOP/s over {t_cpu:.1f}s (1 thread), {omp_gflops:.2f} GFLOP/s "
            f"over {t_omp:.1f}s ({threads} threads); parity max err {parity['max_rel_frob_err']:.3g}")

    out = {
        "metric": "SpMM GFLOP/s (2*nnz*k/s) over the k sweep, % HBM roofline; learned-tuned vs plain",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"rmat-s{args.scale}-ef{int(args.edge_factor)}-directed-binary",
                   "n": n, "nnz": nnz, "k": ks, "x": "f32 uniform[0,1) seed 2", "graph_seed": 1,
                   "tile_rows": st["tile_rows"], "tile_cols": st["tile_cols"], "max_kc": max_kc,
                   "select": args.select},
        "plain": {"value": round(plain_value, 2), "ms_per_step": round(plain_ms_step, 4),
                  "learned_over_plain": round(value / plain_value, 4)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "per_k": per_k,
        "selection": select_info,
        "compare_ms": compare,
        "tiles": {k: st[k] for k in ("n_tiles", "n_items", "n_parts", "blob_bytes", "sum_nnr", "sum_nnc")},
        "model_16k": {"tiles": T, "sum_nnr": R, "sum_nnc": C},
        "prep_s": {"generate": round(t_gen, 1), "model": round(t_model, 1), "build": round(t_build, 1),
                   "select": round(t_select, 1)},
    }
    print(json.dumps(out), flush=True)
    for hd in handles:
        hd.close()
    return 0


# ---------------------------------------------------------------- other modes

def host_info() -> dict:
    """The host the CPU baseline ran on: logical CPUs, CPU model, RAM."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["host_ram_gb"] = round(int(line.split()[1]) / 1048576, 1)
                    break
    except OSError:
        pass
    return info


def sample_rows(rp, n, budget_nnz):
    """Rows 0-63 (the R-MAT hubs) plus 64 evenly spread blocks of consecutive
    rows, sized so that the blocks hold about budget_nnz non-zeros."""
    import numpy as np
    deg = np.diff(rp)
    B = int(max(16, budget_nnz / (64 * max(float(deg.mean()), 1.0))))
    B = min(B, max(16, (n - 64) // 64))
    starts = np.linspace(64, max(64, n - B), 64).astype(np.int64)
    return np.unique(np.concatenate([np.arange(min(64, n))] + [np.arange(s0, min(n, s0 + B)) for s0 in starts]))


def pinned_h2d_gbs(gib=1, reps=5):
    """Host-to-device rate of a plain copy from pinned memory (the link)."""
    import torch
    src = torch.empty(gib << 28, dtype=torch.float32, pin_memory=True)
    dst = torch.empty(gib << 28, dtype=torch.float32, device="cuda")
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src, non_blocking=True)
    b.record()
    torch.cuda.synchronize()
    return (gib << 30) * reps / (a.elapsed_time(b) * 1e-3) / 1e9


def run_other_modes(args, modes) -> int:
    import numpy as np
    import torch

    import oracle
    import paper_1602_02864_amd as pk
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.init()
    big = any(m in ("precision", "apps", "eigs", "dense") for m in modes)
    scale = args.scale if args.scale is not None else (26 if big else 25)
    ef = args.edge_factor if args.edge_factor is not None else (28.0 if big else 44.0)
    sym = big
    t0 = time.perf_counter()
    if modes == ["dense"] or modes == ["sbm"]:     # no R-MAT graph needed
        rp, col = np.zeros(2, np.int64), np.zeros(0, np.int32)
        n, nnz = 1 << scale, 0
    else:
        rp, col = synth.rmat_csr(scale, ef, seed=synth.SEED_GRAPH, symmetrize=sym, progress=log)
        n, nnz = rp.shape[0] - 1, int(col.shape[0])
    workload = f"rmat-s{scale}-ef{int(ef)}-{'symmetrised' if sym else 'directed'}"
    log(f"graph {workload}: n={n} nnz={nnz} ({time.perf_counter() - t0:.1f}s)")
    stream = torch.cuda.current_stream(dev)

    def kernel_ms(h, fn, reps=3):
        fn()
        torch.cuda.synchronize()
        pk.spmm_timing_begin(h)
        for _ in range(reps):
            fn()
        tot, runs = pk.spmm_timing_end(h)
        return tot / max(runs, 1)

    for mode in modes:
        if mode == "stream":
            ks = [int(x) for x in args.ks.split(",")]
            link = pinned_h2d_gbs()
            log(f"pinned host-to-device copy: {link:.1f} GB/s")
            hd = pk.spmm_build_tiles(rp, col, validate=False)
            hs = pk.spmm_build_tiles(rp, col, validate=False, place=pk.SPMM_PLACE_PINNED_HOST,
                                     stream_kib=args.stream_kib, ring_depth=args.ring_depth)
            payload = pk.spmm_get_stats(hs)["blob_bytes"]
            copy = torch.cuda.Stream(dev)
            per_k = {}
            for k in ks:
                X = torch.from_numpy(synth.uniform(n, k, seed=synth.SEED_X)).to(dev)
                Yd = torch.empty((n, k), device=dev)
                Ys = torch.empty((n, k), device=dev)
                t_hbm = time_one(lambda: pk.spmm_run(hd, X, Yd, stream=stream))
                t_str = time_one(lambda: pk.spmm_stream_run(hs, X, Ys, compute=stream, copy=copy))
                torch.cuda.synchronize()
                same = bool(torch.equal(Yd, Ys))
                per_k[str(k)] = {"hbm_ms": round(t_hbm, 3), "stream_ms": round(t_str, 3),
                                 "stream_gflops": round(2.0 * nnz * k / (t_str * 1e-3) / 1e9, 2),
                                 "hbm_gflops": round(2.0 * nnz * k / (t_hbm * 1e-3) / 1e9, 2),
                                 "payload_gbs": round(payload / (t_str * 1e-3) / 1e9, 2),
                                 "link_frac": round(payload / (t_str * 1e-3) / 1e9 / link, 4),
                                 "stream_over_hbm": round(t_hbm / t_str, 4),
                                 "y_identical_to_hbm": same}
                log(f"stream k={k}: {per_k[str(k)]}")
                del X, Yd, Ys
            tot_s = sum(v["stream_ms"] for v in per_k.values())
            out = {"mode": "stream", "metric": "streamed SpMM GFLOP/s (A in pinned host memory) and % of host-to-device link",
                   "value": round(sum(2.0 * nnz * k for k in ks) / (tot_s * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                   "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": workload, "n": n, "nnz": nnz, "k": ks,
                              "stream_kib": args.stream_kib or 262144, "ring_depth": args.ring_depth or 3},
                   "payload_bytes": int(payload), "link_gbs_measured": round(link, 2),
                   "link_frac_min": min(v["link_frac"] for v in per_k.values()),
                   "per_k": per_k}
            print(json.dumps(out), flush=True)
            hd.close()
            hs.close()
        elif mode == "semiext":
            # The semi-external configuration on one GPU: the tile store is
            # built block by block (spmm_build_begin / append_rows / end)
            # into pinned host memory and streamed to HBM for every SpMM; X is
            # resident; Y either resident or streamed back to host memory.
            # The same tiles placed in HBM give the in-HBM rate and the
            # bit-identity check; sampled rows are checked against the oracle.
            ks = [int(x) for x in args.ks.split(",")]
            link = pinned_h2d_gbs()
            log(f"pinned host-to-device copy: {link:.1f} GB/s")

            def slab_build(place):
                t0 = time.perf_counter()
                h = pk.spmm_build_begin(n, keep_row_order=True, validate=False, place=place,
                                        stream_kib=args.stream_kib, ring_depth=args.ring_depth)
                for r0 in range(0, n, args.slab_rows):
                    r1 = min(n, r0 + args.slab_rows)
                    a, b = int(rp[r0]), int(rp[r1])
                    pk.spmm_build_append_rows(h, r0, rp[r0:r1 + 1] - a, col[a:b])
                    if (r0 // args.slab_rows) % 16 == 15 or r1 == n:
                        log(f"slab-wise build ({'host' if place else 'device'}): rows {r1}/{n}")
                pk.spmm_build_end(h)
                return h, time.perf_counter() - t0

            hs, t_bs = slab_build(pk.SPMM_PLACE_PINNED_HOST)
            sst = pk.spmm_get_stats(hs)
            payload = sst["blob_bytes"]
            log(f"host-placed tiles built in {t_bs:.1f}s: {payload / nnz:.2f} B/nnz, {payload / 2**30:.1f} GiB")
            hd, t_bd = slab_build(pk.SPMM_PLACE_DEVICE)
            copy = torch.cuda.Stream(dev)
            out_s = torch.cuda.Stream(dev)
            rng = np.random.default_rng(7)
            sel = np.unique(rng.integers(0, max(1, n // 32), 64) * 32)   # 64 random 32-row tile rows
            sel = np.unique((sel[:, None] + np.arange(32)[None, :]).ravel())
            sel = sel[sel < n]
            per_k = {}
            for k in ks:
                X = torch.from_numpy(synth.uniform(n, k, seed=synth.SEED_X)).to(dev)
                Yd = torch.empty((n, k), device=dev)
                Ys = torch.empty((n, k), device=dev)
                t_hbm = time_one(lambda: pk.spmm_run(hd, X, Yd, stream=stream))
                t_str = time_one(lambda: pk.spmm_stream_run(hs, X, Ys, compute=stream, copy=copy))
                torch.cuda.synchronize()
                same = bool(torch.equal(Yd, Ys))
                Yh = torch.empty((n, k), dtype=torch.float32).pin_memory()

                def yhost():
                    out_s.wait_stream(stream)
                    pk.spmm_stream_run_yhost(hs, X, Yh, compute=stream, copy=copy, out=out_s)
                    stream.wait_stream(out_s)
                t_yh = time_one(yhost)
                torch.cuda.synchronize()
                same_yh = bool(torch.equal(Yd.cpu(), Yh))
                ref = oracle.spmm_sel(rp, col, None, X.cpu().numpy(), sel)
                err = oracle.frob_rel_err(Ys[torch.from_numpy(sel).to(dev)].cpu().numpy(), ref)
                per_k[str(k)] = {"hbm_ms": round(t_hbm, 3), "stream_ms": round(t_str, 3),
                                 "stream_y_host_ms": round(t_yh, 3),
                                 "stream_gflops": round(2.0 * nnz * k / (t_str * 1e-3) / 1e9, 2),
                                 "hbm_gflops": round(2.0 * nnz * k / (t_hbm * 1e-3) / 1e9, 2),
                                 "payload_gbs": round(payload / (t_str * 1e-3) / 1e9, 2),
                                 "link_frac": round(payload / (t_str * 1e-3) / 1e9 / link, 4),
                                 "stream_over_hbm": round(t_hbm / t_str, 4),
                                 "y_identical_to_hbm": same, "y_host_identical_to_hbm": same_yh,
                                 "sampled_rows": int(sel.size), "sampled_rel_err": err}
                log(f"semiext k={k}: {per_k[str(k)]}")
                del X, Yd, Ys, Yh
            tot_s = sum(v["stream_ms"] for v in per_k.values())
            out = {"mode": "semiext", "metric": "semi-external SpMM GFLOP/s (tiles built slab-wise into pinned host "
                                                "memory, streamed per SpMM) and % of host-to-device link",
                   "value": round(sum(2.0 * nnz * k for k in ks) / (tot_s * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                   "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": workload, "n": n, "nnz": nnz, "k": ks, "slab_rows": args.slab_rows,
                              "row_order": "given", "column_order": "given",
                              "stream_kib": args.stream_kib or 262144, "ring_depth": args.ring_depth or 3},
                   "payload_bytes": int(payload), "payload_bytes_per_nnz": round(payload / nnz, 3),
                   "build_s": {"host_placed": round(t_bs, 1), "device_placed": round(t_bd, 1)},
                   "link_gbs_measured": round(link, 2), "per_k": per_k}
            print(json.dumps(out), flush=True)
            hd.close()
            hs.close()
        elif mode == "colblocks":
            # X and Y in pinned host memory too, their columns in blocks: the
            # paper's dense matrix partly in memory (A streamed once per block)
            k = 32
            link = pinned_h2d_gbs()
            hd = pk.spmm_build_tiles(rp, col, validate=False)
            hs = pk.spmm_build_tiles(rp, col, validate=False, place=pk.SPMM_PLACE_PINNED_HOST,
                                     stream_kib=args.stream_kib, ring_depth=args.ring_depth)
            payload = pk.spmm_get_stats(hs)["blob_bytes"]
            Xnp = synth.uniform(n, k, seed=synth.SEED_X)
            Xd = torch.from_numpy(Xnp).to(dev)
            Yd = torch.empty((n, k), device=dev)
            t_hbm = time_one(lambda: pk.spmm_run(hd, Xd, Yd, stream=stream))
            ref = Yd.cpu().numpy()
            log(f"in-HBM k={k}: {t_hbm:.2f} ms")
            per_cb = {}
            for cb in (32, 16, 8, 4, 2, 1):
                # host X and Y in the blocked layout: each block of columns
                # contiguous, so every block crosses the link as one copy
                blocks = [(c0, min(cb, k - c0)) for c0 in range(0, k, cb)]
                Xb = torch.from_numpy(np.concatenate([np.ascontiguousarray(Xnp[:, c0:c0 + w]).ravel()
                                                      for c0, w in blocks])).pin_memory()
                Yb = torch.empty(n * k, dtype=torch.float32).pin_memory()
                pk.spmm_stream_run_host(hs, Xb, Yb, cb, k=k, blocked=True)   # warm-up (ring, buffers)
                t0 = time.perf_counter()
                pk.spmm_stream_run_host(hs, Xb, Yb, cb, k=k, blocked=True)
                t = (time.perf_counter() - t0) * 1e3
                Y = np.empty((n, k), np.float32)
                off = 0
                for c0, w in blocks:
                    Y[:, c0:c0 + w] = Yb[off:off + n * w].numpy().reshape(n, w)
                    off += n * w
                # host -> device: A once per block plus X once (Y returns on the
                # other direction of the full-duplex link)
                h2d = len(blocks) * payload + n * k * 4
                per_cb[str(cb)] = {"ms": round(t, 1), "blocks": len(blocks),
                                   "gflops": round(2.0 * nnz * k / (t * 1e-3) / 1e9, 1),
                                   "of_in_hbm": round(t_hbm / t, 4),
                                   "h2d_gbs": round(h2d / (t * 1e-3) / 1e9, 1),
                                   "link_frac": round(h2d / (t * 1e-3) / 1e9 / link, 4),
                                   "rel_err_vs_in_hbm": oracle.frob_rel_err(Y, ref),
                                   "identical_to_in_hbm": bool(np.array_equal(Y, ref))}
                log(f"columns per block {cb}: {per_cb[str(cb)]}")
                del Xb, Yb, Y
            out = {"mode": "colblocks",
                   "metric": "semi-external SpMM with A, X and Y in host memory, X/Y columns in blocks: "
                             "GFLOP/s and fraction of the in-HBM rate",
                   "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                   "config": {"workload": workload, "n": n, "nnz": nnz, "k": k},
                   "in_hbm_ms": round(t_hbm, 3), "payload_bytes": int(payload),
                   "link_gbs_measured": round(link, 2), "per_columns_per_block": per_cb}
            print(json.dumps(out), flush=True)
            hd.close()
            hs.close()
            del Xd, Yd, ref
        elif mode == "apps_directed":
            # the directed graph: PageRank on the in-link matrix A^T and NMF
            # with A and A^T, both transposed by the library's build
            if sym:
                raise SystemExit("apps_directed needs the directed graph (run it without precision/apps)")
            t0 = time.perf_counter()
            hT = pk.spmm_build_tiles(rp, col, validate=False, transpose=True)
            t_tb = time.perf_counter() - t0
            hA = pk.spmm_build_tiles(rp, col, validate=False)
            log(f"transposed build {t_tb:.1f}s")
            pr = torch.empty(n, device=dev)
            pk.spmm_pagerank(hT, pr, iters=2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            resid = pk.spmm_pagerank(hT, pr, iters=30)
            t_pr = time.perf_counter() - t0
            s_pr = float(pr.double().sum().item())
            W = torch.from_numpy(synth.uniform(n, 16, seed=synth.SEED_W)).to(dev)
            Hm = torch.from_numpy(synth.uniform(n, 16, seed=synth.SEED_H)).to(dev)
            pk.spmm_nmf(hA, hT, W, Hm, iters=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pk.spmm_nmf(hA, hT, W, Hm, iters=10)
            torch.cuda.synchronize()
            t_nmf = time.perf_counter() - t0
            ok_nmf = bool(torch.isfinite(W).all().item() and torch.isfinite(Hm).all().item()
                          and (W >= 0).all().item() and (Hm >= 0).all().item())
            out = {"mode": "apps_directed", "metric": "PageRank and NMF time per iteration (directed graph)",
                   "n_gpus": 1, "data": "synthetic", "config": {"workload": workload, "n": n, "nnz": nnz},
                   "transposed_build_s": round(t_tb, 1),
                   "pagerank_ms_per_iter": round(t_pr * 1e3 / 30, 3), "pagerank_sum": s_pr,
                   "pagerank_resid_first_last": [float(resid[0]), float(resid[-1])],
                   "nmf_ms_per_iter": round(t_nmf * 1e3 / 10, 3),
                   "nmf_spmm_gflops": round(2 * 2.0 * nnz * 16 / (t_nmf / 10) / 1e9, 2),
                   "nmf_factors_finite_nonneg": ok_nmf}
            log(f"apps_directed: {out}")
            print(json.dumps(out), flush=True)
            del W, Hm, pr
            hT.close()
            hA.close()
        elif mode == "precision":
            vals = synth.lognormal_weights(rp, col, seed=synth.SEED_WEIGHT)
            log("weights drawn")
            sel = sample_rows(rp, n, 1.5e6)
            tols = {"f32": 1e-6, "bf16": 1e-2, "fp8": 6e-2}
            res = []
            for weighted in (False, True):
                h = pk.spmm_build_tiles(rp, col, vals if weighted else None, validate=False)
                for k in (16, 32, 64):
                    Xh = synth.uniform(n, k, seed=synth.SEED_X)
                    X = torch.from_numpy(Xh).to(dev)
                    Y = torch.empty((n, k), device=dev)
                    ref = oracle.spmm_sel(rp, col, vals if weighted else None, Xh, sel)
                    seld = torch.from_numpy(sel).to(dev)
                    row = {"weighted": weighted, "k": k}
                    for name, dt in (("f32", pk.SPMM_X_F32), ("bf16", pk.SPMM_X_BF16), ("fp8", pk.SPMM_X_FP8_E4M3)):
                        cs = None
                        if dt == pk.SPMM_X_F32:
                            Xin = X
                        elif dt == pk.SPMM_X_BF16:
                            Xin = torch.empty((n, k), dtype=torch.bfloat16, device=dev)
                            pk.spmm_quantize_x(X, Xin, dt)
                        else:
                            Xin = torch.empty((n, k), dtype=torch.uint8, device=dev)
                            cs = torch.empty(k, dtype=torch.float32, device=dev)
                            pk.spmm_quantize_x(X, Xin, dt, col_scale=cs)
                        fn = (lambda Xin=Xin, dt=dt, cs=cs: pk.spmm_run(h, Xin, Y, dtype=dt, col_scale=cs, stream=stream))
                        t = time_one(fn)
                        tk = kernel_ms(h, fn)
                        got = Y[seld].cpu().numpy()
                        err = oracle.frob_rel_err(got, ref)
                        row[name] = {"rel_frob_err": err, "tolerance": tols[name], "ok": err <= tols[name],
                                     "ms": round(t, 3), "kernel_ms": round(tk, 3),
                                     "gflops": round(2.0 * nnz * k / (t * 1e-3) / 1e9, 2)}
                        del Xin
                    log(f"precision {row}")
                    res.append(row)
                    del X, Y
                h.close()
            out = {"mode": "precision", "metric": "SpMM error vs the FP64 oracle (sampled rows) and GFLOP/s per X type",
                   "n_gpus": 1, "data": "synthetic",
                   "config": {"workload": workload, "n": n, "nnz": nnz, "weights": "binary and lognormal(0,1)",
                              "sample_rows": int(sel.size), "sample_nnz": int(np.diff(rp)[sel].sum())},
                   "all_ok": all(r[d]["ok"] for r in res for d in ("f32", "bf16", "fp8")), "results": res}
            print(json.dumps(out), flush=True)
        elif mode == "apps":
            from paper_1602_02864_amd.selector_train import WEIGHTS
            params = np.load(args.weights or WEIGHTS, allow_pickle=False).astype(np.float32)
            out = {"mode": "apps", "metric": "PageRank and NMF time per iteration", "n_gpus": 1,
                   "data": "synthetic", "config": {"workload": workload, "n": n, "nnz": nnz}}
            for sel_name in ("plain", "learned"):
                h = pk.spmm_build_tiles(rp, col, validate=False)
                if sel_name == "learned":
                    pk.spmm_select_learned(h, params, 1)
                pr = torch.empty(n, device=dev)
                pk.spmm_pagerank(h, pr, iters=2)   # warm-up (upload, graph build)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                resid = pk.spmm_pagerank(h, pr, iters=30)
                t_pr = time.perf_counter() - t0
                s_pr = float(pr.double().sum().item())
                t_spmv = kernel_ms(h, lambda: pk.spmm_run(h, pr[:, None], torch.empty((n, 1), device=dev),
                                                          stream=stream))
                if sel_name == "learned":
                    pk.spmm_select_learned(h, params, 16)
                W = torch.from_numpy(synth.uniform(n, 16, seed=synth.SEED_W)).to(dev)
                Hm = torch.from_numpy(synth.uniform(n, 16, seed=synth.SEED_H)).to(dev)
                pk.spmm_nmf(h, h, W, Hm, iters=1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pk.spmm_nmf(h, h, W, Hm, iters=10)
                torch.cuda.synchronize()
                t_nmf = time.perf_counter() - t0
                ok_nmf = bool(torch.isfinite(W).all().item() and torch.isfinite(Hm).all().item()
                              and (W >= 0).all().item() and (Hm >= 0).all().item())
                out[sel_name] = {
                    "pagerank_ms_per_iter": round(t_pr * 1e3 / 30, 3),
                    "pagerank_spmv_gflops": round(2.0 * nnz / (t_spmv * 1e-3) / 1e9, 2),
                    "pagerank_sum": s_pr, "pagerank_resid_first_last": [float(resid[0]), float(resid[-1])],
                    "nmf_ms_per_iter": round(t_nmf * 1e3 / 10, 3),
                    "nmf_spmm_gflops": round(2 * 2.0 * nnz * 16 / (t_nmf / 10) / 1e9, 2),
                    "nmf_factors_finite_nonneg": ok_nmf}
                log(f"apps {sel_name}: {out[sel_name]}")
                del W, Hm, pr
                h.close()
            out["learned_over_plain_pagerank"] = round(out["plain"]["pagerank_ms_per_iter"] /
                                                       out["learned"]["pagerank_ms_per_iter"], 4)
            out["learned_over_plain_nmf"] = round(out["plain"]["nmf_ms_per_iter"] / out["learned"]["nmf_ms_per_iter"], 4)
            print(json.dumps(out), flush=True)
        elif mode == "dense":
            # the eigensolver's tall-skinny products on n rows of the graph's
            # size, basis stride as the solver lays it out; HBM GB/s from
            # the algorithmic bytes
            import itertools
            out = {"mode": "dense", "metric": "tall-skinny basis products, algorithmic GB/s", "n_gpus": 1,
                   "data": "synthetic", "config": {"n": n}, "shapes": []}
            ld = 136
            A = torch.rand((n, ld), device=dev)
            B = torch.rand((n, 16), device=dev)
            W = torch.rand((n, 64), device=dev)
            work = torch.empty(pk.spmm_dense_tn_workspace(n, 512, 2) // 8, dtype=torch.float64, device=dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for p_, q_ in itertools.product((8, 32, 64, 128), (1, 4, 8)):
                C = torch.rand((p_, q_), dtype=torch.float64, device=dev)
                Bq = B[:, :q_]
                res = {"p": p_, "q": q_}
                for name, fn, nbytes in (
                        ("tn", lambda: pk.spmm_dense_tn(A, Bq, C, work, p=p_, q=q_, stream=stream),
                         4.0 * n * (p_ + q_)),
                        ("nn", lambda: pk.spmm_dense_nn(A, C, W, alpha=1.0, beta=-1.0, p=p_, q=q_, stream=stream),
                         4.0 * n * (p_ + 2 * q_))):
                    fn()
                    e0.record(stream)
                    for _ in range(5):
                        fn()
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / 5
                    res[name + "_ms"] = round(ms, 3)
                    res[name + "_gbs"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
                out["shapes"].append(res)
                log(f"dense {res}")
            # the restart product: basis (m + b columns) times the kept Ritz vectors
            for m_, q_ in ((48, 32), (96, 56), (128, 72)):
                C = torch.rand((m_ + 8, q_), dtype=torch.float64, device=dev)
                Wr = torch.empty((n, q_), device=dev)
                fn = lambda: pk.spmm_dense_nn(A, C, Wr, p=m_ + 8, q=q_, stream=stream)
                fn()
                e0.record(stream)
                for _ in range(3):
                    fn()
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / 3
                res = {"restart_p": m_ + 8, "q": q_, "ms": round(ms, 3),
                       "gbs": round(4.0 * n * (m_ + 8 + q_) / (ms * 1e-3) / 1e9, 1)}
                out["shapes"].append(res)
                log(f"dense {res}")
                del Wr
            del A, B, W, work
            print(json.dumps(out), flush=True)
        elif mode == "sbm":
            # Section 5's stochastic-block-model study: streamed (semi-external)
            # SpMV relative to in-HBM SpMV, clustered vs randomly ordered
            # vertices, for several cluster counts and inside/outside ratios.
            # Tiles keep the given column order (the in-degree relabelling
            # would erase the clusters).
            sn = 1 << args.sbm_scale
            samples = sn * 32
            link = pinned_h2d_gbs()
            out = {"mode": "sbm", "metric": "in-HBM time / streamed time (SpMV and k = 16)", "n_gpus": 1,
                   "data": "synthetic", "config": {"n": sn, "edge_samples": samples, "keep_order": True,
                                                   "link_gbs": round(link, 1)}, "graphs": []}
            copy = torch.cuda.Stream(dev)
            for clusters in (64, 4096):
                for p_in in (0.5, 0.9):
                    for clustered in (True, False):
                        g_rp, g_col = synth.sbm_csr(sn, clusters, samples, p_in, clustered=clustered,
                                                    seed=synth.SEED_GRAPH, progress=log)
                        hd = pk.spmm_build_tiles(g_rp, g_col, validate=False, keep_order=True)
                        hs = pk.spmm_build_tiles(g_rp, g_col, validate=False, keep_order=True,
                                                 place=pk.SPMM_PLACE_PINNED_HOST)
                        res = {"clusters": clusters, "in_out": f"{p_in / (1 - p_in):g}:1",
                               "p_in": p_in, "clustered": clustered, "nnz": int(g_col.shape[0]),
                               "payload_gb": round(pk.spmm_get_stats(hs)["blob_bytes"] / 1e9, 3)}
                        for k in (1, 16):
                            X = torch.from_numpy(synth.uniform(sn, k, seed=synth.SEED_X)).to(dev)
                            Yd = torch.empty((sn, k), device=dev)
                            Ys = torch.empty((sn, k), device=dev)
                            imk = kernel_ms(hd, lambda: pk.spmm_run(hd, X, Yd, stream=stream))
                            torch.cuda.synchronize()
                            t0 = time.perf_counter()
                            for _ in range(3):
                                pk.spmm_run(hd, X, Yd, stream=stream)
                            torch.cuda.synchronize()
                            im = (time.perf_counter() - t0) / 3 * 1e3
                            pk.spmm_stream_run(hs, X, Ys, copy=copy)
                            torch.cuda.synchronize()
                            t0 = time.perf_counter()
                            for _ in range(3):
                                pk.spmm_stream_run(hs, X, Ys, copy=copy)
                                torch.cuda.synchronize()
                            sem = (time.perf_counter() - t0) / 3 * 1e3
                            same = bool(torch.equal(Yd, Ys))
                            res[f"k{k}"] = {"im_ms": round(im, 3), "im_kernel_ms": round(imk, 3),
                                            "sem_ms": round(sem, 3),
                                            "im_over_sem": round(im / sem, 4), "identical": same}
                            del X, Yd, Ys
                        out["graphs"].append(res)
                        log(f"sbm {res}")
                        hd.close()
                        hs.close()
                        del g_rp, g_col
            print(json.dumps(out), flush=True)
        elif mode == "eigs":
            # eight largest-magnitude eigenpairs of the undirected graph
            # (Section 4.2's experiment), for each block size
            nev = args.nev
            h = pk.spmm_build_tiles(rp, col, validate=False)
            out = {"mode": "eigs", "metric": f"time to {nev} eigenpairs (block Krylov-Schur, LM)", "n_gpus": 1,
                   "data": "synthetic", "config": {"workload": workload, "n": n, "nnz": nnz, "nev": nev,
                                                   "tol": args.eig_tol}}
            sel = sample_rows(rp, n, 20_000_000)
            for b in [int(x) for x in args.eig_blocks.split(",")]:
                Xw = torch.from_numpy(synth.uniform(n, b, seed=synth.SEED_X)).to(dev)
                Yw = torch.empty((n, b), device=dev)
                spmm_ms = kernel_ms(h, lambda: pk.spmm_run(h, Xw, Yw, stream=stream))
                del Xw, Yw
                V = torch.empty((n, nev), device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                evals, resid, info = pk.spmm_eigs(h, nev, block=b, tol=args.eig_tol, evecs=V, seed=7)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                Vd = V.double()
                G = torch.stack([(Vd * Vd[:, j:j + 1]).sum(0) for j in range(nev)])    # V^T V, FP64
                orth = float((G - torch.eye(nev, dtype=torch.float64, device=dev)).abs().max().item())
                del Vd, G
                Vh = V.cpu().numpy()
                r_sel = oracle.eig_residuals(rp, col, None, evals, Vh, sel) / np.abs(evals)
                res = {"block": b, "max_dim": info["max_dim"], "seconds": round(wall, 3),
                       "n_spmm": info["n_spmm"], "restarts": info["restarts"],
                       "spmm_s": round(info["spmm_ms"] / 1e3, 3),
                       "spmm_share": round(info["spmm_ms"] / 1e3 / wall, 4),
                       "spmm_k_ms": round(spmm_ms, 3),
                       "dense_s": round(info["dense_ms"] / 1e3, 3),
                       "dense_gbs": round(info["dense_bytes"] / (info["dense_ms"] * 1e-3) / 1e9, 1),
                       "host_s": round((info["total_ms"] - info["spmm_ms"] - info["dense_ms"]) / 1e3, 3),
                       "reorth": f'{info["n_reorth"]}/{info["n_orth"]}',
                       "evals": [float(x) for x in evals],
                       "resid_est_max": float(resid.max()),
                       "sampled_resid_rel_max": float(r_sel.max()),
                       "orth_max": orth,
                       "ok": bool(info["n_converged"] == nev and r_sel.max() <= 4 * args.eig_tol + 2e-6
                                  and orth < 1e-5)}
                out[f"block{b}"] = res
                log(f"eigs block {b}: {res}")
                del V, Vh
            h.close()
            if not args.no_sem:
                # semi-external: tiles in pinned host memory, streamed for every
                # product (the basis stays in HBM); identical results expected
                hs = pk.spmm_build_tiles(rp, col, validate=False, place=pk.SPMM_PLACE_PINNED_HOST,
                                         stream_kib=args.stream_kib, ring_depth=args.ring_depth)
                for b in [int(x) for x in args.eig_blocks.split(",")]:
                    V = torch.empty((n, nev), device=dev)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    evals, resid, info = pk.spmm_eigs(hs, nev, block=b, tol=args.eig_tol, evecs=V, seed=7)
                    torch.cuda.synchronize()
                    wall = time.perf_counter() - t0
                    ref = out[f"block{b}"]
                    res = {"seconds": round(wall, 3), "n_spmm": info["n_spmm"],
                           "spmm_s": round(info["spmm_ms"] / 1e3, 3),
                           "in_hbm_over_sem": round(ref["seconds"] / wall, 4),
                           "evals_equal_in_hbm": [float(x) for x in evals] == ref["evals"]}
                    out[f"sem_block{b}"] = res
                    log(f"eigs semi-external block {b}: {res}")
                    del V
                hs.close()
            out["sampled_rows"] = int(sel.size)
            print(json.dumps(out), flush=True)
        else:
            raise SystemExit(f"unknown mode {mode}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
