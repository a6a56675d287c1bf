#!/usr/bin/env python3
"""SpMM benchmark on one MI355X.

Workload: directed R-MAT graph, scale 25 (33,554,432 vertices), edge factor 44
(1.476e9 samples, ~1.4e9 stored non-zeros after removing duplicates and
self-loops), a/b/c/d = .57/.19/.19/.05, binary A; X is FP32 uniform[0,1)
(seed 2) with k in {1, 2, 4, 8, 16, 32}.  One step = one SpMM Y = A X for
every k of the sweep; the reported value is the aggregate GFLOP/s of a step,
2 * nnz * sum(k) / step time, with X, Y and the tiles resident in HBM.

Printed (one JSON line on stdout): the metric, the roofline of the dominant
kernel under the paper-tile byte model (16K x 16K tiles: A as SCSR, each
tile reading the X rows of its non-empty columns once, each Y row written
once), and the CPU oracle timed on a bounded sample of rows, whose results
also give a sampled full-size parity check of the GPU output.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def model_bytes(T: int, R: int, C: int, nnz: int, n: int, k: int, xbytes: int = 4) -> dict:
    """Paper-tile byte model for one SpMM (Section 3.2 sizes, 16K tiles)."""
    b_a = 2 * R + 2 * nnz + 8 * T
    b_x = C * k * xbytes
    b_y = n * k * 4
    return {"A": b_a, "X": b_x, "Y": b_y, "total": b_a + b_x + b_y,
            "floor": b_a + n * k * xbytes + b_y}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=25)
    ap.add_argument("--edge-factor", type=float, default=44.0)
    ap.add_argument("--ks", default="1,2,4,8,16,32")
    ap.add_argument("--variant", type=int, default=-1, help="fixed tile variant (-1 = default)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--tile-cols", type=int, default=0)
    ap.add_argument("--item-nnz", type=int, default=0)
    ap.add_argument("--max-kc", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time for the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import paper_1602_02864_amd as pk
    import synth

    ks = [int(x) for x in args.ks.split(",")]
    dev = torch.device("cuda:0")
    torch.cuda.init()

    t0 = time.perf_counter()
    rp, col = synth.rmat_csr(args.scale, args.edge_factor, seed=synth.SEED_GRAPH)
    n = rp.shape[0] - 1
    nnz = int(col.shape[0])
    t_gen = time.perf_counter() - t0
    log(f"graph: n={n} nnz={nnz} ({t_gen:.1f}s)")

    t0 = time.perf_counter()
    T, R, C = pk.spmm_model_tiles(rp, col, 16384)
    t_model = time.perf_counter() - t0
    log(f"byte model (16K tiles): tiles={T} sum_nnr={R} sum_nnc={C} ({t_model:.1f}s)")

    t0 = time.perf_counter()
    h = pk.spmm_build_tiles(rp, col, tile_rows=args.tile_rows, tile_cols=args.tile_cols,
                            fixed_variant=args.variant, item_nnz=args.item_nnz,
                            max_kc=args.max_kc, validate=False)
    t_build = time.perf_counter() - t0
    st = pk.spmm_get_stats(h)
    log(f"tiles built in {t_build:.1f}s: items={st['n_items']} parts={st['n_parts']} "
        f"blob={st['blob_bytes'] / nnz:.2f} B/nnz")

    Xs, Ys = {}, {}
    for k in ks:
        Xs[k] = torch.from_numpy(synth.uniform(n, k, seed=synth.SEED_X)).to(dev)
        Ys[k] = torch.empty((n, k), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log("X/Y resident; first call uploads the tiles")

    stream = torch.cuda.current_stream(dev)
    for _ in range(max(args.warmup, 1)):
        for k in ks:
            pk.spmm_run(h, Xs[k], Ys[k], stream=stream)
    torch.cuda.synchronize()
    log("warmup done")

    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for k in ks}
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for s in range(args.steps):
        for k in ks:
            a, b = ev[k][s]
            a.record(stream)
            pk.spmm_run(h, Xs[k], Ys[k], stream=stream)
            b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_k = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k]])) for k in ks}
    log("timed: " + ", ".join(f"k={k}: {ms_k[k]:.3f} ms" for k in ks))

    flop_step = sum(2.0 * nnz * k for k in ks)
    ms_step = wall * 1e3 / args.steps
    value = flop_step / (ms_step * 1e-3) / 1e9

    max_kc = args.max_kc or 32
    per_k = {}
    for k in ks:
        mb = model_bytes(T, R, C, nnz, n, k)
        launches = -(-k // max_kc) if k > max_kc else 1
        per_k[str(k)] = {
            "ms": round(ms_k[k], 4),
            "gflops": round(2.0 * nnz * k / (ms_k[k] * 1e-3) / 1e9, 2),
            "model_gb": round(mb["total"] / 1e9, 4),
            "model_frac": round(mb["total"] / (ms_k[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "floor_frac": round(mb["floor"] / (ms_k[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launches": launches,
        }
    kdom = max(ks, key=lambda k: ms_k[k])
    mb = model_bytes(T, R, C, nnz, n, kdom)
    launches = per_k[str(kdom)]["launches"]
    # per launch: the whole A, this launch's share of the X columns and of Y
    kc = kdom // launches
    launch_bytes = mb["A"] + C * kc * 4 + n * kc * 4
    launch_ms = ms_k[kdom] / launches
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": f"spmm_items k={kdom} (kc={kc}, {launches} launch(es) per SpMM)",
                "bytes_per_launch": int(launch_bytes), "ms_per_launch": round(launch_ms, 4)}

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
        cpu = {"value": round(cpu_gflops, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"{sel.size} rows ({sel_nnz} nnz: rows 0-63 plus spread blocks), "
                         f"k sweep {ks}, FP64 single-threaded CSR loop, {t_cpu:.1f}s"}
        parity = {"rows": int(sel.size), "max_rel_frob_err": max(errs.values()), "per_k": errs,
                  "tolerance": 1e-6, "ok": max(errs.values()) <= 1e-6}
        log(f"cpu oracle {cpu_gflops:.2f} GFLOP/s over {t_cpu:.1f}s; parity max err {parity['max_rel_frob_err']:.3g}")

    out = {
        "metric": "SpMM GFLOP/s (2*nnz*k/s) over the k sweep, % HBM roofline",
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
                   "tile_rows": st["tile_rows"], "tile_cols": st["tile_cols"],
                   "variant": args.variant, "max_kc": max_kc},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "per_k": per_k,
        "tiles": {k: st[k] for k in ("n_tiles", "n_items", "n_parts", "blob_bytes", "sum_nnr", "sum_nnc")},
        "model_16k": {"tiles": T, "sum_nnr": R, "sum_nnc": C},
        "prep_s": {"generate": round(t_gen, 1), "model": round(t_model, 1), "build": round(t_build, 1)},
    }
    print(json.dumps(out), flush=True)
    h.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
