#!/usr/bin/env python3
"""Benchmark: Tectonic pipeline (Algorithm 1 of arXiv 2412.12382) on R-MAT.

Workload (default): R-MAT scale 26, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05),
seeded vertex permutation, raw directed pairs resident in HBM.  One step is one
full pass of the path on the GPU:
    graph build (canonicalise + dedup + degree rank + orientation CSR)
    -> per-edge triangle counts -> Tectonic weights -> prune at delta
    -> connected components (min-vertex labels).
value = undirected edges m / step time (edges/s).  Per-kernel HIP-event times
give the roofline of the dominant kernel (triangle counting) and of the
weight+prune+components part.

Prints ONE JSON line (stdout).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--delta", type=str, default="3/50", help="Tectonic threshold num/den")
    ap.add_argument("--cpu-scale", type=int, default=20, help="R-MAT scale of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(scale: int, ef: int, seed: int, num: int, den: int):
    """The oracle (plain C, OpenMP) on a bounded sample of the same workload
    family: R-MAT at a smaller scale, same generator and threshold."""
    import graphgen as gg
    import oracle

    src, dst, n = gg.rmat(scale, ef, seed=seed)
    tm = {}
    t0 = time.perf_counter()
    r = oracle.run(n, src, dst, oracle.TECTONIC, num, den, tm)
    dt = time.perf_counter() - t0
    m = len(r["lo"])
    return dict(value=m / dt, unit="edges/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"R-MAT scale {scale} edge factor {ef} (n={n}, m={m}), full pipeline "
                       f"(canonicalise, triangles, Tectonic, prune {num}/{den}, BFS components), "
                       f"{dt:.2f} s",
                seconds=dt, stages_s={k: round(v, 3) for k, v in tm.items()})


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is "
              f"described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import graphgen as gg
    import paper_2412_12382_amd.mcd as M

    num, den = (int(x) for x in args.delta.split("/"))
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    log(f"generating R-MAT scale {args.scale} edge factor {args.edge_factor} on the host")
    t0 = time.perf_counter()
    src_h, dst_h, n = gg.rmat(args.scale, args.edge_factor, seed=args.seed)
    P = len(src_h)
    log(f"generated {P} pairs in {time.perf_counter() - t0:.1f} s; copying to HBM")
    src = torch.from_numpy(src_h).to(dev)
    dst = torch.from_numpy(dst_h).to(dev)
    del src_h, dst_h
    torch.cuda.synchronize()

    ctx = M.mcd_ctx_create(0)
    st_b, ws_b = M.mcd_graph_build_sizes(P, n)
    storage = torch.empty(st_b, dtype=torch.uint8, device=dev)
    ws = torch.empty(ws_b, dtype=torch.uint8, device=dev)
    t = torch.empty(P, dtype=torch.int32, device=dev)
    wf = torch.empty(P, dtype=torch.float32, device=dev)
    keep = torch.empty((P + 31) // 32 + 1, dtype=torch.int32, device=dev)
    n_kept = torch.empty(1, dtype=torch.int64, device=dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    ncc = torch.empty(1, dtype=torch.int64, device=dev)
    log(f"HBM in use after allocation: {torch.cuda.memory_allocated() / 2**30:.1f} GiB")

    ev = lambda: torch.cuda.Event(enable_timing=True)
    stage_names = ["build", "triangles", "weights", "prune", "components"]

    def step():
        e = [ev() for _ in range(len(stage_names) + 1)]
        e[0].record()
        g = M.mcd_graph_build(ctx, src, dst, n, storage=storage, ws=ws)
        e[1].record()
        M.mcd_triangles(g, t)
        e[2].record()
        M.mcd_weights(g, M.MCD_SIM_TECTONIC, t, w_f32=wf)
        e[3].record()
        M.mcd_prune(g, M.MCD_SIM_TECTONIC, t, (num, den), keep, n_kept)
        e[4].record()
        M.mcd_components(g, keep, labels, ncc, ws=ws)
        e[5].record()
        return g, e

    for i in range(args.warmup):
        g, _ = step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done (m={g.m})")

    torch.cuda.synchronize()
    stage_ms = {k: [] for k in stage_names}
    t_start = time.perf_counter()
    for i in range(args.steps):
        g, e = step()
        torch.cuda.synchronize()
        for j, k in enumerate(stage_names):
            stage_ms[k].append(e[j].elapsed_time(e[j + 1]))
        log(f"step {i + 1}/{args.steps}: " + ", ".join(f"{k} {stage_ms[k][-1]:.1f} ms" for k in stage_names))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    m = g.m
    avg = {k: float(np.mean(v)) for k, v in stage_ms.items()}

    # algorithmic bytes of the triangle kernel: the lists a merge-based
    # intersection streams for every oriented edge u->v (suffix of N+(u) after
    # v, all of N+(v)), plus t written, src/adj of the edge and row offsets.
    u, v = M.mcd_graph_edges(g)
    outd = torch.bincount(u.long(), minlength=n).double()
    ind = torch.bincount(v.long(), minlength=n).double()
    W = float((outd * (outd - 1) / 2).sum() + (ind * outd).sum())
    del u, v, outd, ind
    tc_bytes = 4.0 * W + 12.0 * m + 8.0 * (n + 1)
    tc_gbs = tc_bytes / (avg["triangles"] * 1e-3) / 1e9
    kept = int(n_kept.item())
    # weight+prune+components: t, src, adj read; deg gathered for both ends;
    # w written; keep bits written and read; kept edges' endpoints re-read by
    # the union step; parent init/finalise and labels over n.
    wpc_bytes = (4.0 * m * 5 + 4.0 * m) + (m / 8.0) * 2 + 8.0 * kept + 16.0 * n
    wpc_ms = avg["weights"] + avg["prune"] + avg["components"]
    wpc_gbs = wpc_bytes / (wpc_ms * 1e-3) / 1e9
    ncomp = int(ncc.item())
    log(f"m={m} kept={kept} components={ncomp} W={W:.3e} tc {tc_gbs:.0f} GB/s, wpc {wpc_gbs:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle on R-MAT scale {args.cpu_scale}")
        cpu = cpu_baseline(args.cpu_scale, args.edge_factor, args.seed, num, den)
        log(f"oracle: {cpu['value']:.3e} edges/s on {cpu['cores']} threads ({cpu['seconds']:.1f} s)")

    out = {
        "metric": "edges/s (weight+prune+CC) R-MAT s26; ARI & latency learned vs swept threshold",
        "value": m / (ms_per_step * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {args.scale}, edge factor {args.edge_factor}, "
                               f"(a,b,c,d)=(0.57,0.19,0.19,0.05), symmetrised, deduplicated; "
                               f"Tectonic weights, prune at {num}/{den}, components",
                   "n": n, "m": m, "pairs": P, "delta": f"{num}/{den}",
                   "step": "build+triangles+weights+prune+components"},
        "stages_ms": {k: round(v, 3) for k, v in avg.items()},
        "wpc_edges_per_s": m / (wpc_ms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": tc_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": tc_gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "triangles",
                     "algorithmic_bytes": tc_bytes, "W": W},
        "roofline_wpc": {"bound": "hbm", "achieved": wpc_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": wpc_gbs / HBM_PEAK_GBS, "algorithmic_bytes": wpc_bytes},
        "results": {"n_kept": kept, "n_components": ncomp},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
