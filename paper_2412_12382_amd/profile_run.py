"""Driver for hardware-counter and kernel-trace runs of the pipeline.

Runs, on R-MAT of the given scale: one calibration kernel of known traffic
(an elementwise int32 add over `--copy-mib` MiB: that many bytes read and
written), the graph build, the triangle count, the one-pass weights + prune +
components once per threshold of `--passes` (default: Tectonic at 1/50, at 0
so that every edge is kept, and TW at -10), and the 16-point sweep, each
once, and prints what it launched; with `--k4` also the 4-clique
participation count.
With `--workload dcsbm` or `--workload batch` it runs instead the 64-threshold
sweep with ARI on the degree-corrected SBM (n = 10^6, with modularity and F1)
or on the 256-graph planted batch.  Used as
    rocprofv3 --kernel-trace --stats -- python3 -m paper_2412_12382_amd.profile_run
    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2412_12382_amd.profile_run
    rocprofv3 --pmc WRITE_SIZE -- python3 -m paper_2412_12382_amd.profile_run
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat", choices=["rmat", "dcsbm", "batch"],
                    help="rmat: the pipeline on R-MAT; dcsbm / batch: the 64-threshold sweep with ARI (and, on "
                         "the degree-corrected SBM, modularity and F1) on the degree-corrected SBM or the "
                         "256-graph planted batch")
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--k4", action="store_true", help="also count 4-cliques per edge")
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--passes", default="tectonic:1/50,tectonic:0/1,tw:-10/1",
                    help="weights + prune + components passes, measure:num/den, comma separated")
    args = ap.parse_args()
    import torch

    import graphgen as gg
    import paper_2412_12382_amd.mcd as M

    dev = torch.device("cuda", 0)
    if args.workload != "rmat":
        import numpy as np
        cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        w = gg.dcsbm() if args.workload == "dcsbm" else gg.sbm_batch(256)
        n = w["n"]
        vb = cu(w["vbase"]) if "vbase" in w else torch.tensor([0, n], dtype=torch.int64, device=dev)
        truth = cu(w["truth"].astype(np.int32))
        ctx = M.mcd_ctx_create(0)
        g = M.mcd_graph_build(ctx, cu(w["src"]), cu(w["dst"]), n)
        t = M.mcd_triangles(g)
        grid = [(9 + 7 * i, 900) for i in range(64)]
        extra = args.workload == "dcsbm"
        out = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, grid, vbase=vb, truth=truth, want_modularity=extra,
                          want_prf=extra)
        torch.cuda.synchronize()
        print(json.dumps(dict(workload=args.workload, n=n, m=g.m, graphs=vb.numel() - 1,
                              best_ari_mean=float(out[1].max(1).values.mean().item()))), flush=True)
        return
    n_el = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n_el, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    torch.add(a, 1, out=b)  # calibration: reads and writes copy_mib MiB
    torch.cuda.synchronize()
    print(f"calibration add: {args.copy_mib} MiB read, {args.copy_mib} MiB written", flush=True)
    del a, b
    s, d, n = gg.rmat(args.scale, seed=args.seed)
    src, dst = torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev)
    del s, d
    ctx = M.mcd_ctx_create(0)
    g = M.mcd_graph_build(ctx, src, dst, n)
    t = M.mcd_triangles(g)
    done = []
    for item in args.passes.split(","):
        name, frac = item.split(":")
        num, den = (int(v) for v in frac.split("/"))
        measure = {"tectonic": M.MCD_SIM_TECTONIC, "tw": M.MCD_SIM_TW}[name]
        r = M.mcd_prune_components(g, measure, t, delta=(num, den), want_i32=(measure == M.MCD_SIM_TW),
                                   want_f32=(measure == M.MCD_SIM_TECTONIC))
        torch.cuda.synchronize()
        done.append(dict(measure=name, delta=[num, den], kept=int(r["n_kept"].item()),
                         components=int(r["n_components"].item())))
        print(f"prune_components {name} {num}/{den}: {done[-1]}", flush=True)
        del r
    M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, [(k, 50) for k in range(16)])
    if args.k4:
        M.mcd_k4(g)
    torch.cuda.synchronize()
    print(json.dumps(dict(scale=args.scale, n=n, m=g.m, passes=done)), flush=True)


if __name__ == "__main__":
    main()
