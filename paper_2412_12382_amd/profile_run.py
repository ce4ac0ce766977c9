"""Driver for hardware-counter and kernel-trace runs of the pipeline.

Runs, on R-MAT of the given scale: one calibration kernel of known traffic
(an elementwise int32 add over `--copy-mib` MiB: that many bytes read and
written), the graph build, the triangle count, the one-pass weights + prune +
components at num/den (default 9/900) and the 16-point sweep, each once, and
prints what it launched; with `--k4` also the 4-clique participation count.
Used as
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
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--k4", action="store_true", help="also count 4-cliques per edge")
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--num", type=int, default=9, help="prune threshold numerator")
    ap.add_argument("--den", type=int, default=900, help="prune threshold denominator")
    args = ap.parse_args()
    import torch

    import graphgen as gg
    import paper_2412_12382_amd.mcd as M

    dev = torch.device("cuda", 0)
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
    r = M.mcd_prune_components(g, M.MCD_SIM_TECTONIC, t, delta=(args.num, args.den))
    ncc, nk = r["n_components"], r["n_kept"]
    M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, [(k, 50) for k in range(16)])
    if args.k4:
        M.mcd_k4(g)
    torch.cuda.synchronize()
    print(json.dumps(dict(scale=args.scale, n=n, m=g.m, kept=int(nk.item()), components=int(ncc.item()))),
          flush=True)


if __name__ == "__main__":
    main()
