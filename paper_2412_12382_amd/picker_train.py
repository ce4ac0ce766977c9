"""Training set and training run of the learned threshold picker.

The picker learns, from a graph's features (the 64-bin Tectonic histogram
and its mean and maximum degree), the threshold of the grid (9 + 7 i) / 900
at which Algorithm 1's partition best matches the planted one.  Its training
graphs are planted partitions whose sweep over the grid, scored by ARI
against the planted labels, supplies both the target and the loss:

  * the 192 training graphs of the 256-graph planted batch (graphs g with
    g % 4 != 3; the others are the validation graphs and are never trained on);
  * n_extra further graphs of the same distribution (graphs 256, 257, ...;
    11,264 by default, so graphs 256 .. 11,519);
  * n_dcsbm small degree-corrected SBMs (power-law degrees and community
    sizes, seeded from 5000), so that heavy-tailed graphs fall inside the
    range the picker was trained on.

Everything on the GPU runs in libmcd.so (graph build, triangle counts, the
sweep with ARI, features, the MLP training kernels); this module generates
the inputs and sequences the calls.

    python -m paper_2412_12382_amd.picker_train --out picker.ckpt
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from . import mcd as M  # noqa: E402
from . import picker as PK  # noqa: E402


def _disjoint_union(graphs):
    srcs, dsts, truths, vbase, cbase = [], [], [], [0], 0
    for w in graphs:
        srcs.append(w["src"] + vbase[-1])
        dsts.append(w["dst"] + vbase[-1])
        truths.append(w["truth"].astype(np.int64) + cbase)
        cbase += int(w["truth"].max()) + 1
        vbase.append(vbase[-1] + w["n"])
    return dict(src=np.concatenate(srcs).astype(np.int32), dst=np.concatenate(dsts).astype(np.int32),
                n=vbase[-1], vbase=np.array(vbase, np.int64), truth=np.concatenate(truths).astype(np.int32))


def dcsbm_params(k: int):
    """Parameters of the k-th small degree-corrected SBM of the training set
    (seed 5000 + k): n log-uniform in [1e4, 2e5], mean degree U[8, 30],
    maximum degree U[300, 3000], mixing U[0.05, 0.5]."""
    import graphgen as gg
    u = gg.uniforms(5000 + k, 0x50494B44, 4)  # "PIKD"
    n = int(np.exp(np.log(1e4) + u[0] * (np.log(2e5) - np.log(1e4))))
    return dict(n=n, mean_deg=8.0 + 22.0 * u[1], max_deg=300.0 + 2700.0 * u[2], mu=0.05 + 0.45 * u[3],
                seed=5000 + k)


def sweep_batch(ctx, b, dev):
    """Features and 64-threshold ARI table of a batch of planted graphs."""
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    vb = cu(b["vbase"])
    g = M.mcd_graph_build(ctx, cu(b["src"]), cu(b["dst"]), b["n"])
    t = M.mcd_triangles(g)
    _, ari, _ = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, PK.GRID, vbase=vb, truth=cu(b["truth"]))
    x = M.mcd_features(g, t, vb)
    return x, ari


def training_set(ctx, n_extra: int = 11264, n_dcsbm: int = 512, log=None):
    """(x float32 [B][66], y float32 [B], ari float64 [B][64]) on the device:
    the C4 training graphs, n_extra more of their distribution and n_dcsbm
    degree-corrected ones."""
    import graphgen as gg
    dev = ctx.device
    xs, aris = [], []
    t0 = time.perf_counter()
    b = gg.sbm_batch(256)
    x, ari = sweep_batch(ctx, b, dev)
    keep = torch.tensor([g for g in range(256) if g % 4 != 3], device=dev)
    xs.append(x[keep])
    aris.append(ari[keep])
    for first in range(256, 256 + n_extra, 256):
        x, ari = sweep_batch(ctx, gg.sbm_batch(min(256, 256 + n_extra - first), first=first), dev)
        xs.append(x)
        aris.append(ari)
    for k0 in range(0, n_dcsbm, 64):
        graphs = []
        for k in range(k0, min(k0 + 64, n_dcsbm)):
            pr = dcsbm_params(k)
            graphs.append(gg.dcsbm(n=pr["n"], mean_deg=pr["mean_deg"], max_deg=pr["max_deg"], mu=pr["mu"],
                                   seed=pr["seed"]))
        x, ari = sweep_batch(ctx, _disjoint_union(graphs), dev)
        xs.append(x)
        aris.append(ari)
    x = torch.cat(xs).contiguous()
    ari = torch.cat(aris).contiguous()
    _, y = M.mcd_sweep_targets(ctx, ari)
    if log:
        log(f"picker training set: {x.shape[0]} graphs in {time.perf_counter() - t0:.1f} s")
    return x, y, ari


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="checkpoint file to write")
    ap.add_argument("--extra", type=int, default=11264)
    ap.add_argument("--dcsbm", type=int, default=512)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    ctx = M.mcd_ctx_create(0)
    x, y, ari = training_set(ctx, args.extra, args.dcsbm, log=print)
    model, losses = PK.train(ctx, x, y, ari=ari, steps=args.steps, seed=args.seed)
    model.save(args.out)
    print(f"trained on {x.shape[0]} graphs, loss {losses[0]:.4f} -> {losses[-1]:.4f}; wrote {args.out}")


if __name__ == "__main__":
    main()
