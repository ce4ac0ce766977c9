"""Learned threshold picker driver (training loop and picking on the GPU).

The arithmetic runs in libmcd.so: features, the FP32 MLP forward/backward/
Adam kernels, the grid snap, per-graph pruning and components.  This module
only sequences those calls.  The threshold grid is delta_i = (9 + 7 i) / 900,
i = 0..63 (64 evenly spaced values in [0.01, 0.5]); a picked index is the
network output snapped to that grid.

The full sweep is the picker's fallback: a graph whose features leave the
training range (widened by MARGIN of its width on each side) takes the
threshold the sweep's rule of thumb picks on the same grid instead.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import mcd as M

GRID_A, GRID_B, GRID_C, GRID_K = 9, 7, 900, 64
GRID = [(GRID_A + GRID_B * i, GRID_C) for i in range(GRID_K)]
MARGIN = 0.25  # of a feature's training range, on each side


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, drawn from the
    seeded counter-based generator of the input module."""
    import graphgen

    u = graphgen.uniforms(seed, 0x4D4C5030, M.MLP_PARAMS)  # "MLP0"
    p = np.zeros(M.MLP_PARAMS, np.float32)
    o = 0
    for fan_out, fan_in in ((64, 66), (64, 64), (1, 64)):
        k = fan_out * fan_in
        bound = math.sqrt(6.0 / fan_in)
        p[o:o + k] = ((2.0 * u[o:o + k] - 1.0) * bound).astype(np.float32)
        o += k + (fan_out if fan_out > 1 else 1)  # skip the bias block
    return p


class Picker:
    def __init__(self, params, mean, std, lo, hi, margin: float = MARGIN):
        self.params, self.mean, self.std = params, mean, std
        self.lo, self.hi, self.margin = lo, hi, margin  # training range of every feature


def train(ctx, x, y, steps: int = 2000, lr: float = 3e-3, seed: int = 0, weight_decay: float = 1.0,
          min_std: float = 1.0):
    """Full-batch Adam (decoupled weight decay) on (x, y) (device tensors);
    returns (Picker, losses)."""
    dev = ctx.device
    params = torch.from_numpy(init_params(seed)).to(dev)
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    mean, std = M.mcd_feature_stats(ctx, x, min_std)
    ws = torch.empty(M.mcd_mlp_workspace_size(x.shape[0]), dtype=torch.uint8, device=dev)
    loss = torch.empty(max(steps, 1), dtype=torch.float32, device=dev)
    for s in range(1, steps + 1):
        M.mcd_mlp_train_step(ctx, params, m1, m2, s, lr, mean, std, x, y, loss=loss[s - 1:s], ws=ws,
                             weight_decay=weight_decay)
    lo, hi = M.mcd_feature_range(ctx, x)
    return Picker(params, mean, std, lo, hi), loss.cpu().numpy()


def pick(g, t, picker: Picker, vbase=None, measure: int = M.MCD_SIM_TECTONIC, fallback: str = "auto"):
    """Features -> MLP -> grid snap -> range guard -> per-graph prune +
    components.  fallback: "auto" (the sweep's rule of thumb for graphs out of
    the training range; the sweep runs only if one is), "force" (for every
    graph) or "off".  Returns (index int32[G]: the network's grid index,
    deltas int64[G][2]: the thresholds used, labels int32[n], n_components,
    flags int32[G]: the range guard's decision, 1 = out of range; with "auto"
    exactly the graphs whose threshold the fallback decided)."""
    if fallback not in ("auto", "force", "off"):
        raise ValueError(f"fallback must be 'auto', 'force' or 'off', not {fallback!r}")
    ctx = g.ctx
    vb = M._vbase(g, vbase)
    x = M.mcd_features(g, t, vb)
    y = M.mcd_mlp_forward(ctx, picker.params, picker.mean, picker.std, x)
    index, deltas = M.mcd_grid_select(ctx, y, GRID_K, GRID_A, GRID_B, GRID_C)
    flags, _ = M.mcd_picker_fallback(ctx, x, picker.lo, picker.hi, picker.margin)
    if fallback == "force" or (fallback == "auto" and bool(flags.any())):
        stats, _, _, q = M.mcd_sweep(g, measure, t, GRID, vbase=vb, want_modularity=True)
        _, rule_delta = M.mcd_sweep_rule(ctx, GRID, stats, q, vbase=vb)
        if fallback == "force":
            deltas = rule_delta
        else:
            M.mcd_picker_fallback(ctx, x, picker.lo, picker.hi, picker.margin, picked=deltas, fallback=rule_delta,
                                  delta=deltas, flags=flags)
    r = M.mcd_prune_components(g, measure, t, deltas=deltas, vbase=vb, want_f32=False, want_keep=False)
    return index, deltas, r["labels"], r["n_components"], flags
