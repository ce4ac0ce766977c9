"""Learned threshold picker: a thin wrapper over the library's mcd_picker.

Everything runs in libmcd.so: the seeded He-uniform initialisation, the
standardisation and training range, the FP32 MLP training loop (forward,
backward and Adam kernels), and the pick sequence (features, network, grid
snap, range guard, the sweep's rule of thumb where the guard fires, prune and
components).  The threshold grid is delta_i = (9 + 7 i) / 900, i = 0..63
(64 evenly spaced values in [0.01, 0.5]); a picked index is the network
output snapped to that grid.

The full sweep is the picker's fallback: a graph whose features leave the
training range (widened by MARGIN of its width on each side) takes the
threshold the sweep's rule of thumb picks on the same grid instead.
"""
from __future__ import annotations

from . import mcd as M

GRID_A, GRID_B, GRID_C, GRID_K = M.PICKER_GRID_A, M.PICKER_GRID_B, M.PICKER_GRID_C, M.PICKER_GRID_K
GRID = [(GRID_A + GRID_B * i, GRID_C) for i in range(GRID_K)]
MARGIN = M.PICKER_MARGIN  # of a feature's training range, on each side
_MODES = {"auto": M.MCD_PICK_AUTO, "force": M.MCD_PICK_FORCE_SWEEP, "off": M.MCD_PICK_NETWORK}


class Picker:
    """A library picker plus device copies of its state (params, mean, std,
    lo, hi) for callers that run the kernels one by one."""

    def __init__(self, handle: M.PickerHandle):
        self.handle = handle
        self.refresh()

    def refresh(self):
        st = M.mcd_picker_export(self.handle)
        self.params, self.mean, self.std = st["params"], st["mean"], st["std"]
        self.lo, self.hi, self.margin = st["lo"], st["hi"], st["margin"]

    def save(self, path: str):
        M.mcd_picker_save(self.handle, path)


def train(ctx, x, y, ari=None, steps: int = 2000, lr: float = 3e-3, seed: int = 0, weight_decay: float | None = None,
          min_std: float = 1.0, mse_weight: float | None = None):
    """Full-batch Adam (decoupled weight decay) from the seeded initial
    weights on features x and targets y (device tensors); with the training
    graphs' ARI table over the grid (ari, float64 [B][64]) the loss also
    rewards the ARI at the network's threshold (mse_weight 0.1, weight decay
    0.1 by default), else it is the squared error to y (weight decay 1).
    Returns (Picker, losses as numpy)."""
    if weight_decay is None:
        weight_decay = 1.0 if ari is None else 0.1
    if mse_weight is None:
        mse_weight = 1.0 if ari is None else 0.1
    h = M.mcd_picker_create(ctx, seed)
    losses = M.mcd_picker_fit(h, x, y, steps, lr, weight_decay, min_std, MARGIN, ari=ari, mse_weight=mse_weight)
    return Picker(h), losses.cpu().numpy()


def load(ctx, path: str) -> Picker:
    """A picker from a checkpoint written by Picker.save."""
    h = M.mcd_picker_create(ctx, 0)
    M.mcd_picker_load(h, path)
    return Picker(h)


def pick(g, t, picker: Picker, vbase=None, measure: int = M.MCD_SIM_TECTONIC, fallback: str = "auto", ws=None):
    """Features -> MLP -> grid snap -> range guard -> per-graph prune +
    components.  fallback: "auto" (the sweep's rule of thumb for graphs out of
    the training range; the sweep runs only if one is), "force" (for every
    graph) or "off" (the network for every graph).  Returns (index int32[G]:
    the network's grid index, deltas int64[G][2]: the thresholds used, labels
    int32[n], n_components, used int32[G]: 1 where the sweep's threshold was
    used)."""
    if fallback not in _MODES:
        raise ValueError(f"fallback must be 'auto', 'force' or 'off', not {fallback!r}")
    index, deltas, used, labels, ncc = M.mcd_picker_pick(picker.handle, g, measure, t, vbase=vbase,
                                                         mode=_MODES[fallback], ws=ws)
    return index, deltas, labels, ncc, used
