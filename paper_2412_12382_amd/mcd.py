"""Thin ctypes binding of libmcd.so (include/mcd.h).

Functions carry the C names and only marshal arguments: torch tensors supply
device memory (``data_ptr``) and the stream; every step runs in the HIP
library.  Outputs that the caller does not pass are allocated as torch
tensors on the context's device.  There is no CPU fallback: if the library is
not built, importing raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcd.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mcd.h")

MCD_SIM_TECTONIC = 0
MCD_SIM_TW = 1
MCD_SIM_K3 = 2
MCD_SIM_JACCARD = 3
MCD_SIM_K4 = 4

STATUS = {0: "MCD_OK", -1: "MCD_ERR_INVALID_ARG", -2: "MCD_ERR_INVALID_VERTEX", -3: "MCD_ERR_RANGE",
          -4: "MCD_ERR_WORKSPACE", -5: "MCD_ERR_NO_DEVICE", -6: "MCD_ERR_DEVICE",
          -7: "MCD_ERR_NOT_CONVERGED", -8: "MCD_ERR_EMPTY", -9: "MCD_ERR_CHECKPOINT"}


class MCDError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class mcd_rational(ctypes.Structure):
    _fields_ = [("num", ctypes.c_int64), ("den", ctypes.c_int64)]


SWEEP_FIELDS = ("m_kept", "n_components", "largest_component", "pairs_cluster", "pairs_class",
                "pairs_both", "pairs_total", "intra_edges", "volume_sq")
SWEEP_MAX = 64


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2412_12382_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "mcd_ctx_create": [ctypes.c_int, P, PP],
            "mcd_ctx_set_stream": [P, P],
            "mcd_ctx_set_param": [P, ctypes.c_char_p, I64],
            "mcd_ctx_get_param": [P, ctypes.c_char_p, ctypes.POINTER(I64)],
            "mcd_triangles_workspace_size": [P, ctypes.POINTER(SZ)],
            "mcd_ctx_destroy": [P],
            "mcd_graph_build_sizes": [I64, I64, ctypes.POINTER(SZ), ctypes.POINTER(SZ)],
            "mcd_graph_build": [P, P, P, I64, I64, P, SZ, P, SZ, PP],
            "mcd_graph_info": [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I32),
                               ctypes.POINTER(I32)],
            "mcd_graph_edges": [P, P, P],
            "mcd_graph_degrees": [P, P],
            "mcd_graph_perm": [P, P],
            "mcd_graph_destroy": [P],
            "mcd_triangles": [P, P, P, SZ],
            "mcd_weights": [P, ctypes.c_int, P, P, P],
            "mcd_prune": [P, ctypes.c_int, P, mcd_rational, P, P],
            "mcd_components_workspace_size": [P, ctypes.POINTER(SZ)],
            "mcd_run_workspace_size": [P, ctypes.POINTER(SZ)],
            "mcd_components": [P, P, P, P, P, SZ],
            "mcd_run": [P, ctypes.c_int, mcd_rational, P, P, P, SZ],
            "mcd_percentile_workspace_size": [P, ctypes.POINTER(SZ)],
            "mcd_sweep_workspace_size": [P, I32, I32, I32, ctypes.POINTER(SZ)],
            "mcd_sweep": [P, ctypes.c_int, P, P, I32, I32, P, P, P, P, P, P, P, P, SZ],
            "mcd_sweep_rule": [P, P, I32, I32, P, P, P, I64, I64, P, P],
            "mcd_features_workspace_size": [I32, ctypes.POINTER(SZ)],
            "mcd_features": [P, P, I32, P, P, P, SZ],
            "mcd_feature_stats": [P, P, I32, ctypes.c_float, P, P],
            "mcd_feature_range": [P, P, I32, P, P],
            "mcd_picker_fallback": [P, P, I32, P, P, ctypes.c_float, P, P, P, P],
            "mcd_mlp_forward": [P, P, P, P, P, I32, P],
            "mcd_mlp_workspace_size": [I32, ctypes.POINTER(SZ)],
            "mcd_mlp_gradient": [P, P, P, P, P, P, P, I32, ctypes.c_float, I32, P, P, P, SZ],
            "mcd_mlp_train_step": [P, P, P, P, I32, ctypes.c_float, ctypes.c_float, P, P, P, P, P, I32,
                                   ctypes.c_float, I32, P, P, SZ],
            "mcd_grid_select": [P, P, I32, I32, I64, I64, I64, P, P],
            "mcd_sweep_targets": [P, P, I32, I32, ctypes.c_double, P, P],
            "mcd_prune_graphs": [P, ctypes.c_int, P, I32, P, P, P, P],
            "mcd_weigh_prune": [P, ctypes.c_int, P, mcd_rational, I32, P, P, P, P, P, P, P, P],
            "mcd_kept_segment_len": [P, ctypes.POINTER(I64)],
            "mcd_components_kept": [P, P, P, P, P, P, SZ],
            "mcd_tune_triangles_workspace_size": [P, ctypes.POINTER(SZ)],
            "mcd_k4": [P, P],
            "mcd_prune_components": [P, ctypes.c_int, P, mcd_rational, I32, P, P, P, P, P, P, P, P, P, SZ],
            "mcd_prune_components_noalloc": [P, ctypes.c_int, P, mcd_rational, I32, P, P, P, P, P, P, P, P],
            "mcd_tune_triangles": [P, P, P, SZ, I32, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_float)],
            "mcd_percentile_threshold": [P, ctypes.c_int, P, I64, I64, P, SZ, ctypes.POINTER(mcd_rational)],
            "mcd_picker_create": [P, ctypes.c_uint64, PP],
            "mcd_picker_destroy": [P],
            "mcd_picker_prepare": [P, P, I32, ctypes.c_float, ctypes.c_float],
            "mcd_picker_train_step": [P, P, P, P, ctypes.c_float, I32, ctypes.c_float, ctypes.c_float, P, P, SZ],
            "mcd_picker_fit": [P, P, P, P, ctypes.c_float, I32, I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, P, P, SZ],
            "mcd_picker_forward": [P, P, I32, P],
            "mcd_picker_pick_workspace_size": [P, I32, ctypes.POINTER(SZ)],
            "mcd_picker_pick": [P, P, ctypes.c_int, P, I32, P, I32, P, P, P, P, P, P, SZ],
            "mcd_picker_export": [P, P, P, P, P, P, ctypes.POINTER(ctypes.c_float)],
            "mcd_picker_import": [P, P, P, P, P, P, ctypes.c_float],
            "mcd_picker_save": [P, ctypes.c_char_p],
            "mcd_picker_load": [P, ctypes.c_char_p],
            "mcd_picker_check_file": [ctypes.c_char_p],
            "mcd_tune_cache_load": [P, P, ctypes.c_char_p, ctypes.POINTER(I32)],
            "mcd_tune_cache_store": [P, P, ctypes.c_char_p, ctypes.c_float],
            "mcd_tune_cache_check_file": [ctypes.c_char_p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.mcd_status_string.argtypes = [ctypes.c_int32]
        L.mcd_status_string.restype = ctypes.c_char_p
        L.mcd_last_error.argtypes = []
        L.mcd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/mcd.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcd_[a-z0-9_]+)\s*\(", text)))


def _check(status: int):
    if status != 0:
        raise MCDError(status, lib().mcd_last_error().decode())


def _p(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(device: torch.device, stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    def __init__(self, handle, device: torch.device):
        self.handle = handle
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcd_ctx_destroy(self.handle)
            self.handle = None


@dataclass
class Graph:
    handle: ctypes.c_void_p
    ctx: Context
    storage: torch.Tensor
    n: int
    m: int
    max_deg: int
    max_outdeg: int

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcd_graph_destroy(self.handle)
            self.handle = None


def _rat(delta) -> mcd_rational:
    num, den = delta
    return mcd_rational(int(num), int(den))


def _empty(shape, dtype, device):
    return torch.empty(shape, dtype=dtype, device=device)


def _bytes(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ context

def mcd_ctx_create(device: int = 0, stream=None) -> Context:
    dev = torch.device("cuda", device)
    h = ctypes.c_void_p()
    _check(lib().mcd_ctx_create(device, _stream_handle(dev, stream), ctypes.byref(h)))
    return Context(h, dev)


def mcd_ctx_set_stream(ctx: Context, stream) -> None:
    _check(lib().mcd_ctx_set_stream(ctx.handle, _stream_handle(ctx.device, stream)))


def mcd_ctx_set_param(ctx: Context, name: str, value: int) -> None:
    _check(lib().mcd_ctx_set_param(ctx.handle, name.encode(), int(value)))


def mcd_ctx_get_param(ctx: Context, name: str) -> int:
    v = ctypes.c_int64()
    _check(lib().mcd_ctx_get_param(ctx.handle, name.encode(), ctypes.byref(v)))
    return v.value


# -------------------------------------------------------------------- graph

def mcd_graph_build_sizes(n_pairs: int, n_vertices: int) -> tuple[int, int]:
    st, ws = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().mcd_graph_build_sizes(n_pairs, n_vertices, ctypes.byref(st), ctypes.byref(ws)))
    return st.value, ws.value


def mcd_graph_build(ctx: Context, src: torch.Tensor, dst: torch.Tensor, n_vertices: int,
                    storage: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> Graph:
    assert src.dtype == torch.int32 and dst.dtype == torch.int32 and src.is_contiguous() and dst.is_contiguous()
    assert src.numel() == dst.numel() and src.device == ctx.device and dst.device == ctx.device
    P = src.numel()
    st_b, ws_b = mcd_graph_build_sizes(P, n_vertices)
    if storage is None:
        storage = _bytes(st_b, ctx.device)
    own_ws = ws is None
    if own_ws:
        ws = _bytes(ws_b, ctx.device)
    h = ctypes.c_void_p()
    _check(lib().mcd_graph_build(ctx.handle, _p(src), _p(dst), P, n_vertices, _p(storage),
                                 storage.numel() * storage.element_size(), _p(ws),
                                 ws.numel() * ws.element_size(), ctypes.byref(h)))
    if own_ws:
        del ws
    n, m = ctypes.c_int64(), ctypes.c_int64()
    md, mo = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mcd_graph_info(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(md), ctypes.byref(mo)))
    return Graph(h, ctx, storage, n.value, m.value, md.value, mo.value)


def mcd_graph_info(g: Graph) -> dict:
    return dict(n=g.n, m=g.m, max_deg=g.max_deg, max_outdeg=g.max_outdeg)


def mcd_graph_edges(g: Graph, u=None, v=None):
    u = _empty(max(g.m, 1), torch.int32, g.ctx.device) if u is None else u
    v = _empty(max(g.m, 1), torch.int32, g.ctx.device) if v is None else v
    _check(lib().mcd_graph_edges(g.handle, _p(u), _p(v)))
    return u[:g.m], v[:g.m]


def mcd_graph_degrees(g: Graph, deg=None):
    deg = _empty(max(g.n, 1), torch.int32, g.ctx.device) if deg is None else deg
    _check(lib().mcd_graph_degrees(g.handle, _p(deg)))
    return deg[:g.n]


def mcd_graph_perm(g: Graph, perm=None):
    perm = _empty(max(g.n, 1), torch.int32, g.ctx.device) if perm is None else perm
    _check(lib().mcd_graph_perm(g.handle, _p(perm)))
    return perm[:g.n]


# -------------------------------------------------------------------- steps

def mcd_triangles_workspace_size(g: Graph) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_triangles_workspace_size(g.handle, ctypes.byref(b)))
    return b.value


def mcd_triangles(g: Graph, t=None, ws=None):
    t = _empty(max(g.m, 1), torch.int32, g.ctx.device) if t is None else t
    if ws is None:
        ws = _bytes(mcd_triangles_workspace_size(g), g.ctx.device)
    _check(lib().mcd_triangles(g.handle, _p(t), _p(ws), ws.numel() * ws.element_size()))
    return t[:g.m]


def mcd_k4(g: Graph, k4=None):
    """Number of 4-cliques containing every edge (library edge order)."""
    k4 = _empty(max(g.m, 1), torch.int32, g.ctx.device) if k4 is None else k4
    _check(lib().mcd_k4(g.handle, _p(k4)))
    return k4[:g.m]


def mcd_weights(g: Graph, measure: int, t, w_f32=None, w_i32=None, want_f32=True, want_i32=False):
    if w_f32 is None and want_f32:
        w_f32 = _empty(max(g.m, 1), torch.float32, g.ctx.device)
    if w_i32 is None and want_i32:
        w_i32 = _empty(max(g.m, 1), torch.int32, g.ctx.device)
    _check(lib().mcd_weights(g.handle, measure, _p(t), _p(w_f32), _p(w_i32)))
    return (None if w_f32 is None else w_f32[:g.m]), (None if w_i32 is None else w_i32[:g.m])


def mcd_prune(g: Graph, measure: int, t, delta, keep_bits=None, n_kept=None):
    words = max((g.m + 31) // 32, 1)
    keep_bits = _empty(words, torch.int32, g.ctx.device) if keep_bits is None else keep_bits
    n_kept = _empty(1, torch.int64, g.ctx.device) if n_kept is None else n_kept
    _check(lib().mcd_prune(g.handle, measure, _p(t), _rat(delta), _p(keep_bits), _p(n_kept)))
    return keep_bits, n_kept


def mcd_components_workspace_size(g: Graph) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_components_workspace_size(g.handle, ctypes.byref(b)))
    return b.value


def mcd_run_workspace_size(g: Graph) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_run_workspace_size(g.handle, ctypes.byref(b)))
    return b.value


def mcd_components(g: Graph, keep_bits=None, labels=None, n_components=None, ws=None):
    labels = _empty(max(g.n, 1), torch.int32, g.ctx.device) if labels is None else labels
    n_components = _empty(1, torch.int64, g.ctx.device) if n_components is None else n_components
    if ws is None:
        ws = _bytes(mcd_components_workspace_size(g), g.ctx.device)
    _check(lib().mcd_components(g.handle, _p(keep_bits), _p(labels), _p(n_components), _p(ws),
                                ws.numel() * ws.element_size()))
    return labels[:g.n], n_components


def mcd_run(g: Graph, measure: int, delta, labels=None, n_components=None, ws=None):
    labels = _empty(max(g.n, 1), torch.int32, g.ctx.device) if labels is None else labels
    n_components = _empty(1, torch.int64, g.ctx.device) if n_components is None else n_components
    if ws is None:
        ws = _bytes(mcd_run_workspace_size(g), g.ctx.device)
    _check(lib().mcd_run(g.handle, measure, _rat(delta), _p(labels), _p(n_components), _p(ws),
                         ws.numel() * ws.element_size()))
    return labels[:g.n], n_components


def mcd_percentile_workspace_size(g: Graph) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_percentile_workspace_size(g.handle, ctypes.byref(b)))
    return b.value


def mcd_percentile_threshold(g: Graph, measure: int, t, pct_num: int, pct_den: int, ws=None):
    if ws is None:
        ws = _bytes(mcd_percentile_workspace_size(g), g.ctx.device)
    out = mcd_rational()
    _check(lib().mcd_percentile_threshold(g.handle, measure, _p(t), pct_num, pct_den, _p(ws),
                                          ws.numel() * ws.element_size(), ctypes.byref(out)))
    return out.num, out.den


def mcd_sweep_workspace_size(g: Graph, n_graphs: int, K: int, has_truth: bool) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_sweep_workspace_size(g.handle, n_graphs, K, int(has_truth), ctypes.byref(b)))
    return b.value


def mcd_sweep(g: Graph, measure: int, t, deltas, vbase=None, truth=None, stats=None, ari=None,
              labels=None, want_labels=False, ws=None, modularity=None, want_modularity=False, prf=None,
              want_prf=False):
    """Returns (stats int64[G][K][9], ari float64[G][K] or None, labels int32[K][n] or None),
    plus modularity float64[G][K] as a fourth item when want_modularity or modularity is given,
    plus precision/recall/F1 float64[G][K][3] as a fifth when want_prf or prf is given."""
    K = len(deltas)
    dev = g.ctx.device
    if vbase is None:
        vbase = torch.tensor([0, g.n], dtype=torch.int64, device=dev)
    G = vbase.numel() - 1
    arr = (mcd_rational * K)(*[mcd_rational(int(a), int(b)) for a, b in deltas])
    if stats is None:
        stats = _empty((G, K, len(SWEEP_FIELDS)), torch.int64, dev)
    if ari is None and truth is not None:
        ari = _empty((G, K), torch.float64, dev)
    if labels is None and want_labels:
        labels = _empty((K, max(g.n, 1)), torch.int32, dev)
    with_prf = want_prf or prf is not None
    with_q = want_modularity or modularity is not None or with_prf
    if modularity is None and want_modularity:
        modularity = _empty((G, K), torch.float64, dev)
    if prf is None and want_prf:
        prf = _empty((G, K, 3), torch.float64, dev)
    if ws is None:
        ws = _bytes(mcd_sweep_workspace_size(g, G, K, truth is not None), dev)
    _check(lib().mcd_sweep(g.handle, measure, _p(t), ctypes.cast(arr, ctypes.c_void_p), K, G, _p(vbase),
                           _p(truth), _p(stats), _p(ari), _p(modularity), _p(prf), _p(labels), _p(ws),
                           ws.numel() * ws.element_size()))
    if with_prf:
        return stats, ari, labels, modularity, prf
    return (stats, ari, labels, modularity) if with_q else (stats, ari, labels)


def mcd_sweep_rule(ctx: Context, deltas, stats, modularity=None, vbase=None, jump=(1, 10), index=None,
                   delta=None):
    """The rule-of-thumb threshold per graph from a sweep: (index int32[G], delta int64[G][2])."""
    K = len(deltas)
    G = stats.shape[0]
    dev = ctx.device
    if vbase is None:
        raise ValueError("vbase is required (the graphs' vertex ranges)")
    arr = (mcd_rational * K)(*[mcd_rational(int(a), int(b)) for a, b in deltas])
    index = _empty(G, torch.int32, dev) if index is None else index
    delta = _empty((G, 2), torch.int64, dev) if delta is None else delta
    _check(lib().mcd_sweep_rule(ctx.handle, ctypes.cast(arr, ctypes.c_void_p), K, G, _p(vbase), _p(stats),
                                _p(modularity), int(jump[0]), int(jump[1]), _p(index), _p(delta)))
    return index, delta


MLP_IN, MLP_HIDDEN, MLP_PARAMS = 66, 64, 8513


def _vbase(g: Graph, vbase):
    if vbase is None:
        return torch.tensor([0, g.n], dtype=torch.int64, device=g.ctx.device)
    return vbase


def mcd_features_workspace_size(n_graphs: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_features_workspace_size(n_graphs, ctypes.byref(b)))
    return b.value


def mcd_features(g: Graph, t, vbase=None, x=None, ws=None):
    vb = _vbase(g, vbase)
    G = vb.numel() - 1
    x = _empty((G, MLP_IN), torch.float32, g.ctx.device) if x is None else x
    if ws is None:
        ws = _bytes(mcd_features_workspace_size(G), g.ctx.device)
    _check(lib().mcd_features(g.handle, _p(t), G, _p(vb), _p(x), _p(ws), ws.numel() * ws.element_size()))
    return x


def mcd_feature_stats(ctx: Context, x, min_std: float = 1e-2, mean=None, std=None):
    mean = _empty(MLP_IN, torch.float32, ctx.device) if mean is None else mean
    std = _empty(MLP_IN, torch.float32, ctx.device) if std is None else std
    _check(lib().mcd_feature_stats(ctx.handle, _p(x), x.shape[0], min_std, _p(mean), _p(std)))
    return mean, std


def mcd_feature_range(ctx: Context, x, lo=None, hi=None):
    lo = _empty(MLP_IN, torch.float32, ctx.device) if lo is None else lo
    hi = _empty(MLP_IN, torch.float32, ctx.device) if hi is None else hi
    _check(lib().mcd_feature_range(ctx.handle, _p(x), x.shape[0], _p(lo), _p(hi)))
    return lo, hi


def mcd_picker_fallback(ctx: Context, x, lo, hi, margin: float, picked=None, fallback=None, delta=None,
                        flags=None, want_flags=True):
    """Out-of-range flags per graph and, given both threshold tables, the
    threshold each graph uses (fallback where flagged)."""
    B = x.shape[0]
    if flags is None and want_flags:
        flags = _empty(max(B, 1), torch.int32, ctx.device)
    if delta is None and picked is not None:
        delta = _empty((max(B, 1), 2), torch.int64, ctx.device)
    _check(lib().mcd_picker_fallback(ctx.handle, _p(x), B, _p(lo), _p(hi), margin, _p(picked), _p(fallback),
                                     _p(delta), _p(flags)))
    return (None if flags is None else flags[:B]), (None if delta is None else delta[:B])


def mcd_mlp_forward(ctx: Context, params, mean, std, x, y=None):
    B = x.shape[0]
    y = _empty(max(B, 1), torch.float32, ctx.device) if y is None else y
    _check(lib().mcd_mlp_forward(ctx.handle, _p(params), _p(mean), _p(std), _p(x), B, _p(y)))
    return y[:B]


def mcd_mlp_workspace_size(batch: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_mlp_workspace_size(batch, ctypes.byref(b)))
    return b.value


def mcd_mlp_gradient(ctx: Context, params, mean, std, x, target, grad=None, loss=None, ws=None, ari=None,
                     mse_weight: float = 1.0):
    """ari: optional device float64 [B][K] ARI table (the loss then subtracts
    the ARI interpolated at (K-1) y)."""
    B = x.shape[0]
    K = 0 if ari is None else ari.shape[1]
    grad = _empty(MLP_PARAMS, torch.float32, ctx.device) if grad is None else grad
    loss = _empty(1, torch.float32, ctx.device) if loss is None else loss
    ws = _bytes(mcd_mlp_workspace_size(B), ctx.device) if ws is None else ws
    _check(lib().mcd_mlp_gradient(ctx.handle, _p(params), _p(mean), _p(std), _p(x), _p(target), _p(ari), K,
                                  mse_weight, B, _p(grad), _p(loss), _p(ws), ws.numel() * ws.element_size()))
    return grad, loss


def mcd_mlp_train_step(ctx: Context, params, adam_m, adam_v, step: int, lr: float, mean, std, x, target,
                       loss=None, ws=None, weight_decay: float = 0.0, ari=None, mse_weight: float = 1.0):
    B = x.shape[0]
    K = 0 if ari is None else ari.shape[1]
    loss = _empty(1, torch.float32, ctx.device) if loss is None else loss
    ws = _bytes(mcd_mlp_workspace_size(B), ctx.device) if ws is None else ws
    _check(lib().mcd_mlp_train_step(ctx.handle, _p(params), _p(adam_m), _p(adam_v), step, lr, weight_decay,
                                    _p(mean), _p(std), _p(x), _p(target), _p(ari), K, mse_weight, B, _p(loss),
                                    _p(ws), ws.numel() * ws.element_size()))
    return loss


def mcd_grid_select(ctx: Context, y, K: int, a: int, b: int, c: int, index=None, delta=None):
    B = y.numel()
    index = _empty(max(B, 1), torch.int32, ctx.device) if index is None else index
    delta = _empty((max(B, 1), 2), torch.int64, ctx.device) if delta is None else delta
    _check(lib().mcd_grid_select(ctx.handle, _p(y), B, K, a, b, c, _p(index), _p(delta)))
    return index[:B], delta[:B]


def mcd_sweep_targets(ctx: Context, ari, frac: float = 0.95, index=None, y=None):
    G, K = ari.shape
    index = _empty(G, torch.int32, ctx.device) if index is None else index
    y = _empty(G, torch.float32, ctx.device) if y is None else y
    _check(lib().mcd_sweep_targets(ctx.handle, _p(ari), G, K, frac, _p(index), _p(y)))
    return index, y


def mcd_prune_graphs(g: Graph, measure: int, t, deltas, vbase=None, keep_bits=None, n_kept=None):
    vb = _vbase(g, vbase)
    words = max((g.m + 31) // 32, 1)
    keep_bits = _empty(words, torch.int32, g.ctx.device) if keep_bits is None else keep_bits
    n_kept = _empty(1, torch.int64, g.ctx.device) if n_kept is None else n_kept
    _check(lib().mcd_prune_graphs(g.handle, measure, _p(t), vb.numel() - 1, _p(vb), _p(deltas), _p(keep_bits),
                                  _p(n_kept)))
    return keep_bits, n_kept


# ------------------------------------------------------ picker as an object

PICKER_GRID_K, PICKER_GRID_A, PICKER_GRID_B, PICKER_GRID_C = 64, 9, 7, 900
PICKER_MARGIN = 0.25
MCD_PICK_AUTO, MCD_PICK_FORCE_SWEEP, MCD_PICK_NETWORK = 0, 1, 2


class PickerHandle:
    """An mcd_picker and the context it lives in."""

    def __init__(self, handle, ctx: Context):
        self.handle = handle
        self.ctx = ctx

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcd_picker_destroy(self.handle)
            self.handle = None


def mcd_picker_create(ctx: Context, seed: int = 0) -> PickerHandle:
    h = ctypes.c_void_p()
    _check(lib().mcd_picker_create(ctx.handle, int(seed), ctypes.byref(h)))
    return PickerHandle(h, ctx)


def mcd_picker_prepare(p: PickerHandle, x, min_std: float = 1.0, margin: float = PICKER_MARGIN) -> None:
    _check(lib().mcd_picker_prepare(p.handle, _p(x), x.shape[0], min_std, margin))


def mcd_picker_train_step(p: PickerHandle, x, y, lr: float, weight_decay: float = 0.0, loss=None, ws=None,
                          ari=None, mse_weight: float = 1.0):
    B = x.shape[0]
    loss = _empty(1, torch.float32, p.ctx.device) if loss is None else loss
    ws = _bytes(mcd_mlp_workspace_size(B), p.ctx.device) if ws is None else ws
    _check(lib().mcd_picker_train_step(p.handle, _p(x), _p(y), _p(ari), mse_weight, B, lr, weight_decay, _p(loss),
                                       _p(ws), ws.numel() * ws.element_size()))
    return loss


def mcd_picker_fit(p: PickerHandle, x, y, steps: int, lr: float, weight_decay: float = 0.0, min_std: float = 1.0,
                   margin: float = PICKER_MARGIN, losses=None, ws=None, ari=None, mse_weight: float = 1.0):
    """ari: optional device float64 [B][64] ARI table over the picker's grid."""
    B = x.shape[0]
    losses = _empty(max(steps, 1), torch.float32, p.ctx.device) if losses is None else losses
    ws = _bytes(mcd_mlp_workspace_size(B), p.ctx.device) if ws is None else ws
    _check(lib().mcd_picker_fit(p.handle, _p(x), _p(y), _p(ari), mse_weight, B, steps, lr, weight_decay, min_std,
                                margin, _p(losses), _p(ws), ws.numel() * ws.element_size()))
    return losses[:steps]


def mcd_picker_forward(p: PickerHandle, x, y=None):
    B = x.shape[0]
    y = _empty(max(B, 1), torch.float32, p.ctx.device) if y is None else y
    _check(lib().mcd_picker_forward(p.handle, _p(x), B, _p(y)))
    return y[:B]


def mcd_picker_pick_workspace_size(g: Graph, n_graphs: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_picker_pick_workspace_size(g.handle, n_graphs, ctypes.byref(b)))
    return b.value


def mcd_picker_pick(p: PickerHandle, g: Graph, measure: int, t, vbase=None, mode: int = MCD_PICK_AUTO, index=None,
                    deltas=None, used_fallback=None, labels=None, n_components=None, ws=None):
    """Returns (index int32[G], deltas int64[G][2], used_fallback int32[G],
    labels int32[n], n_components int64[1])."""
    vb = _vbase(g, vbase)
    G = vb.numel() - 1
    dev = g.ctx.device
    index = _empty(G, torch.int32, dev) if index is None else index
    deltas = _empty((G, 2), torch.int64, dev) if deltas is None else deltas
    used_fallback = _empty(G, torch.int32, dev) if used_fallback is None else used_fallback
    labels = _empty(max(g.n, 1), torch.int32, dev) if labels is None else labels
    n_components = _empty(1, torch.int64, dev) if n_components is None else n_components
    ws = _bytes(mcd_picker_pick_workspace_size(g, G), dev) if ws is None else ws
    _check(lib().mcd_picker_pick(p.handle, g.handle, measure, _p(t), G, _p(vb), mode, _p(index), _p(deltas),
                                 _p(used_fallback), _p(labels), _p(n_components), _p(ws),
                                 ws.numel() * ws.element_size()))
    return index, deltas, used_fallback, labels[:g.n], n_components


def mcd_picker_export(p: PickerHandle) -> dict:
    dev = p.ctx.device
    out = dict(params=_empty(MLP_PARAMS, torch.float32, dev), mean=_empty(MLP_IN, torch.float32, dev),
               std=_empty(MLP_IN, torch.float32, dev), lo=_empty(MLP_IN, torch.float32, dev),
               hi=_empty(MLP_IN, torch.float32, dev))
    margin = ctypes.c_float()
    _check(lib().mcd_picker_export(p.handle, _p(out["params"]), _p(out["mean"]), _p(out["std"]), _p(out["lo"]),
                                   _p(out["hi"]), ctypes.byref(margin)))
    out["margin"] = margin.value
    return out


def mcd_picker_import(p: PickerHandle, params, mean, std, lo, hi, margin: float = PICKER_MARGIN) -> None:
    _check(lib().mcd_picker_import(p.handle, _p(params), _p(mean), _p(std), _p(lo), _p(hi), margin))


def mcd_picker_save(p: PickerHandle, path: str) -> None:
    _check(lib().mcd_picker_save(p.handle, os.fsencode(path)))


def mcd_picker_load(p: PickerHandle, path: str) -> None:
    _check(lib().mcd_picker_load(p.handle, os.fsencode(path)))


def mcd_picker_check_file(path: str) -> None:
    _check(lib().mcd_picker_check_file(os.fsencode(path)))


KEPT_SEGMENTS = 16384
NOALLOC_MAX_VERTICES = 1 << 24
TUNE_PARAMS = ("tc_chunk", "tc_lds_max", "tc_packed_range", "tc_window_max")
# the launch parameters an autotune cache entry holds
CACHED_PARAMS = TUNE_PARAMS + ("tc_window_occupancy", "sweep_shape")


def mcd_tune_triangles_workspace_size(g: Graph) -> int:
    b = ctypes.c_size_t()
    _check(lib().mcd_tune_triangles_workspace_size(g.handle, ctypes.byref(b)))
    return b.value


def mcd_tune_triangles(g: Graph, t=None, ws=None, reps: int = 2):
    """Autotune the triangle-count parameters on g; returns ({name: value}, ms)."""
    t = _empty(max(g.m, 1), torch.int32, g.ctx.device) if t is None else t
    if ws is None:
        b = ctypes.c_size_t()
        _check(lib().mcd_tune_triangles_workspace_size(g.handle, ctypes.byref(b)))
        ws = _bytes(b.value, g.ctx.device)
    best = (ctypes.c_int64 * 4)()
    ms = ctypes.c_float()
    _check(lib().mcd_tune_triangles(g.handle, _p(t), _p(ws), ws.numel() * ws.element_size(), reps, best,
                                    ctypes.byref(ms)))
    return dict(zip(TUNE_PARAMS, list(best))), ms.value


def mcd_tune_cache_load(g: Graph, path: str) -> bool:
    """Sets g's context from the autotune cache at path; True on a hit."""
    hit = ctypes.c_int32()
    _check(lib().mcd_tune_cache_load(g.ctx.handle, g.handle, os.fsencode(path), ctypes.byref(hit)))
    return bool(hit.value)


def mcd_tune_cache_store(g: Graph, path: str, ms: float) -> None:
    """Records g's context's current launch parameters in the cache at path."""
    _check(lib().mcd_tune_cache_store(g.ctx.handle, g.handle, os.fsencode(path), float(ms)))


def mcd_tune_cache_check_file(path: str) -> None:
    _check(lib().mcd_tune_cache_check_file(os.fsencode(path)))


def tune_sweep_shape(ctx: Context, run, reps: int = 1):
    """Times `run` (a call of mcd_sweep on the context's stream) under each
    launch shape of the sweep's level loop and keeps the fastest; returns
    ({shape: ms}, best shape)."""
    times = {}
    for shape in (0, 1, 2):
        mcd_ctx_set_param(ctx, "sweep_shape", shape)
        run()  # warm-up
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        times[shape] = best
    shape = min(times, key=times.get)
    mcd_ctx_set_param(ctx, "sweep_shape", shape)
    return times, shape


def mcd_kept_segment_len(g: Graph) -> int:
    v = ctypes.c_int64()
    _check(lib().mcd_kept_segment_len(g.handle, ctypes.byref(v)))
    return v.value


class KeptList:
    """Segmented kept-edge list written by mcd_weigh_prune (pairs of internal
    vertex numbers, int32[2 m], and per-segment counts)."""

    def __init__(self, g: Graph, pairs=None, counts=None):
        dev = g.ctx.device
        self.seg_len = mcd_kept_segment_len(g)
        need = 2 * KEPT_SEGMENTS * self.seg_len
        if pairs is None:
            pairs = _empty(max(need, 2), torch.int32, dev)
        elif pairs.numel() < need:
            raise ValueError(f"kept_pairs holds {pairs.numel()} int32, needs {need}")
        self.pairs = pairs
        self.counts = _empty(KEPT_SEGMENTS, torch.int32, dev) if counts is None else counts

    @staticmethod
    def capacity(m: int) -> int:
        """int32 elements of kept_pairs for a graph of m edges."""
        L = 64 * ((((m + 63) // 64) + KEPT_SEGMENTS - 1) // KEPT_SEGMENTS)
        return 2 * KEPT_SEGMENTS * L

    def edges(self):
        """The kept pairs, segment by segment, as an int32 [k, 2] tensor."""
        cnt = self.counts.cpu().tolist()
        p = self.pairs.view(-1, 2)
        parts = [p[s * self.seg_len: s * self.seg_len + c] for s, c in enumerate(cnt) if c]
        return torch.cat(parts) if parts else p[:0]

    def edge_ids(self, m: int):
        """Library edge ids in the order the list visits them (runs of
        seg_len edges, one per segment, in edge order): 0 .. m-1."""
        import numpy as np
        return np.arange(m, dtype=np.int64)


def mcd_weigh_prune(g: Graph, measure: int, t, delta=None, deltas=None, vbase=None, w_f32=None, w_i32=None,
                    keep_bits=None, kept=None, n_kept=None, want_f32=True, want_i32=False, want_keep=True,
                    want_kept=True):
    """One pass of weights and prune.  delta: a host (num, den), or deltas: a
    device int64 [G, 2] tensor of per-graph thresholds with vbase."""
    dev = g.ctx.device
    if w_f32 is None and want_f32:
        w_f32 = _empty(max(g.m, 1), torch.float32, dev)
    if w_i32 is None and want_i32:
        w_i32 = _empty(max(g.m, 1), torch.int32, dev)
    if keep_bits is None and want_keep:
        keep_bits = _empty(max((g.m + 31) // 32, 1), torch.int32, dev)
    if kept is None and want_kept:
        kept = KeptList(g)
    n_kept = _empty(1, torch.int64, dev) if n_kept is None else n_kept
    if deltas is not None:
        vb = _vbase(g, vbase)
        G, vbp, rat = vb.numel() - 1, _p(vb), mcd_rational(0, 1)
    else:
        G, vbp, rat = 1, None, _rat(delta)
    _check(lib().mcd_weigh_prune(g.handle, measure, _p(t), rat, G, vbp, _p(deltas), _p(w_f32), _p(w_i32),
                                 _p(keep_bits), None if kept is None else _p(kept.pairs),
                                 None if kept is None else _p(kept.counts), _p(n_kept)))
    return dict(w_f32=None if w_f32 is None else w_f32[:g.m], w_i32=None if w_i32 is None else w_i32[:g.m],
                keep_bits=keep_bits, kept=kept, n_kept=n_kept)


def mcd_prune_components(g: Graph, measure: int, t, delta=None, deltas=None, vbase=None, w_f32=None, w_i32=None,
                         keep_bits=None, n_kept=None, labels=None, n_components=None, ws=None, want_f32=True,
                         want_i32=False, want_keep=True):
    """Weights, prune and components in one pass (no kept list).  delta / deltas
    as mcd_weigh_prune; returns a dict of the outputs."""
    dev = g.ctx.device
    if w_f32 is None and want_f32:
        w_f32 = _empty(max(g.m, 1), torch.float32, dev)
    if w_i32 is None and want_i32:
        w_i32 = _empty(max(g.m, 1), torch.int32, dev)
    if keep_bits is None and want_keep:
        keep_bits = _empty(max((g.m + 31) // 32, 1), torch.int32, dev)
    n_kept = _empty(1, torch.int64, dev) if n_kept is None else n_kept
    labels = _empty(max(g.n, 1), torch.int32, dev) if labels is None else labels
    n_components = _empty(1, torch.int64, dev) if n_components is None else n_components
    if ws is None:
        ws = _bytes(mcd_components_workspace_size(g), dev)
    if deltas is not None:
        vb = _vbase(g, vbase)
        G, vbp, rat = vb.numel() - 1, _p(vb), mcd_rational(0, 1)
    else:
        G, vbp, rat = 1, None, _rat(delta)
    _check(lib().mcd_prune_components(g.handle, measure, _p(t), rat, G, vbp, _p(deltas), _p(w_f32), _p(w_i32),
                                      _p(keep_bits), _p(n_kept), _p(labels), _p(n_components), _p(ws),
                                      ws.numel() * ws.element_size()))
    return dict(w_f32=None if w_f32 is None else w_f32[:g.m], w_i32=None if w_i32 is None else w_i32[:g.m],
                keep_bits=keep_bits, n_kept=n_kept, labels=labels[:g.n], n_components=n_components)


def mcd_prune_components_noalloc(g: Graph, measure: int, t, delta=None, deltas=None, vbase=None, w_f32=None,
                                 w_i32=None, keep_bits=None, n_kept=None, labels=None, n_components=None,
                                 want_f32=True, want_i32=False, want_keep=True):
    """mcd_prune_components with the library's own device scratch instead of a
    workspace (graphs of at most NOALLOC_MAX_VERTICES vertices).  Outputs the
    caller does not pass are allocated here, by torch, before the call."""
    dev = g.ctx.device
    if w_f32 is None and want_f32:
        w_f32 = _empty(max(g.m, 1), torch.float32, dev)
    if w_i32 is None and want_i32:
        w_i32 = _empty(max(g.m, 1), torch.int32, dev)
    if keep_bits is None and want_keep:
        keep_bits = _empty(max((g.m + 31) // 32, 1), torch.int32, dev)
    n_kept = _empty(1, torch.int64, dev) if n_kept is None else n_kept
    labels = _empty(max(g.n, 1), torch.int32, dev) if labels is None else labels
    n_components = _empty(1, torch.int64, dev) if n_components is None else n_components
    if deltas is not None:
        vb = _vbase(g, vbase)
        G, vbp, rat = vb.numel() - 1, _p(vb), mcd_rational(0, 1)
    else:
        G, vbp, rat = 1, None, _rat(delta)
    _check(lib().mcd_prune_components_noalloc(g.handle, measure, _p(t), rat, G, vbp, _p(deltas), _p(w_f32),
                                              _p(w_i32), _p(keep_bits), _p(n_kept), _p(labels), _p(n_components)))
    return dict(w_f32=None if w_f32 is None else w_f32[:g.m], w_i32=None if w_i32 is None else w_i32[:g.m],
                keep_bits=keep_bits, n_kept=n_kept, labels=labels[:g.n], n_components=n_components)


def mcd_components_kept(g: Graph, kept: KeptList, labels=None, n_components=None, ws=None):
    labels = _empty(max(g.n, 1), torch.int32, g.ctx.device) if labels is None else labels
    n_components = _empty(1, torch.int64, g.ctx.device) if n_components is None else n_components
    if ws is None:
        ws = _bytes(mcd_components_workspace_size(g), g.ctx.device)
    _check(lib().mcd_components_kept(g.handle, _p(kept.pairs), _p(kept.counts), _p(labels), _p(n_components),
                                     _p(ws), ws.numel() * ws.element_size()))
    return labels[:g.n], n_components


def mcd_status_string(status: int) -> str:
    return lib().mcd_status_string(status).decode()


def mcd_last_error() -> str:
    return lib().mcd_last_error().decode()

