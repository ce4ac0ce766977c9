"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
bring its outputs into the oracle's canonical edge order (sorted (lo, hi))."""
import numpy as np
import torch

import paper_2412_12382_amd.mcd as M

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = M.mcd_ctx_create(0)
    return _CTX


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda:0")


def unpack_bits(keep_bits, m):
    w = keep_bits.detach().cpu().numpy().view(np.uint32)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return bits[:m].astype(np.uint8)


def build(src, dst, n):
    return M.mcd_graph_build(ctx(), to_dev(src), to_dev(dst), n)


def canonical_order(g):
    """(lo, hi, order): canonical endpoints and the permutation that sorts
    library edge order into (lo, hi) order."""
    u, v = M.mcd_graph_edges(g)
    u = u.cpu().numpy().astype(np.int64)
    v = v.cpu().numpy().astype(np.int64)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    order = np.argsort(lo * (g.n + 1) + hi, kind="stable")
    return lo[order].astype(np.int32), hi[order].astype(np.int32), order


def gpu_all(src, dst, n, measure, delta):
    """Every product of the pipeline on the GPU, canonical edge order."""
    g = build(src, dst, n)
    lo, hi, order = canonical_order(g)
    deg = M.mcd_graph_degrees(g).cpu().numpy()
    t = M.mcd_triangles(g)
    ints = measure in (M.MCD_SIM_TW, M.MCD_SIM_K3)
    wf, wi = M.mcd_weights(g, measure, t, want_f32=True, want_i32=ints)
    keep, nk = M.mcd_prune(g, measure, t, delta)
    labels, ncc = M.mcd_components(g, keep)
    labels_run, ncc_run = M.mcd_run(g, measure, delta)
    fused = M.mcd_weigh_prune(g, measure, t, delta=delta, want_i32=ints)
    labels_k, ncc_k = M.mcd_components_kept(g, fused["kept"])
    pc = M.mcd_prune_components(g, measure, t, delta=delta, want_i32=ints)
    torch.cuda.synchronize()
    out = dict(g=g, lo=lo, hi=hi, deg=deg[:n], t=t.cpu().numpy()[order],
               w=wf.cpu().numpy()[order] if g.m else np.zeros(0, np.float32),
               keep=unpack_bits(keep, g.m)[order], n_kept=int(nk.item()),
               labels=labels.cpu().numpy(), ncc=int(ncc.item()),
               labels_run=labels_run.cpu().numpy(), ncc_run=int(ncc_run.item()))
    if wi is not None:
        out["tw"] = wi.cpu().numpy()[order]
    # fused pass: the kept list, mapped to original ids, must be the kept
    # edges in the list's documented order (segment s: groups s, s + S, ...)
    u, v = M.mcd_graph_edges(g)
    u, v = u.cpu().numpy(), v.cpu().numpy()
    keep_lib = unpack_bits(fused["keep_bits"], g.m).astype(bool)
    perm = M.mcd_graph_perm(g).cpu().numpy()
    kp = fused["kept"].edges().cpu().numpy().astype(np.int64)
    out["fused"] = dict(
        w=fused["w_f32"].cpu().numpy()[order] if g.m else np.zeros(0, np.float32),
        tw=None if fused["w_i32"] is None else fused["w_i32"].cpu().numpy()[order],
        keep=keep_lib.astype(np.uint8)[order], n_kept=int(fused["n_kept"].item()),
        kept_u=perm[kp[:, 0]] if len(kp) else np.zeros(0, np.int32),
        kept_v=perm[kp[:, 1]] if len(kp) else np.zeros(0, np.int32),
        want_u=u[fused["kept"].edge_ids(g.m)][keep_lib[fused["kept"].edge_ids(g.m)]],
        want_v=v[fused["kept"].edge_ids(g.m)][keep_lib[fused["kept"].edge_ids(g.m)]],
        labels=labels_k.cpu().numpy(), ncc=int(ncc_k.item()))
    # weights + prune + components in one pass
    out["pc"] = dict(
        w=pc["w_f32"].cpu().numpy()[order] if g.m else np.zeros(0, np.float32),
        tw=None if pc["w_i32"] is None else pc["w_i32"].cpu().numpy()[order],
        keep=unpack_bits(pc["keep_bits"], g.m)[order], n_kept=int(pc["n_kept"].item()),
        labels=pc["labels"].cpu().numpy(), ncc=int(pc["n_components"].item()))
    return out
