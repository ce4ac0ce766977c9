#!/usr/bin/env python3
"""Writes rmat_s26_seed3_digests.json: the CPU oracle's results on R-MAT
scale 26 (edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), seed 3), reduced to
counts and SHA-256 digests so the GPU test can compare every edge and every
vertex without the oracle's hour of CPU work.

Calls only oracle/ (and graphgen/ for the input pairs).  Run from the
repository root:  python tests/golden/make_rmat_s26_digests.py
It needs about 50 GB of host memory and, on 8 cores, about half an hour.

Array layouts that the digests cover (little-endian, in chunks of 2^25
elements; the keep mask as bits, 2^25 edges per chunk):
  lo, hi   int32[m]  canonical edges, sorted by (lo, hi), lo < hi
  deg      int32[n]  degree by original vertex id
  t        int32[m]  t(e) = |N(lo) n N(hi)| in canonical edge order
  keep     bit[m]    NOT (sim(e) < delta) in canonical order, packed
                     least-significant bit first (numpy bitorder='little')
  labels   int32[n]  smallest vertex id of each vertex's component
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat_s26_seed3_digests.json")
CHUNK = 1 << 25

# thresholds whose keep masks and labels are digested: Tectonic at the
# rule-of-thumb value 1/50, the picker grid's 9/900 and 0 (every edge kept);
# TW at -10, a point of the paper's TW grid (Table tab:params)
DIGESTED = [("tectonic", oracle.TECTONIC, 1, 50), ("tectonic", oracle.TECTONIC, 9, 900),
            ("tectonic", oracle.TECTONIC, 0, 50), ("tw", oracle.TW, -10, 1)]


def chunk_sha(a: np.ndarray, chunk: int = CHUNK):
    a = np.ascontiguousarray(a)
    return [hashlib.sha256(memoryview(a[i:i + chunk]).cast("B")).hexdigest() for i in range(0, len(a), chunk)]


def bits_sha(keep: np.ndarray):
    packed = np.packbits(keep.astype(np.uint8), bitorder="little")
    return [hashlib.sha256(memoryview(packed[i:i + CHUNK // 8])).hexdigest()
            for i in range(0, len(packed), CHUNK // 8)]


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def host_facts():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), omp_threads=oracle.num_threads(),
                machine=platform.machine())


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, default=26, help="a smaller scale writes to --out (a dry run)")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    out, scale = args.out, args.scale
    rec = dict(workload=f"R-MAT scale {scale}, edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), seed 3, "
                        "symmetrised, deduplicated, self-loops removed",
               scale=scale, edge_factor=16, seed=3, chunk=CHUNK, host=host_facts(), seconds={})

    def save():
        rec["peak_rss_gib"] = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 2**20
        with open(out + ".tmp", "w") as f:
            json.dump(rec, f, indent=1)
        os.replace(out + ".tmp", out)

    t0 = time.perf_counter()
    src, dst, n = gg.rmat(scale, 16, seed=3)
    rec.update(n=int(n), pairs=int(len(src)))
    rec["seconds"]["generate"] = time.perf_counter() - t0
    log(f"generated {len(src)} pairs")

    t0 = time.perf_counter()
    lo, hi = oracle.canon(n, src, dst)
    del src, dst
    m = len(lo)
    rec["seconds"]["canon"] = time.perf_counter() - t0
    rec["m"] = int(m)
    rec["lo_sha256"], rec["hi_sha256"] = chunk_sha(lo.astype("<i4")), chunk_sha(hi.astype("<i4"))
    deg = oracle.degrees(n, lo, hi)
    rec["deg_sha256"] = chunk_sha(deg.astype("<i4"))
    rec["max_degree"] = int(deg.max())
    log(f"canonical graph: m={m}, max degree {rec['max_degree']} ({rec['seconds']['canon']:.0f} s)")
    save()

    t0 = time.perf_counter()
    t = oracle.triangles(n, lo, hi)
    rec["seconds"]["triangles"] = time.perf_counter() - t0
    rec["t_sum"] = int(t.sum(dtype=np.int64))
    rec["triangles"] = rec["t_sum"] // 3
    rec["t_max"] = int(t.max())
    rec["t_sha256"] = chunk_sha(t.astype("<i4"))
    log(f"triangles: {rec['triangles']} ({rec['seconds']['triangles']:.0f} s)")
    save()

    rec["digested"] = []
    for name, meas, num, den in DIGESTED:
        t0 = time.perf_counter()
        keep = oracle.prune(meas, lo, hi, t, deg, num, den)
        lab, ncc = oracle.components(n, lo, hi, keep)
        sizes = np.bincount(lab, minlength=1)
        r = dict(measure=name, delta=[num, den], n_kept=int(keep.sum(dtype=np.int64)), n_components=int(ncc),
                 largest_component=int(sizes.max()), keep_sha256=bits_sha(keep),
                 labels_sha256=chunk_sha(lab.astype("<i4")), seconds=time.perf_counter() - t0)
        del keep, lab, sizes
        rec["digested"].append(r)
        log(f"{name} {num}/{den}: kept {r['n_kept']}, components {r['n_components']}, "
            f"largest {r['largest_component']} ({r['seconds']:.0f} s)")
        save()

    # the 16-point check sweep k/50 (Tectonic): kept edges, components and the
    # largest component per threshold
    sweep = []
    for k in range(16):
        t0 = time.perf_counter()
        keep = oracle.prune(oracle.TECTONIC, lo, hi, t, deg, k, 50)
        lab, ncc = oracle.components(n, lo, hi, keep)
        sweep.append(dict(delta=[k, 50], n_kept=int(keep.sum(dtype=np.int64)), n_components=int(ncc),
                          largest_component=int(np.bincount(lab).max())))
        del keep, lab
        log(f"sweep {k}/50: {sweep[-1]} ({time.perf_counter() - t0:.0f} s)")
        rec["sweep16"] = sweep
        save()
    log(f"done; peak RSS {rec['peak_rss_gib']:.1f} GiB -> {out}")


if __name__ == "__main__":
    main()
