"""Traversal work of the benchmarked launches, from the instrumented library.

``python -m paper_2609_18316_amd.workcount`` loads ``libkdt_counts.so`` (the
same kernels, compiled to count the node boxes and point records their
traversals read), replays the launches bench.py times, and prints one JSON
line with the counts.  They give the traversal term of the algorithmic bytes
of each launch: leaf points scanned x record bytes + node boxes read x box
bytes (records and boxes are 16 and 32 bytes at d = 3).  Run it in a process
of its own: the product library and the instrumented one cannot share one.

Launches (the bench's configurations):
  knn_c2     kNN k = 32 of 2^22 uniform queries (Hilbert order, one query
             per lane) on the 2^24-point clustered tree, tuned leaf size;
  range_c2   closed-ball counts r = 0.01 of the same queries (wave-shared);
  knn_d8 / knn_d16   kNN k = 16 of every point of 2^22 uniform points in
             d = 8 and 16, leaf size and traversal from the tuning table.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--no-dims", action="store_true", help="skip the d = 8, 16 launches")
    args = ap.parse_args()
    import torch

    from paper_2609_18316_amd import autotune, kdt, workloads

    if not torch.cuda.is_available():
        print("workcount needs a GPU", file=sys.stderr)
        sys.exit(2)
    kdt.load(kdt.LIB_COUNTS_PATH)
    dev = torch.device("cuda:0")
    out = {}

    def rec_box(d):
        return 4 * ((d + 1 + 3) // 4 * 4), 2 * 4 * ((d + 3) // 4 * 4)

    x = torch.from_numpy(workloads.clustered(1 << 24, seed=2)).to(dev)
    q = torch.from_numpy(workloads.uniform(1 << 22, 3, seed=102)).to(dev)
    tree = kdt.build(x, leaf_size=0, tune_k=32)  # the tuned leaf size, as the bench
    order = tree.query_order(q)
    kdt.visits(reset=True)
    tree.knn(q, 32, order=order)
    c = kdt.visits(reset=True)
    rb, bb = rec_box(3)
    out["knn_c2"] = dict(c, queries=1 << 22, d=3, k=32, record_bytes=rb, box_bytes=bb)
    print(f"[workcount] knn_c2 {c}", file=sys.stderr, flush=True)
    tree.range(q, 0.01)
    c = kdt.visits(reset=True)
    out["range_c2"] = dict(c, queries=1 << 22, d=3, r=0.01, record_bytes=rb, box_bytes=bb)
    print(f"[workcount] range_c2 {c}", file=sys.stderr, flush=True)
    tree.close()
    del x, q
    if not args.no_dims:
        n = 1 << 22
        for d in (8, 16):
            pts = torch.from_numpy(workloads.uniform(n, d, 300 + d)).to(dev)
            cfg = autotune.lookup(n, d, 16, "self-uniform")
            trav = 2 if cfg.queries_per_wave == 64 else 1
            t = kdt.build(pts, leaf_size=cfg.leaf_size)
            kdt.visits(reset=True)
            t.knn(None, 16, traversal=trav)
            c = kdt.visits(reset=True)
            rb, bb = rec_box(d)
            out[f"knn_d{d}"] = dict(c, queries=n, d=d, k=16, leaf_size=cfg.leaf_size,
                                    traversal="lane" if trav == 1 else "wave",
                                    record_bytes=rb, box_bytes=bb)
            print(f"[workcount] knn_d{d} {c}", file=sys.stderr, flush=True)
            t.close()
            del pts
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
