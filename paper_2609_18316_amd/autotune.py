"""Autotuner for the tree and traversal parameters.

The paper tunes the leaf size by hand (Sec. 2.1 and App. A: 10-20 is best on
its CPUs, 16 by default, and the optimum moves with N and D).  Here the choice
is measured on the GPU for a given workload shape:

* leaf size (N_leaf) -- trades build time against leaf scanning in queries;
* queries per wave -- 1 (one independent traversal per lane) or 64 (one
  traversal shared by a wave of spatially coherent queries);
* traversal stack depth -- not tuned: with median splits it is exactly the
  tree depth L = ceil(log2(ceil(n / N_leaf))), known from n.

`tune()` times build + query for every candidate, returns the fastest and
installs it in the running library (kdt_tuning_set), so that leaf_size = 0
and traversal = 0 pick it for the rest of the process; `lookup()` reads
results stored by earlier tuning runs (a JSON table next to this file, keyed
by workload shape), falling back to the paper's regime.  `write_inc()` turns
that table into csrc/kdt_tuning.inc, the table compiled into the library:
run this module on a GPU (``python -m paper_2609_18316_amd.autotune``) to
measure the standard shapes, store them and regenerate it; the library picks
the new table up at its next build.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict, dataclass

import torch

from . import kdt

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_table.json")
INC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "kdt_tuning.inc")
# Query kinds in the order the compiled-in table prefers them when several
# kinds were measured for one (d, log2 n, k): the library cannot tell them apart.
KIND_ORDER = ("uniform-queries", "self", "self-uniform", "batch-clustered", "self-normal")
LEAF_CANDIDATES = (8, 12, 16, 24, 32, 48, 64)


@dataclass
class Choice:
    leaf_size: int
    queries_per_wave: int  # 1 or 64
    stack_depth: int
    build_ms: float
    query_ms: float


def key(n: int, d: int, k: int, kind: str) -> str:
    """Table key: log2 of n rounded, dimension, k and the query kind."""
    return f"n2^{int(round(math.log2(max(n, 1))))}-d{d}-k{k}-{kind}"


def _time(fn, reps: int) -> float:
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    fn()
    e.record()
    torch.cuda.synchronize()
    best = s.elapsed_time(e)
    if best > 200.0:  # slow candidates (high d): the first run is representative enough
        reps = 1
    for _ in range(reps):
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        best = min(best, s.elapsed_time(e))
    return best


def tune(points: torch.Tensor, k: int, queries: torch.Tensor | None = None,
         leaf_sizes=LEAF_CANDIDATES, reps: int = 3, query_weight: float = 1.0,
         verbose: bool = False) -> Choice:
    """Measures build + kNN (k) for each candidate; minimises build + weight * query."""
    n, d = points.shape
    best: Choice | None = None
    for leaf in leaf_sizes:
        build_ms = _time(lambda: kdt.build(points, leaf_size=leaf, check_finite=False), reps)
        tree = kdt.build(points, leaf_size=leaf, check_finite=False)
        order = tree.query_order(queries) if queries is not None else None
        for trav in ((1, 2) if leaf <= 64 else (1,)):
            q_ms = _time(lambda: tree.knn(queries, k, order=order, traversal=trav), reps)
            c = Choice(leaf, 64 if trav == 2 else 1, tree.info.levels + 1, build_ms, q_ms)
            if verbose:
                print(f"  leaf {leaf} traversal {trav}: build {build_ms:.3f} ms, "
                      f"query {q_ms:.3f} ms", flush=True)
            score = build_ms + query_weight * q_ms
            if best is None or score < best.build_ms + query_weight * best.query_ms:
                best = c
        tree.close()
    assert best is not None
    kdt.tuning_set(d, n, k, best.leaf_size, best.queries_per_wave)
    return best


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def store(entries: dict, path: str = TABLE) -> None:
    table = load_table(path)
    table.update({k: asdict(v) if isinstance(v, Choice) else v for k, v in entries.items()})
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def lookup(n: int, d: int, k: int, kind: str, path: str = TABLE) -> Choice:
    """Stored choice for the workload shape, else the default (leaf 32, wave packets)."""
    entry = load_table(path).get(key(n, d, k, kind))
    if entry:
        return Choice(**entry)
    leaf = 32
    levels = 0
    while -(-n // (1 << levels)) > leaf:
        levels += 1
    return Choice(leaf, 64, levels + 1, float("nan"), float("nan"))


def _parse_key(name: str):
    """(d, log2 n, k, kind) of a table key."""
    n_part, d_part, k_part, kind = name.split("-", 3)
    return int(d_part[1:]), int(n_part[3:]), int(k_part[1:]), kind


def write_inc(table: dict | None = None, path: str = INC) -> None:
    """Writes the compiled-in tuning table: one initializer {d, log2 n, k,
    leaf, queries per wave} per shape, the preferred kind first."""
    table = load_table() if table is None else table
    rows = []
    for name, e in table.items():
        d, l2, k, kind = _parse_key(name)
        rank = KIND_ORDER.index(kind) if kind in KIND_ORDER else len(KIND_ORDER)
        rows.append((d, l2, k, rank, name, e["leaf_size"], e["queries_per_wave"]))
    rows.sort()
    lines = ["// Generated by paper_2609_18316_amd/autotune.py (write_inc) from",
             "// autotune_table.json: {d, log2 n, k, leaf size, queries per traversal}."]
    for d, l2, k, _, name, leaf, qpw in rows:
        lines.append(f"{{{d}, {l2}, {k}, {leaf}, {qpw}}},  // {name}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _standard_workloads():
    """The workload shapes the benchmark and the parity configurations use."""
    from . import workloads
    dev = torch.device("cuda:0")
    gen = torch.Generator().manual_seed(0)
    x = torch.from_numpy(workloads.clustered(1 << 24, seed=2)).to(dev)
    q = torch.from_numpy(workloads.uniform(1 << 22, 3, seed=102)).to(dev)
    yield key(1 << 24, 3, 32, "uniform-queries"), x, q, 32
    sel = torch.randperm(x.shape[0], generator=gen)[: 1 << 20].to(dev)
    yield key(1 << 24, 3, 32, "self"), x, x[sel].contiguous(), 32
    for d in (2, 4, 8, 16):
        for dist in ("uniform", "normal"):
            pts = workloads.uniform(1 << 22, d, 300 + d) if dist == "uniform" else \
                workloads.normal(1 << 22, d, 400 + d)
            xt = torch.from_numpy(pts).to(dev)
            sel = torch.randperm(xt.shape[0], generator=gen)[: 1 << 16].to(dev)
            yield key(1 << 22, d, 16, f"self-{dist}"), xt, xt[sel].contiguous(), 16
    # set sizes of the batched mode (clustered sets, k = 8, every point a query)
    for e in (10, 12, 14, 16, 18, 20):
        xs = torch.from_numpy(workloads.clustered(1 << e, seed=500 + e)).to(dev)
        yield key(1 << e, 3, 8, "batch-clustered"), xs, None, 8


def main(argv=None) -> None:
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="", help="substring of the shapes to measure")
    ap.add_argument("--out-dir", default="",
                    help="write autotune_table.json and kdt_tuning.inc there instead of in place")
    args = ap.parse_args(argv)
    results = {}
    for name, pts, qs, kk in _standard_workloads():
        if args.only and args.only not in name:
            continue
        print(name, flush=True)
        c = tune(pts, kk, qs, verbose=True)
        results[name] = c
        print(name, asdict(c), flush=True)
    table_path = os.path.join(args.out_dir, "autotune_table.json") if args.out_dir else TABLE
    if args.out_dir:
        os.makedirs(args.out_dir, exist_ok=True)
        with open(table_path, "w") as f:
            json.dump(load_table(), f, indent=1, sort_keys=True)
    store(results, table_path)
    write_inc(load_table(table_path),
              os.path.join(args.out_dir, "kdt_tuning.inc") if args.out_dir else INC)


if __name__ == "__main__":
    main()
