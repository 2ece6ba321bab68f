"""Benchmark of the k-d tree hot path on one MI355X.

One step runs every stage of the path on the clustered workload: a tree over
2^24 clustered 3-D points (2000 Gaussian halos + 20 % uniform background),
kNN (k = 32) of 2^22 uniform query points, closed-ball counts (r = 0.01) of the
same queries, friends-of-friends of the 2^24 points (b = 0.2), SPH smoothing
lengths (distance to the 32nd neighbour of every point), the particle-to-mesh
deposit onto a 256^3 mesh and its adjoint, and -- when the batched plan is
available -- the batched forest of 256 clustered sets (kNN k = 8 + FoF).

Inputs are generated on the host and copied to the GPU before timing.  Each
stage is timed with HIP events on the stream that runs it; the headline value
is kNN queries per second of the k = 32 stage.  After the timed steps, outside
them: the per-set baseline of the batched mode, the dimensionality sweep
(build and k = 16 kNN of every point over 2^22 points in d = 2, 4, 8, 16,
uniform and normal, autotuned leaf size) and the CPU oracle on a bounded sample.  Prints ONE JSON
line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_POINTS = 1 << 24
N_QUERIES = 1 << 22
K = 32
RADIUS = 0.01
FOF_B = 0.2
GRID = 256
LEAF = 0         # the clustered workload's tree: the tuned leaf size (kdt_build picks it)
LEAF_FIXED = 32  # the small uniform workload, the batched sets and the oracle's tree
LARGE_K_QUERIES = 100_000
LARGE_KS = (100, 1000, 10_000)
HBM_PEAK_GBS = 8000.0
BATCH_SETS = 256


# Hardware counter passes, each a child run of this script under
# rocprofv3 --pmc (counters are read by the profiler around the program, so
# they cannot be taken from inside it).  The child replays three launches:
# the VALU-only probe (known instruction count: the issue-rate reference),
# a plain 1 GiB copy (the reference that scales FETCH_SIZE and WRITE_SIZE,
# in KiB per dispatch, to bytes) and the kNN traversal of the timed step.
COUNTER_PASSES = (("FETCH_SIZE",), ("WRITE_SIZE",), ("TCC_HIT_sum", "TCC_MISS_sum"),
                  ("SQ_WAVES", "SQ_INSTS_VALU", "GRBM_GUI_ACTIVE"))
KNN_KERNEL = "k_knn_lane<3, 32, false"
COPY_BYTES = 1 << 30
N_XCD = 8  # GRBM_GUI_ACTIVE is summed over the chip's 8 XCDs


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=1 << 14,
                    help="queries of the one-thread oracle timing")
    ap.add_argument("--cpu-queries-threaded", type=int, default=1 << 18,
                    help="queries of the oracle timing over the host's threads")
    ap.add_argument("--no-dsweep", action="store_true")
    ap.add_argument("--no-box", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small uniform workload (65536 points)")
    ap.add_argument("--no-large-k", action="store_true")
    ap.add_argument("--no-torus", action="store_true")
    ap.add_argument("--no-midpoint", action="store_true")
    ap.add_argument("--no-cloud", action="store_true")
    ap.add_argument("--no-grf", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-workcount", action="store_true")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the rocprofv3 counter passes over the kNN launch")
    ap.add_argument("--counter-child", action="store_true",
                    help="(run by the counter passes) only run the VALU probe, a 1 GiB copy "
                         "and the kNN launch of the step, once each")
    return ap.parse_args()


def counter_child(torch, kdt, workloads) -> None:
    """The launches the counter passes read: the VALU probe, a plain copy of
    COPY_BYTES, and the step's kNN launch (same inputs, tree and order)."""
    kdt.load()
    dev = torch.device("cuda:0")
    kdt.valu_probe()
    a = torch.ones(COPY_BYTES // 4, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    xt = torch.from_numpy(workloads.clustered(N_POINTS, seed=2)).to(dev)
    qt = torch.from_numpy(workloads.uniform(N_QUERIES, 3, seed=102)).to(dev)
    tree = kdt.build(xt, leaf_size=LEAF, tune_k=K, check_finite=True)
    order = tree.query_order(qt)
    tree.knn(qt, K, order=order)
    torch.cuda.synchronize()
    tree.close()


def counter_passes():
    """Runs the COUNTER_PASSES (a child of this script under rocprofv3 each)
    and returns the kNN launch's counters, scaled by the references, or a
    dict with an "error" entry."""
    import csv
    import shutil
    import signal
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3")
    if prof is None:
        return {"error": "rocprofv3 not found"}
    got = {}
    env = dict(os.environ, TMPDIR="/tmp")
    for i, counters in enumerate(COUNTER_PASSES):
        d = tempfile.mkdtemp(prefix="kdt_pmc_", dir="/tmp")
        cmd = [prof, "--pmc", *counters, "--output-format", "csv", "-d", d, "-o", "c", "--",
               sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--counter-child"]
        print(f"[bench] counter pass {i + 1}/{len(COUNTER_PASSES)}: {' '.join(counters)}",
              file=sys.stderr, flush=True)
        p = subprocess.Popen(cmd, cwd="/tmp", env=env, stdout=subprocess.PIPE,
                             stderr=subprocess.STDOUT, start_new_session=True)
        try:
            log, _ = p.communicate(timeout=180)
        except subprocess.TimeoutExpired:
            os.killpg(p.pid, signal.SIGKILL)
            p.communicate()
            return {"error": f"counter pass {counters} timed out"}
        path = os.path.join(d, "c_counter_collection.csv")
        if p.returncode != 0 and not os.path.exists(path):
            return {"error": f"counter pass {counters} exited {p.returncode}: "
                             + log.decode(errors="replace")[-300:]}
        per = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"]
                who = ("probe" if "k_valu_probe" in name else
                       "copy" if "copyBuffer" in name else
                       "knn" if KNN_KERNEL in name else None)
                if who is None:
                    continue
                e = per.setdefault((who, r["Dispatch_Id"]), {
                    "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
                e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        shutil.rmtree(d, ignore_errors=True)
        # one dispatch each: the longest (the library's own small copies are
        # copy dispatches too; the reference copy is the 1 GiB one)
        for who in ("probe", "copy", "knn"):
            runs = [e for (w, _), e in per.items() if w == who]
            if runs:
                got.setdefault(who, {}).update(max(runs, key=lambda e: e["ns"]))
    if set(got) != {"probe", "copy", "knn"}:
        return {"error": f"counter passes found {sorted(got)} of probe, copy, knn"}
    kib = 1024.0
    fetch_scale = COPY_BYTES / (got["copy"]["FETCH_SIZE"] * kib)
    write_scale = COPY_BYTES / (got["copy"]["WRITE_SIZE"] * kib)
    k, pr = got["knn"], got["probe"]
    fetch = k["FETCH_SIZE"] * kib * fetch_scale
    write = k["WRITE_SIZE"] * kib * write_scale
    probe_rate = pr["SQ_INSTS_VALU"] / (pr["GRBM_GUI_ACTIVE"] / N_XCD)
    knn_rate = k["SQ_INSTS_VALU"] / (k["GRBM_GUI_ACTIVE"] / N_XCD)
    hit, miss = k["TCC_HIT_sum"], k["TCC_MISS_sum"]
    return {
        "hbm_fetch_bytes": fetch, "hbm_write_bytes": write, "hbm_bytes": fetch + write,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "l2_hit_rate": hit / (hit + miss),
        "valu_per_wave": k["SQ_INSTS_VALU"] / k["SQ_WAVES"],
        "valu_per_cycle": knn_rate, "probe_valu_per_cycle": probe_rate,
        "valu_issue_frac": knn_rate / probe_rate,
        "clock_ghz": k["GRBM_GUI_ACTIVE"] / N_XCD / k["ns"],
    }


def small_uniform(torch, kdt, workloads, dev) -> dict:
    """The small uniform workload: 65536 points uniform in [0, 1)^3 (seed 1),
    leaf 32, every point a query: build, kNN k = 8 and closed-ball counts
    r = 0.02.  Each stage runs 20 times after 3 warm-ups; the median of the
    HIP-event times on the current stream is reported."""
    n = 1 << 16
    xt = torch.from_numpy(workloads.uniform(n, 3, seed=1)).to(dev)
    stream = torch.cuda.current_stream()

    def med(call, reps=20):
        for _ in range(3):
            keep = call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            keep = call()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
            del keep
        return float(np.median(ts))

    build_ms = med(lambda: kdt.build(xt, leaf_size=LEAF_FIXED, check_finite=True))
    tree = kdt.build(xt, leaf_size=LEAF_FIXED)
    knn_ms = med(lambda: tree.knn(None, 8))
    range_ms = med(lambda: tree.range(None, 0.02))
    tree.close()
    res = {"n_points": n, "leaf_size": LEAF_FIXED, "build_ms": build_ms,
           "build_mpts_s": n / (build_ms * 1e-3) / 1e6,
           "knn_k8_ms": knn_ms, "knn_queries_s": n / (knn_ms * 1e-3),
           "range_r002_ms": range_ms, "range_queries_s": n / (range_ms * 1e-3)}
    print(f"[bench] small uniform (65536): {res}", file=sys.stderr, flush=True)
    return res


def linking_length(n: int) -> float:
    return float(np.float32(FOF_B * (1.0 / n) ** (1.0 / 3.0)))


def workcount():
    """Counts of the instrumented library for the benchmarked launches (a
    child process: it loads libkdt_counts.so), or None if it is not built."""
    import subprocess
    from paper_2609_18316_amd import kdt
    if not os.path.exists(kdt.LIB_COUNTS_PATH):
        return None
    print("[bench] counting traversal work (instrumented library)", file=sys.stderr, flush=True)
    r = subprocess.run([sys.executable, "-m", "paper_2609_18316_amd.workcount"], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    sys.stderr.write(r.stderr[-2000:])
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def host_cpu():
    """CPU model (from /proc/cpuinfo) and core counts of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    return model, nproc, usable


def cpu_baseline(x, q, n_q1, n_qt):
    """The CPU oracle as written (single-threaded C): its sliding-midpoint tree
    over all points (one thread), kNN k = 32 of the first n_q1 queries on one
    thread, then of the first n_qt queries in contiguous slices over T host
    threads sharing the read-only tree (the paper runs its targets
    concurrently the same way).  T is the host's cores, at most 16."""
    import oracle
    model, nproc, usable = host_cpu()
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    tree = oracle.Tree(x, LEAF_FIXED)
    t1 = time.perf_counter()
    tree.knn(q[:n_q1], K)
    t2 = time.perf_counter()
    tree.knn(q[:n_qt], K, threads=threads)
    t3 = time.perf_counter()
    one = n_q1 / (t2 - t1)
    many = n_qt / (t3 - t2)
    return {"value": many, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle tree over all {x.shape[0]} points (one thread: build "
                      f"{t1 - t0:.1f} s, {x.shape[0] / (t1 - t0) / 1e6:.2f} Mpts/s), kNN k={K} of "
                      f"the first {n_qt} of the {q.shape[0]} queries in slices over {threads} "
                      f"threads; one thread on the first {n_q1}: {one:.4g} queries/s",
            "single_thread_value": one, "build_mpts_s": x.shape[0] / (t1 - t0) / 1e6,
            "cpu_model": model, "nproc": nproc, "usable_cpus": usable}


def dimension_sweep(torch, kdt, workloads, dev):
    """Build and kNN (k = 16, every point as a query) over 2^22 points in
    d = 2, 4, 8, 16, uniform and standard normal, with the leaf size and
    traversal the autotuner stored for each shape.  At d = 16 the search is
    close to brute force: about 12 s per distribution."""
    from paper_2609_18316_amd import autotune
    n, k = 1 << 22, 16
    rows = []
    for d in (2, 4, 8, 16):
        for dist in ("uniform", "normal"):
            pts = workloads.uniform(n, d, 300 + d) if dist == "uniform" else \
                workloads.normal(n, d, 400 + d)
            xt = torch.from_numpy(pts).to(dev)
            c = autotune.lookup(n, d, k, f"self-{dist}")
            trav = 2 if c.queries_per_wave == 64 else 1
            kdt.build(xt, leaf_size=c.leaf_size, check_finite=False).close()  # warm-up
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            t = kdt.build(xt, leaf_size=c.leaf_size, check_finite=False)
            e.record()
            torch.cuda.synchronize()
            build_ms = s.elapsed_time(e)
            nq = n
            s.record()
            t.knn(None, k, traversal=trav)
            e.record()
            torch.cuda.synchronize()
            knn_ms = s.elapsed_time(e)
            rows.append({"d": d, "dist": dist, "n": n, "leaf_size": c.leaf_size,
                         "traversal": "lane" if trav == 1 else "wave", "build_ms": build_ms,
                         "build_mpts_s": n / (build_ms * 1e-3) / 1e6, "queries": nq,
                         "knn_ms": knn_ms, "knn_queries_s": nq / (knn_ms * 1e-3)})
            t.close()
            del xt
            print(f"[bench] d={d} {dist}: build {build_ms:.2f} ms, kNN {knn_ms:.2f} ms "
                  f"({nq} queries)", file=sys.stderr, flush=True)
    return rows


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2609_18316_amd import kdt, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.counter_child:
        counter_child(torch, kdt, workloads)
        return
    kdt.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    t_gen = time.perf_counter()
    x = workloads.clustered(N_POINTS, seed=2)
    q = workloads.uniform(N_QUERIES, 3, seed=102)
    m = workloads.masses(N_POINTS, seed=5)
    print(f"[bench] inputs generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    xt = torch.from_numpy(x).to(dev)
    qt = torch.from_numpy(q).to(dev)
    mt = torch.from_numpy(m).to(dev)
    gen = torch.Generator(device=dev).manual_seed(7)
    gg = torch.randn((GRID,) * 3, device=dev, generator=gen)
    lo, cell, shape = (0.0, 0.0, 0.0), 1.0 / GRID, (GRID,) * 3
    l_fof = linking_length(N_POINTS)

    batch = None
    if not args.no_batch and hasattr(kdt.load(), "kdt_batch_plan_create"):
        sizes = workloads.batch_sizes(BATCH_SETS, 3.0, 6.0, seed=4)
        bx, boff = workloads.batched_clustered(sizes, seed_base=40000)
        bl = np.array([linking_length(int(s)) for s in sizes], np.float32)
        plan = kdt.BatchPlan(boff, 3, 8, LEAF_FIXED)
        bxt = torch.from_numpy(bx).to(dev)
        blt = torch.from_numpy(bl).to(dev)
        bout = (torch.empty((int(boff[-1]), 8), dtype=torch.int32, device=dev),
                torch.empty((int(boff[-1]), 8), dtype=torch.float32, device=dev),
                torch.empty(int(boff[-1]), dtype=torch.int32, device=dev))
        batch = (plan, bxt, blt, bout, int(boff[-1]))

    phases = ["build", "knn_order", "knn", "range", "fof", "hsml", "p2m_fwd", "p2m_bwd"]
    if batch:
        phases += ["batch_graph"]
    ev = {p: [] for p in phases}
    torch.cuda.synchronize()

    def step(record):
        marks = {}

        def mark(name):
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            marks[name] = e

        mark("start")
        # the finiteness check is deferred (no host wait inside the step) and
        # read once after the timed steps
        tree = kdt.build(xt, leaf_size=LEAF, tune_k=K, check_finite="deferred")
        mark("build")
        order = tree.query_order(qt)
        mark("knn_order")
        idx, d2 = tree.knn(qt, K, order=order)
        mark("knn")
        cnt = tree.range(qt, RADIUS)  # sorts its queries (Hilbert order) itself
        mark("range")
        lab = tree.fof(l_fof)
        mark("fof")
        # smoothing lengths, masses and gradients in tree order: every pass of
        # the deposit streams contiguous arrays; the gradients go back to
        # input order at the end
        h = tree.knn(None, K, kth_only=2, tree_rows=True)
        mark("hsml")
        m_t = tree.gather(mt)
        rho = kdt.p2m_tree(tree, m_t, h, lo, cell, shape)
        mark("p2m_fwd")
        gm_t, gx_t = kdt.p2m_tree_backward(tree, m_t, h, lo, cell, shape, gg)
        gm, gx = tree.scatter(gm_t), tree.scatter(gx_t)
        mark("p2m_bwd")
        if batch:
            plan, bxt, blt, bout, _ = batch
            plan.launch(bxt, blt, use_graph=1, out=bout)
            mark("batch_graph")
        if record:
            order = ["start"] + phases
            torch.cuda.synchronize()
            for a, b in zip(order[:-1], order[1:]):
                ev[b].append(marks[a].elapsed_time(marks[b]))
        return tree, (idx, d2, cnt, lab, rho, gm, gx)

    for _ in range(args.warmup):
        keep = step(False)
        del keep
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        keep = step(True)
        last_tree = keep[0]
        del keep
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last_tree.check()  # the deferred finiteness check of the step's build
    del last_tree
    ms_step = elapsed * 1e3 / args.steps
    avg = {p: float(np.mean(ev[p])) for p in phases}

    # Headline: the whole kNN call as a user makes it (ordering the queries
    # along the tree, then the traversal kernel).
    knn_qps = N_QUERIES / ((avg["knn_order"] + avg["knn"]) * 1e-3)
    # Roofline of the traversal kernel (one launch, timed alone): compulsory
    # bytes per query are the query coordinates in (4 d) plus k (index, d2)
    # pairs out (8 k).
    knn_bytes = N_QUERIES * (4 * 3 + 8 * K)
    achieved = knn_bytes / (avg["knn"] * 1e-3) / 1e9
    out = {
        "metric": "kNN queries/s (k=32, 2^24 pts) + build Mpts/s; batched speedup; P2M bwd/fwd",
        "value": knn_qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "clustered 3-D, 2^24 points (2000 Gaussian halos + 20% uniform), "
                        "2^22 uniform queries, kNN k=32, ball r=0.01, FoF b=0.2, "
                        "SPH P2M 256^3 with adjoint, batched 256 clustered sets",
            "n_points": N_POINTS, "n_queries": N_QUERIES, "k": K, "radius": RADIUS,
            "leaf_size": kdt.tuning_get(3, N_POINTS, K)[0], "grid": GRID,
            "fof_linking_length": l_fof,
        },
        "phases_ms": avg,
        "build_mpts_s": N_POINTS / (avg["build"] * 1e-3) / 1e6,
        "knn_queries_s": knn_qps,
        "range_queries_s": N_QUERIES / (avg["range"] * 1e-3),
        "fof_mpts_s": N_POINTS / (avg["fof"] * 1e-3) / 1e6,
        "p2m_bwd_over_fwd": avg["p2m_bwd"] / avg["p2m_fwd"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_knn_lane<3,32,false> (kNN traversal, k=32, one query per lane): "
                               "compulsory bytes 4d + 8k = 268 per query"},
    }
    if batch:
        # The baseline (the single-tree entry points once per set, eager) is
        # timed outside the timed steps: it is a comparison, not the path.
        plan, bxt, blt, bout, _ = batch
        plan.launch(bxt, blt, use_graph=0, out=bout)
        torch.cuda.synchronize()
        reps = []
        for _ in range(2):
            t_b = time.perf_counter()
            plan.launch(bxt, blt, use_graph=0, out=bout)
            torch.cuda.synchronize()
            reps.append((time.perf_counter() - t_b) * 1e3)
        out["batch_per_set_eager_ms"] = float(np.mean(reps))
        out["batched_speedup"] = out["batch_per_set_eager_ms"] / avg["batch_graph"]
        out["batched_points"] = batch[4]
    if not args.no_small:
        out["small_uniform"] = small_uniform(torch, kdt, workloads, dev)
    if not args.no_box:
        # Box queries (the rectangular ranges, a widening of the path): cubes of
        # the ball's volume (side 0.0161 for r = 0.01) centred on the 2^22
        # queries, counts on the step's tree, built again; outside the timed steps.
        half = 0.5 * (4.0 / 3.0 * np.pi) ** (1.0 / 3.0) * RADIUS
        blo, bhi = (qt - half).contiguous(), (qt + half).contiguous()
        tree = kdt.build(xt, leaf_size=LEAF, tune_k=K)
        tree.box(blo, bhi)
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            tree.box(blo, bhi)
            e1.record()
            torch.cuda.synchronize()
            reps.append(e0.elapsed_time(e1))
        box_ms = float(np.median(reps))
        out["box"] = {"ms": box_ms, "queries_s": N_QUERIES / (box_ms * 1e-3),
                      "side": 2 * half, "n_boxes": N_QUERIES}
        del blo, bhi
        # Ball lists (CSR) of the same r = 0.01 balls of the 2^22 queries: the
        # whole call (counts and offsets, a host read of the total, the fill
        # and the per-row sort), timed on the host around a synchronised call.
        tree.range(qt, RADIUS, lists=True)
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            t_l = time.perf_counter()
            lc, loff, lidx = tree.range(qt, RADIUS, lists=True)
            torch.cuda.synchronize()
            reps.append((time.perf_counter() - t_l) * 1e3)
        lists_ms = float(np.median(reps))
        out["ball_lists"] = {"ms": lists_ms, "queries_s": N_QUERIES / (lists_ms * 1e-3),
                             "pairs": int(lidx.numel()),
                             "pairs_s": lidx.numel() / (lists_ms * 1e-3)}
        del lc, loff, lidx
        tree.close()
    if not args.no_large_k:
        # kNN with k above the 64 register entries (the ball-and-sort path, a
        # widening of the path): 10^5 of the queries, k = 100 (the paper's
        # parallel test), 1000 and 10^4 (the top of its k sweep), full lists,
        # on the step's tree built again; outside the timed steps.
        tree = kdt.build(xt, leaf_size=LEAF, tune_k=K)
        qk = qt[:LARGE_K_QUERIES].contiguous()
        out["large_k"] = {"n_queries": LARGE_K_QUERIES}
        for kk in LARGE_KS:
            r = tree.knn(qk, kk)
            del r
            torch.cuda.synchronize()
            reps = []
            for _ in range(2):
                t_k = time.perf_counter()
                r = tree.knn(qk, kk)
                torch.cuda.synchronize()
                reps.append((time.perf_counter() - t_k) * 1e3)
                del r
            ms = float(np.min(reps))
            out["large_k"][str(kk)] = {"ms": ms, "queries_s": LARGE_K_QUERIES / (ms * 1e-3)}
        tree.close()
    if not args.no_torus:
        # Periodic boundaries (the unit box as a 3-torus, a widening of the
        # path): kNN k = 32 of the 2^22 queries, r = 0.01 counts and FoF
        # b = 0.2 of the 2^24 points, one traversal per lane, on the step's
        # tree built again; best of two calls each, outside the timed steps.
        tree = kdt.build(xt, leaf_size=LEAF, tune_k=K)
        out["torus"] = {"period": 1.0}
        calls = {"knn": lambda: tree.knn(qt, K, period=1.0),
                 "range": lambda: tree.range(qt, RADIUS, period=1.0),
                 "fof": lambda: tree.fof(l_fof, period=1.0)}
        for name, call in calls.items():
            r = call()
            del r
            torch.cuda.synchronize()
            reps = []
            for _ in range(2):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                r = call()
                e1.record()
                torch.cuda.synchronize()
                reps.append(e0.elapsed_time(e1))
                del r
            out["torus"][name + "_ms"] = float(min(reps))
        out["torus"]["knn_queries_s"] = N_QUERIES / (out["torus"]["knn_ms"] * 1e-3)
        tree.close()
    if not args.no_midpoint:
        # The paper's sliding-midpoint split rule (outside the timed step):
        # build, kNN k = 32 of the 2^22 queries and r = 0.01 counts on that
        # tree, best of three calls each, beside the median tree of the step.
        def timed(call, reps=3):
            r = call()
            del r
            torch.cuda.synchronize()
            best = None
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                r = call()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
                del r
            return best
        b_ms = timed(lambda: kdt.build(xt, leaf_size=LEAF, tune_k=K, check_finite=False,
                                       split_rule=kdt.SPLIT_MIDPOINT))
        mtree = kdt.build(xt, leaf_size=LEAF, tune_k=K, split_rule=kdt.SPLIT_MIDPOINT)
        k_ms = timed(lambda: mtree.knn(qt, K))
        r_ms = timed(lambda: mtree.range(qt, RADIUS))
        out["midpoint"] = {"leaf_size": mtree.info.leaf_size, "depth": mtree.info.levels,
                           "n_nodes": mtree.info.n_nodes, "build_ms": b_ms,
                           "build_mpts_s": N_POINTS / (b_ms * 1e-3) / 1e6, "knn_ms": k_ms,
                           "knn_queries_s": N_QUERIES / (k_ms * 1e-3), "range_ms": r_ms,
                           "range_queries_s": N_QUERIES / (r_ms * 1e-3),
                           "median_tree": {"build_ms": avg["build"],
                                           "knn_ms": avg["knn_order"] + avg["knn"],
                                           "range_ms": avg["range"]}}
        mtree.close()
        # the like-for-like comparison: the median tree with one traversal per
        # lane for the counts as well (the sliding-midpoint tree has no
        # wave-shared count)
        mt2 = kdt.build(xt, leaf_size=LEAF, tune_k=K)
        out["midpoint"]["median_tree"]["range_lane_ms"] = timed(
            lambda: mt2.range(qt, RADIUS, traversal=1))
        mt2.close()
        print(f"[bench] sliding midpoint: build {b_ms:.2f} ms, kNN {k_ms:.2f} ms, "
              f"counts {r_ms:.2f} ms", file=sys.stderr, flush=True)
    if not args.no_cloud:
        # The fixed-cloud deposits the paper compares the adaptive one with
        # (Table 3): the same 2^24 particles and 256^3 mesh in tree order as
        # the adaptive deposit of the step (masses gathered into tree order
        # inside the timed call, as there), best of three after one warm-up;
        # then the caller's arrays visited through the tree order
        # ("perm_order") and in input order (no order given).
        out["cloud"] = {"p2m_sph_fwd_ms": avg["p2m_fwd"]}
        ctree = kdt.build(xt, leaf_size=LEAF, tune_k=K)
        h_c = ctree.knn(None, K, kth_only=2)
        for scheme, how in (("ngp", "tree"), ("cic", "tree"), ("tsc", "tree"),
                            ("tsc", "perm_order"), ("tsc", "input_order"),
                            ("sph", "perm_order"), ("sph", "input_order")):
            best = None
            order_ptr = ctree.perm_ptr if how == "perm_order" else None
            for _ in range(4):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                if how == "tree":
                    r = kdt.p2m_tree(ctree, ctree.gather(mt), None, lo, cell, shape,
                                     scheme=scheme)
                elif scheme == "sph":
                    r = kdt.p2m(xt, mt, h_c, lo, cell, shape, order_ptr=order_ptr)
                else:
                    r = kdt.p2m_cloud(xt, mt, lo, cell, shape, scheme, order_ptr=order_ptr)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                if _ > 0:  # the first call warms up
                    best = ms if best is None else min(best, ms)
                del r
            out["cloud"][scheme + ("" if how == "tree" else "_" + how) + "_ms"] = best
        ctree.close()
        out["cloud"]["sph_over_tsc"] = avg["p2m_fwd"] / out["cloud"]["tsc_ms"]
    if not args.no_f64:
        # Float64 coordinates (the double-precision real kind of Sec. 2.4):
        # the same 2^24 points and 2^22 queries widened to float64, tuned
        # leaf; build, kNN k = 32 and r = 0.01 counts, best of three.
        x64 = xt.double()
        q64 = qt.double()

        def best3(call):
            call()
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                keep = call()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
                del keep
            return float(min(ts))

        f_build = best3(lambda: kdt.build_f64(x64, leaf_size=LEAF, tune_k=K, check_finite=False))
        ft = kdt.build_f64(x64, leaf_size=LEAF, tune_k=K)
        f_knn = best3(lambda: ft.knn(q64, K))
        f_rng = best3(lambda: ft.range(q64, RADIUS))
        out["f64"] = {"build_ms": f_build, "knn_ms": f_knn, "range_ms": f_rng,
                      "build_mpts_s": N_POINTS / (f_build * 1e-3) / 1e6,
                      "knn_queries_s": N_QUERIES / (f_knn * 1e-3),
                      "range_queries_s": N_QUERIES / (f_rng * 1e-3),
                      "leaf_size": ft.info.leaf_size}
        ft.close()
        del x64, q64
        print(f"[bench] float64 coordinates: {out['f64']}", file=sys.stderr, flush=True)
    if not args.no_grf:
        # The paper's inhomogeneous mock (Sec. 3.1): 2^24 points from a
        # Gaussian random field of spectral index -2; build, kNN k = 32 of the
        # 2^22 uniform queries, r = 0.01 counts and FoF b = 0.2 on it.
        t_g = time.perf_counter()
        xg = torch.from_numpy(workloads.grf(N_POINTS, seed=7)).to(dev)
        gen_s = time.perf_counter() - t_g

        def best_of(call, reps=3):
            r = call()
            del r
            torch.cuda.synchronize()
            best = None
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                r = call()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
                del r
            return best
        gtree = kdt.build(xg, leaf_size=LEAF, tune_k=K)
        out["grf"] = {
            "n_points": N_POINTS, "generation_s": gen_s,
            "build_ms": best_of(lambda: kdt.build(xg, leaf_size=LEAF, tune_k=K, check_finite=False)),
            "knn_ms": best_of(lambda: gtree.knn(qt, K)),
            "range_ms": best_of(lambda: gtree.range(qt, RADIUS)),
            "fof_ms": best_of(lambda: gtree.fof(l_fof)),
            "midpoint_build_ms": best_of(lambda: kdt.build(
                xg, leaf_size=LEAF, tune_k=K, check_finite=False, split_rule=kdt.SPLIT_MIDPOINT), reps=2),
        }
        out["grf"]["knn_queries_s"] = N_QUERIES / (out["grf"]["knn_ms"] * 1e-3)
        gtree.close()
        del xg
        print(f"[bench] GRF mock: {out['grf']}", file=sys.stderr, flush=True)
    if not args.no_dsweep:
        out["dsweep"] = dimension_sweep(torch, kdt, workloads, dev)
    if not args.no_workcount:
        # Algorithmic bytes of the kNN launch: the compulsory term (queries
        # in, results out) plus the traversal term, leaf points scanned x
        # record bytes + node boxes read x box bytes, counted by the
        # instrumented library in a child process on the same launch.
        wc = workcount()
        if wc:
            out["workcount"] = wc
            kc = wc["knn_c2"]
            trav = kc["lane_points"] * kc["record_bytes"] + kc["lane_nodes"] * kc["box_bytes"]
            rf = out["roofline"]
            rf["algorithmic_bytes"] = {
                "compulsory": knn_bytes, "traversal": trav,
                "leaf_points_per_query": kc["lane_points"] / N_QUERIES,
                "nodes_per_query": kc["lane_nodes"] / N_QUERIES,
                "list_inserts_per_query": kc["lane_inserts"] / N_QUERIES,
                "box_reloads_per_query": kc["lane_node_reloads"] / N_QUERIES}
            rf["compulsory_frac"] = rf["frac"]
            rf["achieved"] = (knn_bytes + trav) / (avg["knn"] * 1e-3) / 1e9
            rf["frac"] = rf["achieved"] / HBM_PEAK_GBS
            rf["kernel"] += "; traversal bytes: leaf points x 16 + node boxes x 32"
    if not args.no_counters:
        # HBM traffic, L2 hit rate and VALU issue of the kNN launch, from
        # counter passes over the same launch (children of this script).
        c = counter_passes()
        rf = out["roofline"]
        rf["counters"] = c
        if "error" not in c:
            rf["traffic"] = c["hbm_bytes"]
            rf["traffic_gbs"] = c["hbm_bytes"] / (avg["knn"] * 1e-3) / 1e9
            rf["l2_hit_rate"] = c["l2_hit_rate"]
            rf["valu_issue_frac"] = c["valu_issue_frac"]
        print(f"[bench] counters: {c}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(x, q, args.cpu_queries, args.cpu_queries_threaded)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
