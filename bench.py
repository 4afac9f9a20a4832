"""Benchmark of the per-tick k-NN join on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload clustered_1m]

A step is one tick of the whole hot path on device-resident inputs: the
snapshot copy into the context, the index build (Morton codes, radix sort,
leaf split, node tables) and one k-NN query per object (Sec. 4 of arXiv
1412.6170).  Positions of every tick are generated and copied to HBM before
the timed region; results stay in HBM (fetching them is not part of a tick).

Prints one JSON line: queries/s over the K timed ticks, p50/p99 tick latency,
a roofline entry for the dominant kernel (the leaf-sweep query kernel,
algorithmic bytes over its mean device time from the library's HIP events on
the stream it runs on) and the CPU oracle timed on the host cores on a
bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def query_kernel_bytes(n, nq, k):
    """Algorithmic bytes of one launch of the query kernel: every sorted
    object read once (x, y, id: 12 B) and every result row written once
    (k ids + k squared distances + a count: 8k + 4 B)."""
    return 12 * n + nq * (8 * k + 4)


def tick_bytes(n, nq, k):
    """Algorithmic bytes of a whole tick: positions read (8 B), sorted
    objects written (12 B) and read back (12 B), results written."""
    return 32 * n + nq * (8 * k + 4)


def host_threads():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, 16))


def cpu_baseline(w):
    """The oracle as it stands, on tick 0 of the workload: quadtree build plus
    every query, split by query over the host threads."""
    import oracle
    x, y, _, _, k = w.tick(0)
    threads = host_threads()
    oracle.knn(x[:20000], y[:20000], k=k, threads=threads)  # load + warm the library
    t0 = time.perf_counter()
    oracle.knn(x, y, k=k, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": len(x) / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "tick 0 of %s: index build + all %d queries (k=%d), %.2f s" % (
                w.name, len(x), k, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered_1m")
    ap.add_argument("--leaf-capacity", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the k-NN tick on a single MI355X "
              "and has no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1412_6170_amd import binding, workloads

    torch.cuda.set_device(0)
    w = workloads.WORKLOADS[args.workload]()
    n, k = w.n, w.k
    print("bench: generating %d ticks of %s" % (w.ticks, w.name), file=sys.stderr, flush=True)
    dev = []
    for t in range(w.ticks):
        x, y, _, _, _ = w.tick(t)
        dev.append((torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()))
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ctx = binding.Context(n, n, k, leaf_capacity=args.leaf_capacity, k_hint=k,
                          stream=stream.cuda_stream, timing=True)

    def step(s):
        x, y = dev[s % w.ticks]
        ctx.load_positions(x, y)
        ctx.advance_tick()
        ctx.query(k=k)

    for s in range(args.warmup):
        step(s)
    ctx.sync()
    ctx.reset_timing()
    print("bench: warmup done, timing %d steps" % args.steps, file=sys.stderr, flush=True)

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        starts[s].record(stream)
        step(s)
        ends[s].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()

    lat = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    st = ctx.stats()
    nq = n
    value = args.steps * nq / wall
    kern_ms = st["ms_query_main_mean"]
    kern_bytes = query_kernel_bytes(n, nq, k)
    achieved = kern_bytes / (kern_ms * 1e-3) / 1e9
    tick_ms = float(np.mean(lat))
    out = {
        "metric": "k-NN queries/sec per tick (build+query), 1M objs k=32; p50/p99 tick latency",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "objects": n, "queries_per_tick": nq, "k": k,
                   "ticks": w.ticks, "leaf_capacity": st["leaf_capacity"],
                   "description": w.description},
        "p50_tick_ms": float(np.percentile(lat, 50)),
        "p99_tick_ms": float(np.percentile(lat, 99)),
        "device_ms_build_mean": st["ms_build_mean"],
        "device_ms_query_mean": st["ms_query_mean"],
        "tick_hbm_frac": tick_bytes(n, nq, k) / (tick_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "leaves": st["leaves"],
        "deepest_level": st["deepest_level"],
        "roofline": {"bound": "hbm", "kernel": "k_knn_tiles<32> (leaf sweeps)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel_ms": kern_ms, "bytes_per_launch": kern_bytes},
        "cpu_baseline": None,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
