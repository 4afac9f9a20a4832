"""Benchmark of the per-tick k-NN join on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload clustered_1m]
                    [--leaf-capacity TH | --autotune] [--max-level L] [--no-graph]
                    [--counters] [--no-cpu-baseline]
    python bench.py --serving [--scenes 64] [--rate R] [--slots 4]

A step is one tick of the whole hot path on device-resident inputs: the
index build (Morton codes, radix sort, leaf split, node tables) over the
tick's positions and one k-NN query per object (Sec. 4 of arXiv 1412.6170).
Positions of every tick are generated and copied to HBM before the timed
region; the library reads them in place; results stay in HBM (fetching them
is not part of a tick).

The schedule (leaf capacity, maximum quadtree level, sweep flavour and,
for variable k, k grouping) is chosen during warm-up by the library's
autotuner (coordinate descent over device time per tick, SCHEDULE_SPACE);
--no-autotune takes the autotuner's stored choice for the workload on
MI355X (TUNED_SCHEDULE), and --leaf-capacity / --max-level / --sweep fix a
dimension.  Results never depend on the schedule.

Prints one JSON line: queries/s over the K timed ticks, p50/p99 tick latency,
a roofline entry for the dominant kernel (the leaf-sweep query kernel,
algorithmic bytes over its mean device time from the library's HIP events on
the stream it runs on), the same ticks replayed as captured HIP graphs, the
same ticks with two in flight on two streams (a tick's build overlapping
the previous tick's query), the same ticks with index reuse (refit ticks
between rebuilds, Sec. 4.1), and the CPU oracle timed on the host cores on
a bounded sample.
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
TH_CANDIDATES = (16, 24, 32, 48, 64, 96, 128, 192, 256, 384)
# The autotuner's search space: leaf capacity, maximum quadtree level (l_max,
# Sec. 4.1: the build sorts only the top 2 * l_max bits of the Morton codes,
# so 12 saves a radix pass over 16), sweep flavour (one query per lane, or
# one query per wavefront: Sec. 4.2.1's cached and coalesced-writes
# variants) and, for variable k, k grouping.
SCHEDULE_SPACE = {"leaf_capacity": TH_CANDIDATES, "max_level": (8, 10, 12, 14, 16),
                  "sweep": ("lane", "wave", "group"), "group_k": (False, True)}
# The autotuner's choice on MI355X per workload, used with --no-autotune.
TUNED_SCHEDULE = {
    "uniform_10k": {"leaf_capacity": 24, "max_level": 8, "sweep": "lane", "group_k": False},
    "clustered_1m": {"leaf_capacity": 32, "max_level": 12, "sweep": "lane", "group_k": False},
    "network_4m": {"leaf_capacity": 128, "max_level": 12, "sweep": "group", "group_k": False},
    "mixed_16m": {"leaf_capacity": 384, "max_level": 16, "sweep": "group", "group_k": False},
}
CPU_SAMPLE_SECONDS = 10.0
# Maximum quadtree level of the served scenes: three radix passes per build
# (the default level 16 takes four); a level-12 cell holds few objects even
# in the cores of the 2M-object scenes at leaf capacity 32.
SERVING_MAX_LEVEL = 12

# HBM bytes per launch of the query kernel on clustered_1m for the schedules
# the autotuner picks there, from two rocprofv3 --pmc runs per schedule
# (FETCH_SIZE, then WRITE_SIZE), each scaled by what the same counter reads
# for a plain device copy of known size, and its VALU instructions per launch
# (SQ_INSTS_VALU, a third run).  Valid only for the kernel code they were
# taken on (digest of the query kernel's sources without comments);
# otherwise the roofline's traffic is null.
MEASURED_TRAFFIC = [
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 24, "max_level": 12,
     "fetch_bytes": 55443392, "write_bytes": 290688408, "valu_insts": 144883969},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 32, "max_level": 12,
     "fetch_bytes": 50939307, "write_bytes": 290666216, "valu_insts": 145872259},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 48, "max_level": 12,
     "fetch_bytes": 44609942, "write_bytes": 290686464, "valu_insts": 152216302},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 64, "max_level": 12,
     "fetch_bytes": 40127199, "write_bytes": 290706072, "valu_insts": 162763306},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 96, "max_level": 12,
     "fetch_bytes": 37453098, "write_bytes": 290729992, "valu_insts": 174469002},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 24, "max_level": 14,
     "fetch_bytes": 55767587, "write_bytes": 290656272, "valu_insts": 143746888},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 32, "max_level": 14,
     "fetch_bytes": 51718662, "write_bytes": 290709408, "valu_insts": 144770354},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 48, "max_level": 14,
     "fetch_bytes": 45067886, "write_bytes": 290707864, "valu_insts": 151193084},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 64, "max_level": 14,
     "fetch_bytes": 40372394, "write_bytes": 290692296, "valu_insts": 161846035},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 96, "max_level": 14,
     "fetch_bytes": 37656760, "write_bytes": 290724896, "valu_insts": 173701547},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 32, "max_level": 16,
     "fetch_bytes": 51747844, "write_bytes": 290688760, "valu_insts": 144708232},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 48, "max_level": 16,
     "fetch_bytes": 45383506, "write_bytes": 290706072, "valu_insts": 151134466},
    {"digest": "9adfa7701465ad9e", "workload": "clustered_1m", "leaf_capacity": 64, "max_level": 16,
     "fetch_bytes": 40397928, "write_bytes": 290736048, "valu_insts": 161788745},
]


def code_only(text):
    """C++ source without comments and with runs of blank space collapsed:
    what the compiler sees, so editing a comment keeps a digest valid."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


# Sources a query kernel is compiled from: its flavour's file and the
# shared headers.
DIGEST_COMMON = ("query.hpp", "query_device.hpp", "mknn_internal.hpp")
DIGEST_FLAVOUR = {"lane": "query.hip", "group": "query_group.hip", "wave": "query_wave.hip"}


def digest_files(sweep="lane"):
    return (DIGEST_FLAVOUR[sweep],) + DIGEST_COMMON


DIGEST_FILES = digest_files("lane")


def query_source_digest(read=None, sweep="lane"):
    import hashlib
    h = hashlib.sha256()
    for f in digest_files(sweep):
        if read is None:
            with open(os.path.join(ROOT, "paper_1412_6170_amd", "csrc", f)) as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(code_only(text).encode())
    return h.hexdigest()[:16]


def _measured(workload, leaf_capacity, max_level, sweep="lane"):
    digest = None
    for m in MEASURED_TRAFFIC:
        if (m["workload"] == workload and m["leaf_capacity"] == leaf_capacity
                and m.get("max_level", 16) == max_level and m.get("sweep", "lane") == sweep):
            digest = digest or query_source_digest(sweep=sweep)
            if m["digest"] == digest:
                return m
    return None


def measured_traffic(workload, leaf_capacity, max_level=16, sweep="lane"):
    m = _measured(workload, leaf_capacity, max_level, sweep)
    return None if m is None else m["fetch_bytes"] + m["write_bytes"]


# VALU issue peak of MI355X without packed arithmetic: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz lane operations per second.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def valu_issue(workload, leaf_capacity, max_level, kernel_ms, sweep="lane"):
    """VALU lane operations the query kernel issues per second (the stored
    SQ_INSTS_VALU count of one launch, 64 lanes each, over the kernel's
    measured mean time) against the issue peak, or None if the count was
    taken on other code or another configuration."""
    m = _measured(workload, leaf_capacity, max_level, sweep)
    if m is None or not m.get("valu_insts") or not kernel_ms:
        return None
    ops = m["valu_insts"] * 64 / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": ops / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
            "unit": "T lane-ops/s", "frac": ops / VALU_PEAK_LANE_OPS,
            "note": "executed VALU instructions (SQ_INSTS_VALU, rocprofv3 --pmc) x 64 lanes "
                    "per launch over the kernel's mean time; not algorithmic work"}


def query_kernel_bytes(n, nq, entries):
    """Algorithmic bytes of one launch of the query kernel: every sorted
    object read once (x, y, id: 12 B) and every result row written once
    (k ids + k squared distances + a count: 8k + 4 B per query; entries is
    the sum of k over the queries)."""
    return 12 * n + 8 * entries + 4 * nq


def tick_bytes(n, nq, entries, subset):
    """Algorithmic bytes of a whole tick: positions read (8 B), sorted
    objects written (12 B) and read back (12 B), the query list read when
    a subset queries (issuer and k: 8 B per query), results written."""
    return 32 * n + (8 * nq if subset else 0) + 8 * entries + 4 * nq


def roofline_entry(workload, leaf_capacity, max_level, k, kern_ms, kern_bytes, sweep="lane"):
    """Roofline entry of the query kernel.  Both roofs are computed: HBM
    (algorithmic bytes per launch over the kernel's mean device time, against
    8 TB/s) and VALU issue (the stored executed-instruction count of a
    launch, 64 lanes each, over the same time, against the issue peak).
    `bound` names the roof the kernel is closer to; the HBM figures are kept
    beside it whichever it is."""
    achieved = kern_bytes / (kern_ms * 1e-3) / 1e9
    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS,
           "traffic": measured_traffic(workload, leaf_capacity, max_level, sweep)}
    if sweep == "wave":
        kclass = max(64, 1 << (max(k, 1) - 1).bit_length())
        name = "k_knn_wave (one query per wavefront), list of %d keys" % kclass
    elif sweep == "group":
        kclass = max(32, 1 << (max(k, 1) - 1).bit_length())
        name = "k_knn_group (one query per %d lanes), list of %d keys" % (kclass // 16, kclass)
    else:
        kclass = 8 if k <= 8 else 16 if k <= 16 else 32 if k <= 32 else 64 if k <= 64 else 128
        name = "k_knn_tiles (one query per lane), k class %d" % kclass
    common = {"kernel": name, "kernel_ms": kern_ms, "bytes_per_launch": kern_bytes}
    valu = valu_issue(workload, leaf_capacity, max_level, kern_ms, sweep)
    if valu is not None and valu["frac"] > hbm["frac"]:
        out = {"bound": "alu", "achieved": valu["achieved"], "peak": valu["peak"],
               "unit": valu["unit"], "frac": valu["frac"], "traffic": hbm["traffic"],
               "hbm_achieved_gbs": hbm["achieved"], "hbm_frac": hbm["frac"],
               "alu_note": valu["note"]}
    else:
        out = hbm
    out.update(common)
    return out


def host_threads():
    """Every core this process may run on (its affinity set)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def cpu_model():
    """Host CPU model name and logical core count, from /proc/cpuinfo."""
    name, count = None, 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    count += 1
                    if name is None:
                        name = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return {"model": name or "unknown", "logical_cpus": count or (os.cpu_count() or 0)}


def _oracle_tick(oracle, w, tick, threads, rng, cap):
    """One tick of the oracle: quadtree build plus the tick's queries (above
    `cap` queries, a fixed random sample of `cap` of them)."""
    x, y, iss, ks = tick
    nq = len(x) if iss is None else len(iss)
    if nq > cap:
        pick = np.sort(rng.choice(nq, cap, replace=False))
        iss = pick.astype(np.int32) if iss is None else iss[pick]
        ks = None if ks is None else ks[pick]
        nq = len(pick)
    if ks is None:
        oracle.knn(x, y, issuers=iss, k=w.k, threads=threads)
    else:
        oracle.knn(x, y, issuers=iss, ks=ks, threads=threads)
    return nq


def cpu_baseline(w, host_ticks, seconds_all=CPU_SAMPLE_SECONDS, seconds_one=CPU_SAMPLE_SECONDS):
    """The oracle as it stands: quadtree build plus the queries of a tick,
    timed twice on the host: split by query over every core of the
    process's affinity set, and on one thread (the paper's sequential
    competitor setting).  Each leg repeats the workload's ticks until its
    time budget has passed (at least one tick); above 2M queries per tick
    a fixed random sample of 1M of them is answered."""
    import oracle
    threads = host_threads()
    x0, y0, _, _ = host_ticks[0]
    oracle.knn(x0[:20000], y0[:20000], k=8, threads=threads)  # load + warm the library

    def leg(nthreads, budget):
        rng = np.random.default_rng(1)
        done, queries = 0, 0
        t0 = time.perf_counter()
        while True:
            queries += _oracle_tick(oracle, w, host_ticks[done % len(host_ticks)], nthreads,
                                    rng, 1_000_000)
            done += 1
            dt = time.perf_counter() - t0
            if dt >= budget:
                return queries / dt, done, queries, dt

    v_all, t_all, q_all, s_all = leg(threads, seconds_all)
    v_one, t_one, q_one, s_one = leg(1, seconds_one)
    cpu = cpu_model()
    return {"value": v_all, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "value_1thread": v_one, "threads_all": threads, "cpu_model": cpu["model"],
            "host_logical_cpus": cpu["logical_cpus"],
            "sample": "all cores (%d threads): %d ticks of %s (cycling over %d generated ticks), "
                      "index build + %d queries, %.1f s; 1 thread: %d ticks, %d queries, "
                      "%.1f s" % (threads, t_all, w.name, len(host_ticks), q_all, s_all,
                                  t_one, q_one, s_one)}


def copy_calibration():
    """A plain 256 MiB device copy, repeated: what FETCH_SIZE and WRITE_SIZE
    read for it scales those counters to bytes for the query kernel."""
    import torch
    torch.cuda.set_device(0)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": src.numel() * 4,
                      "repeats": 5}), flush=True)


def run_serving(args):
    """Many independent scenes served with continuous batching: scene sizes
    log-uniform in [10k, 2M] objects, k in {8, 32}, tick requests arriving as
    a Poisson process; latency from arrival to device completion.  Returns
    the summary (saturation rate, then the Poisson run at 0.7 x that rate
    unless args.rate is set)."""
    import torch
    from paper_1412_6170_amd import serving, workloads
    torch.cuda.set_device(0)
    rng = np.random.default_rng(args.serving_seed)
    scenes = []
    print("bench: generating %d scenes" % args.scenes, file=sys.stderr, flush=True)
    for sid in range(args.scenes):
        n = int(round(np.exp(rng.uniform(np.log(10_000), np.log(2_000_000)))))
        k = int(rng.choice([8, 32]))
        w = workloads.clustered_1m(n=n, ticks=args.scene_ticks)
        pos = []
        for t in range(args.scene_ticks):
            x, y, _, _, _ = w.tick(t)
            pos.append((torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()))
        scenes.append(serving.Scene(sid, pos, k, leaf_capacity=args.leaf_capacity or 32,
                                    max_level=args.max_level or SERVING_MAX_LEVEL,
                                    tile_queries=args.tile_queries))
    torch.cuda.synchronize()
    budget = int(args.hbm_budget_gib * 2 ** 30)
    srv = serving.Server(scenes, hbm_budget=budget, slots=args.slots)
    ids = [s.sid for s in scenes]
    by_id = {s.sid: s for s in scenes}
    # warm-up: one tick of every scene (contexts created, kernels loaded)
    srv.run([(0.0, sid, 0) for sid in ids])
    # Saturation: every request of the schedule present at once.
    sat_done = srv.run([(0.0, sid, t) for sid in ids for t in range(args.scene_ticks)])
    sat = serving.summarize(sat_done, by_id)
    sat_rate = sat["requests"] / sat["makespan_s"]
    rate = args.rate if args.rate > 0 else 0.7 * sat_rate
    arrivals = serving.poisson_arrivals(ids, args.scene_ticks, rate=rate,
                                        seed=args.serving_seed + 1)
    print("bench: saturation %.0f requests/s; serving %d requests at %.0f/s" % (
        sat_rate, len(arrivals), rate), file=sys.stderr, flush=True)
    done = srv.run(arrivals)
    summ = serving.summarize(done, by_id)
    # Algorithmic bytes of the served ticks (as tick_bytes), over the span.
    served_bytes = sum(tick_bytes(r.scene.n, r.scene.n, r.scene.n * r.scene.k, False)
                       for r in done)
    out = {"queries_per_s": summ["queries_per_s"], "unit": "queries/s",
           "p50_latency_ms": summ["p50_latency_ms"], "p99_latency_ms": summ["p99_latency_ms"],
           "requests": summ["requests"], "makespan_s": summ["makespan_s"],
           "rate_per_s": rate, "saturation_requests_per_s": sat_rate,
           "saturation_queries_per_s": sat["queries_per_s"],
           "tick_hbm_frac": served_bytes / summ["makespan_s"] / 1e9 / HBM_PEAK_GBS,
           "scenes": args.scenes, "objects_total": int(sum(s.n for s in scenes)),
           "ticks_per_scene": args.scene_ticks, "slots": args.slots,
           "hbm_budget_gib": args.hbm_budget_gib,
           "admissions": srv.admissions, "evictions": srv.evictions,
           "description": "scene sizes log-uniform in [1e4, 2e6], k in {8, 32}, clustered "
                          "moving objects, Poisson tick requests at 0.7 x the saturation rate "
                          "unless a rate is given; latency from arrival to device completion"}
    srv.close()
    del scenes
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def serving_bench(args):
    """The serving workload alone, printed as its own JSON line."""
    r = run_serving(args)
    out = {"metric": "served k-NN queries/s and tick latency, many scenes, continuous batching",
           "value": r["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "serving_mix", "scenes": r["scenes"],
                      "objects_total": r["objects_total"],
                      "ticks_per_scene": r["ticks_per_scene"], "rate_per_s": r["rate_per_s"],
                      "saturation_requests_per_s": r["saturation_requests_per_s"],
                      "saturation_queries_per_s": r["saturation_queries_per_s"],
                      "slots": r["slots"], "hbm_budget_gib": r["hbm_budget_gib"],
                      "description": r["description"]},
           "p50_latency_ms": r["p50_latency_ms"], "p99_latency_ms": r["p99_latency_ms"],
           "requests": r["requests"], "makespan_s": r["makespan_s"],
           "tick_hbm_frac": r["tick_hbm_frac"],
           "admissions": r["admissions"], "evictions": r["evictions"]}
    print(json.dumps(out), flush=True)


class TimingEvent:
    """A HIP event for timing only: recorded without a system-scope fence,
    so it does not write back caches between the kernels it separates (an
    event with the default flags costs the tick several microseconds)."""
    _hip = None

    def __init__(self):
        import ctypes
        if TimingEvent._hip is None:
            h = ctypes.CDLL("libamdhip64.so")
            vp = ctypes.c_void_p
            h.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(vp), ctypes.c_uint]
            h.hipEventRecord.argtypes = [vp, vp]
            h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), vp, vp]
            h.hipEventDestroy.argtypes = [vp]
            TimingEvent._hip = h
        self._ev = ctypes.c_void_p()
        rc = self._hip.hipEventCreateWithFlags(ctypes.byref(self._ev), 0x20000000)
        if rc != 0:
            raise RuntimeError("hipEventCreateWithFlags failed (%d)" % rc)

    def record(self, stream):
        import ctypes
        rc = self._hip.hipEventRecord(self._ev, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError("hipEventRecord failed (%d)" % rc)

    def elapsed_time(self, end):
        import ctypes
        ms = ctypes.c_float()
        rc = self._hip.hipEventElapsedTime(ctypes.byref(ms), self._ev, end._ev)
        if rc != 0:
            raise RuntimeError("hipEventElapsedTime failed (%d)" % rc)
        return ms.value

    def __del__(self):
        if self._hip is not None and self._ev:
            self._hip.hipEventDestroy(self._ev)


def timed(stream, steps, one_step, streams=None):
    """Run `steps` steps bracketed by synchronisations; per-step device
    latency from timing events on the step's stream (stream, or
    streams[s % len(streams)])."""
    import torch
    starts = [TimingEvent() for _ in range(steps)]
    ends = [TimingEvent() for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        st = streams[s % len(streams)] if streams else stream
        starts[s].record(st)
        one_step(s)
        ends[s].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    return wall, lat


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered_1m")
    ap.add_argument("--ticks", type=int, default=0,
                    help="generate at most this many ticks and cycle over them (0: all, "
                         "but at most 10 for workloads above 2M objects)")
    ap.add_argument("--max-level", type=int, default=0,
                    help="fix the maximum quadtree level 1..16 (0: tuned)")
    ap.add_argument("--leaf-capacity", type=int, default=0,
                    help="fix the leaf capacity (0: tuned)")
    ap.add_argument("--sweep", choices=("lane", "wave", "group"), default=None,
                    help="fix the sweep flavour (default: tuned)")
    ap.add_argument("--group-k", action="store_true",
                    help="fix k grouping on (variable k: each k class with its own list size)")
    ap.add_argument("--autotune", dest="autotune", action="store_true", default=True,
                    help="choose the schedule during warm-up over %s (default)" % (SCHEDULE_SPACE,))
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="use the stored choice for the workload %s" % (TUNED_SCHEDULE,))
    ap.add_argument("--th-candidates", default="",
                    help="comma-separated leaf capacities for the autotuner")
    ap.add_argument("--graph", action="store_true", default=True,
                    help="also replay the ticks as captured HIP graphs (default on)")
    ap.add_argument("--no-graph", dest="graph", action="store_false")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pipeline", dest="pipeline", action="store_false", default=True,
                    help="skip the line with two ticks in flight on two streams")
    ap.add_argument("--no-reuse", dest="reuse", action="store_false", default=True,
                    help="skip the index-reuse line (refit ticks under the rebuild policy)")
    ap.add_argument("--reuse-factor", type=float, default=1.15,
                    help="rebuild when a query takes this factor longer than after the build "
                         "(1.15: best of 1.1, 1.15, 1.3 on clustered_1m)")
    ap.add_argument("--counters", action="store_true",
                    help="also count the query kernel's work (adds atomics; not for timing)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy 5 times (reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    ap.add_argument("--serving", action="store_true",
                    help="serving mode: many scenes, Poisson tick requests, p50/p99 latency")
    ap.add_argument("--scenes", type=int, default=64)
    ap.add_argument("--scene-ticks", type=int, default=8)
    ap.add_argument("--rate", type=float, default=0.0,
                    help="tick requests per second (0: 0.7 x the measured saturation rate)")
    ap.add_argument("--slots", type=int, default=4, help="ticks in flight at most")
    ap.add_argument("--hbm-budget-gib", type=float, default=64.0)
    ap.add_argument("--serving-seed", type=int, default=7)
    ap.add_argument("--tile-queries", type=int, default=0, choices=(0, 8, 16, 32, 64),
                    help="lane flavour queries per wavefront (0: automatic)")
    ap.add_argument("--no-serving", dest="serving_leg", action="store_false", default=True,
                    help="skip the serving leg of the default line")
    args = ap.parse_args()

    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the k-NN tick on a single MI355X "
              "and has no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.serving:
        serving_bench(args)
        return

    import torch
    from paper_1412_6170_amd import binding, workloads

    torch.cuda.set_device(0)
    w = workloads.WORKLOADS[args.workload]()
    n, k = w.n, w.k
    n_ticks = args.ticks or (w.ticks if w.n <= 2_000_000 else min(w.ticks, 10))
    n_ticks = min(n_ticks, w.ticks)
    print("bench: generating %d ticks of %s" % (n_ticks, w.name), file=sys.stderr, flush=True)
    # Per generated tick: device positions, and the device query list when a
    # subset of the objects queries (issuers and per-query k).
    dev, host, queries = [], [], []
    for t in range(n_ticks):
        x, y, iss, ks, _ = w.tick(t)
        host.append((x, y, iss, ks))
        dev.append((torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()))
        if iss is None:
            queries.append((None, None, n, n * k))
        else:
            queries.append((torch.from_numpy(iss).cuda(), torch.from_numpy(ks).cuda(), len(iss),
                            int(np.sum(ks, dtype=np.int64))))
        del x, y
    torch.cuda.synchronize()
    subset = queries[0][0] is not None
    nq_max = max(q[2] for q in queries)
    nq_mean = float(np.mean([q[2] for q in queries]))
    entries_mean = float(np.mean([q[3] for q in queries]))

    def tick_nq(s):
        return queries[s % n_ticks][2]

    def run_query(c, s):
        iss, ks, nq_s, _ = queries[s % n_ticks]
        if iss is None:
            c.query(k=k, nq=nq_s)
        else:
            c.query(issuers=iss, ks=ks)

    stream = torch.cuda.Stream()
    variable_k = queries[0][1] is not None
    sched = dict(TUNED_SCHEDULE.get(w.name, {"leaf_capacity": 0, "max_level": 16,
                                               "sweep": "lane", "group_k": False}))
    if k > 128 and sched["sweep"] == "lane":
        sched["sweep"] = "group"
    space = {dim: list(v) for dim, v in SCHEDULE_SPACE.items()}
    # Levels whose cells would average more than 16 objects of uniformly
    # spread data are not tried (their trials on large workloads are slow).
    space["max_level"] = [lv for lv in space["max_level"] if 4 ** lv * 16 >= n]
    if args.th_candidates:
        space["leaf_capacity"] = [int(v) for v in args.th_candidates.split(",")]
    if k > 128:
        space["sweep"] = ["wave", "group"]
    if not variable_k:
        space["group_k"] = []
    for dim, val in (("leaf_capacity", args.leaf_capacity or None),
                     ("max_level", args.max_level or None), ("sweep", args.sweep),
                     ("group_k", True if args.group_k else None)):
        if val is not None:
            sched[dim] = val
            space[dim] = []
    # Node tables sized for the smallest leaf capacity and the deepest level
    # the autotuner may try.
    th0 = min(space["leaf_capacity"] + [sched["leaf_capacity"] or 10 ** 9])
    l0 = max(space["max_level"] + [sched["max_level"]])
    ctx = binding.Context(n, nq_max, k, leaf_capacity=th0 if th0 < 10 ** 9 else 0, k_hint=k,
                          max_level=l0, stream=stream.cuda_stream, timing=True,
                          counters=args.counters)
    if args.tile_queries:
        sched["tile_queries"] = args.tile_queries
    ctx.set_schedule(**{d: v for d, v in sched.items() if not (d == "leaf_capacity" and not v)})

    def step(s):
        x, y = dev[s % n_ticks]
        ctx.load_positions(x, y)
        ctx.advance_tick()
        run_query(ctx, s)

    with torch.cuda.stream(stream):
        tune = None
        if args.autotune and any(space.values()):
            best, times = binding.autotune_schedule(
                ctx, step, space["leaf_capacity"], max_levels=space["max_level"],
                sweeps=space["sweep"], group_k=space["group_k"], repeats=3, rounds=2,
                finalists=4, final_repeats=8)
            tune = {"chosen": best, "device_ms_per_tick": times}
            print("bench: autotuned schedule %s" % (best,), file=sys.stderr, flush=True)
        sched = ctx.schedule()
        for s in range(args.warmup):
            step(s)
        ctx.sync()
        ctx.reset_timing()
        print("bench: timing %d steps" % args.steps, file=sys.stderr, flush=True)
        wall, lat = timed(stream, args.steps, step)
        ctx.sync()
        st = ctx.stats()

    total_q = sum(tick_nq(s) for s in range(args.steps))
    value = total_q / wall
    kern_ms = st["ms_query_main_mean"]
    kern_bytes = query_kernel_bytes(n, nq_mean, entries_mean)
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
        "config": {"workload": w.name, "objects": n, "queries_per_tick": nq_mean,
                   "k": k if not subset else "per query, mean %.1f" % (entries_mean / nq_mean),
                   "ticks": w.ticks, "ticks_generated": n_ticks,
                   "leaf_capacity": st["leaf_capacity"], "max_level": sched["max_level"],
                   "sweep": sched["sweep"], "group_k": sched["group_k"],
                   "description": w.description},
        "p50_tick_ms": float(np.percentile(lat, 50)),
        "p99_tick_ms": float(np.percentile(lat, 99)),
        "device_ms_build_mean": st["ms_build_mean"],
        "device_ms_query_mean": st["ms_query_mean"],
        "tick_hbm_frac": tick_bytes(n, nq_mean, entries_mean, subset) / (tick_ms * 1e-3) / 1e9
        / HBM_PEAK_GBS,
        "leaves": st["leaves"],
        "deepest_level": st["deepest_level"],
        "autotune": tune,
        "roofline": roofline_entry(w.name, st["leaf_capacity"], sched["max_level"], k, kern_ms,
                                   kern_bytes, sched["sweep"]),
        "graph": None,
        "cpu_baseline": None,
    }
    if args.counters and st["wavefronts"]:
        wf = st["wavefronts"]
        out["per_wavefront"] = {"candidate_steps": st["wave_candidate_steps"] / wf,
                                "merges": st["wave_merges"] / wf,
                                "node_visits": st["wave_node_visits"] / wf,
                                "leaf_sweeps": st["wave_leaf_sweeps"] / wf}
    ctx.close()

    def scheduled_context(strm, timing=False):
        """A context for another leg of the benchmark, with the schedule
        the timed ticks ran with."""
        c = binding.Context(n, nq_max, k, leaf_capacity=sched["leaf_capacity"],
                            max_level=sched["max_level"], k_hint=k, stream=strm.cuda_stream,
                            timing=timing)
        c.set_schedule(**sched)
        return c

    if args.graph:
        # The same ticks, each captured once as a HIP graph (one graph per
        # tick's input buffers) and replayed; no timing events inside.
        gctx = scheduled_context(stream)

        def gstep(s):
            x, y = dev[s % n_ticks]
            gctx.load_positions(x, y)
            gctx.advance_tick()
            run_query(gctx, s)

        with torch.cuda.stream(stream):
            gstep(0)
            gctx.sync()
            graphs = []
            for t in range(n_ticks):
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=stream):
                    gstep(t)
                graphs.append(g)
            for s in range(args.warmup):
                graphs[s % n_ticks].replay()
            gwall, glat = timed(stream, args.steps, lambda s: graphs[s % n_ticks].replay())
        out["graph"] = {"value": total_q / gwall, "unit": "queries/s",
                        "ms_per_step": gwall * 1e3 / args.steps,
                        "p50_tick_ms": float(np.percentile(glat, 50)),
                        "p99_tick_ms": float(np.percentile(glat, 99))}
        del graphs
        gctx.close()

    if args.pipeline:
        # Two ticks in flight: tick s runs (build + query) on stream s % 2
        # with its own context, so a tick's index build overlaps the previous
        # tick's query.  Every tick still builds its index and answers all
        # queries.
        pstreams = [torch.cuda.Stream(), torch.cuda.Stream()]  # default priority
        pctx = [scheduled_context(ps) for ps in pstreams]

        def pstep(s):
            c = pctx[s % 2]
            x, y = dev[s % n_ticks]
            c.load_positions(x, y)
            c.advance_tick()
            with torch.cuda.stream(pstreams[s % 2]):
                run_query(c, s)

        for s in range(args.warmup):
            pstep(s)
        torch.cuda.synchronize()
        pwall, plat = timed(None, args.steps, pstep, streams=pstreams)
        out["pipelined"] = {"value": total_q / pwall, "unit": "queries/s",
                            "ms_per_step": pwall * 1e3 / args.steps,
                            "p50_tick_ms": float(np.percentile(plat, 50)),
                            "p99_tick_ms": float(np.percentile(plat, 99)),
                            "ticks_in_flight": 2}
        for c in pctx:
            c.close()

    if args.reuse:
        # The same ticks with index reuse (Sec. 4.1): refit ticks while
        # queries stay within reuse_factor of the query after the last full
        # build, else rebuild.  The policy reads the device time of the
        # query two ticks back (waiting for it alone keeps the host two
        # ticks ahead and the GPU busy).
        rctx = scheduled_context(stream, timing=True)
        pol = binding.ReusePolicy(factor=args.reuse_factor)

        def rstep(s):
            x, y = dev[s % n_ticks]
            pol.tick(rctx, x, y)
            run_query(rctx, s)

        with torch.cuda.stream(stream):
            for s in range(args.warmup):
                rstep(s)
            pol.rebuilds = pol.refits = 0
            rwall, rlat = timed(stream, args.steps, rstep)
        out["reuse"] = {"value": total_q / rwall, "unit": "queries/s",
                        "ms_per_step": rwall * 1e3 / args.steps,
                        "p50_tick_ms": float(np.percentile(rlat, 50)),
                        "p99_tick_ms": float(np.percentile(rlat, 99)),
                        "rebuilds": pol.rebuilds, "refits": pol.refits,
                        "factor": args.reuse_factor}
        rctx.close()

    if args.serving_leg and args.workload == "clustered_1m":
        # The served form of the same path: many scenes (up to 2M objects,
        # k in {8, 32}) under continuous batching.
        out["serving"] = run_serving(args)

    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        cb = cpu_baseline(w, host)
        cb["gpu_over_cpu_all_cores"] = value / cb["value"]
        cb["gpu_over_cpu_1thread"] = value / cb["value_1thread"]
        cb["paper_context"] = ("10x-20x speed-up of the paper's GPU pipeline over a sequential "
                               "1-core CPU k-NN (FLANN kd-tree), NVIDIA GTX 580 vs Intel "
                               "i7-2600 @ 3.4 GHz (Sec. 6)")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
