"""Serving many independent scenes with continuous batching.

Each scene is a set of moving objects with its own k; a request asks for
one tick of one scene (its positions are already on the device).  The
server keeps scenes resident -- one library context per scene, holding the
scene's snapshot, quadtree and results -- and admits a scene only while
the sum of resident footprints (``mknn_footprint``) stays within an HBM
budget; an idle resident scene is evicted (least recently used) to make
room.  Requests are taken as they arrive: whenever a slot (a bound on ticks
in flight) is free and the scene is resident and idle, the tick is enqueued
on the scene's own stream, so ticks of different scenes overlap on the
device.  Latency is measured from a request's arrival to the completion of
its tick on the device (the paper's tick latency, Sec. 2.2: queueing plus
processing time).

Host-side scheduling only; every tick runs entirely in the HIP library.
"""
import collections
import time

import numpy as np

from . import binding


class Scene:
    def __init__(self, sid, positions, k, leaf_capacity=0, max_level=0, tile_queries=0):
        """positions: list of (x, y) device tensors, one per tick; they
        stay unchanged while the scene is served.  leaf_capacity, max_level
        and tile_queries tune the scene's index and query (0: the library's
        defaults); results never depend on them."""
        self.sid = sid
        self.positions = positions
        self.n = int(positions[0][0].numel())
        self.k = int(k)
        self.leaf_capacity = int(leaf_capacity)
        self.max_level = int(max_level)
        self.tile_queries = int(tile_queries)
        self.ctx = None
        self.stream = None
        self.busy = False
        self.last_used = 0.0
        self.footprint = binding.footprint(n_max=self.n, k_max=self.k,
                                           leaf_capacity=leaf_capacity, max_level=max_level)


class Request:
    __slots__ = ("scene", "tick", "arrival", "start", "done", "event")

    def __init__(self, scene, tick, arrival):
        self.scene = scene
        self.tick = tick
        self.arrival = arrival
        self.start = None
        self.done = None
        self.event = None


class Server:
    def __init__(self, scenes, hbm_budget, slots=8, on_complete=None):
        import torch
        self.torch = torch
        self.scenes = {s.sid: s for s in scenes}
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.resident = 0
        self.on_complete = on_complete
        self.admissions = 0
        self.evictions = 0
        for s in scenes:
            if s.footprint > self.budget:
                raise ValueError("scene %s needs %d bytes, above the budget" % (s.sid, s.footprint))

    # -- residency -----------------------------------------------------------
    def _admit(self, scene, now):
        if scene.ctx is not None:
            return True
        while self.resident + scene.footprint > self.budget:
            idle = [s for s in self.scenes.values() if s.ctx is not None and not s.busy]
            if not idle:
                return False
            victim = min(idle, key=lambda s: s.last_used)
            victim.ctx.close()
            victim.ctx = None
            victim.stream = None
            self.resident -= victim.footprint
            self.evictions += 1
        scene.stream = self.torch.cuda.Stream()   # default priority
        scene.ctx = binding.Context(scene.n, scene.n, scene.k,
                                    leaf_capacity=scene.leaf_capacity,
                                    max_level=scene.max_level, stream=scene.stream)
        if scene.tile_queries:
            scene.ctx.set_schedule(tile_queries=scene.tile_queries)
        self.resident += scene.footprint
        self.admissions += 1
        return True

    def _launch(self, req, now):
        sc = req.scene
        x, y = sc.positions[req.tick % len(sc.positions)]
        # Positions are complete (run() synchronised before serving), so the
        # tick is enqueued from the scene's own stream: the binding has no
        # other stream to order it after.
        with self.torch.cuda.stream(sc.stream):
            sc.ctx.load_positions(x, y)
            sc.ctx.advance_tick()
            sc.ctx.query(k=sc.k, nq=sc.n)
        ev = self.torch.cuda.Event()
        ev.record(sc.stream)
        req.event = ev
        req.start = now
        sc.busy = True
        sc.last_used = now

    # -- the loop ------------------------------------------------------------
    def run(self, arrivals):
        """arrivals: list of (t_seconds, scene_id, tick), t relative to the
        start.  Returns the completed requests in completion order."""
        arrivals = sorted(arrivals, key=lambda a: a[0])
        # Scene positions may still be being written by earlier work on any
        # stream: finish it once, so that ticks can be enqueued from the
        # scenes' own streams with nothing else to wait for.
        self.torch.cuda.synchronize()
        pending = collections.deque()
        inflight = []
        done = []
        t0 = time.perf_counter()
        i = 0
        while i < len(arrivals) or pending or inflight:
            now = time.perf_counter() - t0
            while i < len(arrivals) and arrivals[i][0] <= now:
                a = arrivals[i]
                pending.append(Request(self.scenes[a[1]], a[2], a[0]))
                i += 1
            # completions
            still = []
            for r in inflight:
                if r.event.query():
                    r.done = time.perf_counter() - t0
                    r.scene.busy = False
                    done.append(r)
                    if self.on_complete:
                        self.on_complete(r)
                else:
                    still.append(r)
            inflight = still
            # admissions: first come first served among requests whose scene
            # is idle; a request that cannot be admitted waits in place.
            if len(inflight) < self.slots and pending:
                kept = collections.deque()
                while pending:
                    r = pending.popleft()
                    if len(inflight) < self.slots and not r.scene.busy and self._admit(r.scene, now):
                        self._launch(r, now)
                        inflight.append(r)
                    else:
                        kept.append(r)
                pending = kept
            if not inflight and not pending and i < len(arrivals):
                wait = arrivals[i][0] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        return done

    def close(self):
        for s in self.scenes.values():
            if s.ctx is not None:
                s.ctx.close()
                s.ctx = None
        self.resident = 0


def poisson_arrivals(scene_ids, ticks_per_scene, rate, seed):
    """Tick requests of every scene (ticks in order) at Poisson-distributed
    times with the given aggregate rate (requests per second)."""
    rng = np.random.default_rng(seed)
    order = []
    left = {s: ticks_per_scene for s in scene_ids}
    nxt = {s: 0 for s in scene_ids}
    total = len(scene_ids) * ticks_per_scene
    t = 0.0
    for _ in range(total):
        t += rng.exponential(1.0 / rate)
        choices = [s for s in scene_ids if left[s] > 0]
        s = choices[int(rng.integers(0, len(choices)))]
        order.append((t, s, nxt[s]))
        nxt[s] += 1
        left[s] -= 1
    return order


def summarize(done, scenes):
    lat = np.array([r.done - r.arrival for r in done])
    queries = sum(scenes[r.scene.sid].n for r in done)
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return {"requests": len(done), "queries": int(queries),
            "queries_per_s": queries / span if span > 0 else None,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "makespan_s": span}
