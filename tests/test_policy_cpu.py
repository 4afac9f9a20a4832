"""CPU: the index-reuse policy's decisions, on a scripted context (no GPU).
It refits from the second tick on, keeps refitting while the query two
ticks back stays within the factor of the query of the last full build,
rebuilds when it does not, after max_refits refits in a row or when the
object count changes, and never waits for the last query (which would
leave the GPU idle).  Also the autotuner's finalists stage."""
import pytest

from paper_1412_6170_amd import binding


class ScriptedContext:
    """Stands in for binding.Context: query times by tick, None = running."""

    def __init__(self, times):
        self.times = times
        self.ticks = 0
        self.asked = []

    def query_time(self, back=0, wait=False):
        q = self.ticks - 1 - back
        self.asked.append(q)
        assert back >= 1, "waiting for the last query would idle the GPU"
        return self.times.get(q)

    def load_positions(self, x, y):
        pass

    def refit_tick(self):
        self.ticks += 1

    def advance_tick(self):
        self.ticks += 1


POS = [0.5] * 10   # ten objects; the scripted context ignores positions


def run(times, n, **kw):
    ctx = ScriptedContext(times)
    pol = binding.ReusePolicy(**kw)
    kinds = [pol.tick(ctx, POS, POS) for _ in range(n)]
    return kinds, ctx, pol


def test_refits_while_queries_stay_within_the_factor():
    kinds, ctx, pol = run({i: 1.0 for i in range(10)}, 8, factor=1.3)
    assert kinds == ["build"] + ["refit"] * 7
    assert pol.reference == 1.0 and pol.rebuilds == 1 and pol.refits == 7
    assert all(q >= 0 for q in ctx.asked)


def test_rebuilds_when_the_query_two_ticks_back_grew():
    # Tick 0 builds (1.0 ms); ticks 1.. refit and slow down; tick 3's
    # query (2.0 ms) is seen at tick 5, which rebuilds; its query (1.0 ms,
    # seen at tick 7) becomes the new reference.
    times = {0: 1.0, 1: 1.1, 2: 1.2, 3: 2.0, 4: 2.1, 5: 1.0, 6: 1.1, 7: 1.1}
    kinds, ctx, pol = run(times, 8, factor=1.5)
    assert kinds == ["build", "refit", "refit", "refit", "refit", "build", "refit", "refit"]
    assert pol.reference == 1.0


def test_unfinished_queries_keep_the_last_decision_basis():
    times = {0: 1.0, 1: None, 2: None, 3: None}
    kinds, ctx, pol = run(times, 5, factor=1.3)
    assert kinds == ["build"] + ["refit"] * 4


def test_max_refits_in_a_row():
    kinds, ctx, pol = run({i: 1.0 for i in range(12)}, 9, factor=10.0, max_refits=3)
    assert kinds == ["build", "refit", "refit", "refit", "build", "refit", "refit", "refit",
                     "build"]


def test_a_new_object_count_rebuilds():
    ctx = ScriptedContext({i: 1.0 for i in range(10)})
    pol = binding.ReusePolicy(factor=10.0)
    sizes = [10, 10, 10, 12, 12, 9, 9]
    kinds = [pol.tick(ctx, [0.5] * m, [0.5] * m) for m in sizes]
    assert kinds == ["build", "refit", "refit", "build", "refit", "build", "refit"]


class _TunedCtx:
    """A context whose timings are scripted per leaf capacity: the first
    timing of a setting may be off (noise), later ones are its true cost."""

    def __init__(self, first, true):
        self.sched = {"leaf_capacity": 16, "max_level": 12, "sweep": "lane", "group_k": False,
                      "tile_queries": 0}
        self.first, self.true, self.seen = first, true, set()

    def schedule(self):
        return dict(self.sched)

    def set_schedule(self, **kw):
        self.sched.update(kw)

    def sync(self):
        pass

    def reset_timing(self):
        pass

    def stats(self):
        th = self.sched["leaf_capacity"]
        ms = self.first.get(th, self.true[th]) if th not in self.seen else self.true[th]
        self.seen.add(th)
        return {"ms_build_mean": 0.0, "ms_query_mean": ms}


def test_autotune_finalists_retime_the_fastest_settings():
    """One noisy timing makes leaf capacity 48 look fastest; coordinate
    descent alone keeps it, the finalists stage times the fastest settings
    again and picks 32, the fastest on average."""
    true = {16: 1.00, 32: 0.90, 48: 0.95}
    first = {48: 0.80}
    best, _ = binding.autotune_schedule(_TunedCtx(first, true), lambda i: None, (16, 32, 48))
    assert best["leaf_capacity"] == 48
    best, times = binding.autotune_schedule(_TunedCtx(first, true), lambda i: None, (16, 32, 48),
                                            finalists=2, final_repeats=2)
    assert best["leaf_capacity"] == 32
    means = {dict(p.split("=") for p in key.split(", "))["leaf_capacity"]: v
             for key, v in times.items()}
    assert means["32"] == pytest.approx(0.90) and means["48"] == pytest.approx(0.95)
