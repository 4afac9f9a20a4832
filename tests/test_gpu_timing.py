"""GPU: per-phase device times (MKNN_FLAG_TIMING).  The build, the whole
query and its leaf-sweep kernel are timed from HIP events on the context's
stream; the statistics must be positive, ordered (the kernel is part of the
query) and averaged over exactly the ticks since the last reset.  Results
with timing on are the same as with timing off."""
import numpy as np
import pytest

from paper_1412_6170_amd import binding, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    yield


def say(*a):
    print(*a, flush=True)


def run(ctx, x, y, k, issuers=None, ks=None):
    ctx.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    ctx.advance_tick()
    if issuers is None:
        ctx.query(k=k, nq=len(x))
    else:
        ctx.query(issuers=torch.from_numpy(issuers).cuda(),
                  ks=None if ks is None else torch.from_numpy(ks).cuda())
    return ctx.fetch()


@pytest.mark.parametrize("subset", [False, True])
def test_times_positive_ordered_and_counted(subset):
    w = workloads.clustered_1m(n=100_000, ticks=5)
    k = 16
    n = w.n
    rng = np.random.default_rng(5)
    say("timing: subset=%s n=%d" % (subset, n))
    with binding.Context(n, n, k, timing=True) as ct, binding.Context(n, n, k) as cp:
        ct.reset_timing()
        for t in range(5):
            x, y, _, _, _ = w.tick(t)
            iss = ks = None
            if subset:
                iss = rng.permutation(n)[: n // 3].astype(np.int32)
                ks = rng.integers(1, k + 1, len(iss)).astype(np.int32)
            a = run(ct, x, y, k, iss, ks)
            b = run(cp, x, y, k, iss, ks)
            for u, v in zip(a, b):
                if u is not None:
                    assert np.array_equal(np.asarray(u).view(np.uint8), np.asarray(v).view(np.uint8))
        ct.sync()
        st = ct.stats()
        say(st)
        assert st["timed_ticks"] == 5
        assert st["ms_build"] > 0 and st["ms_query"] > 0 and st["ms_query_main"] > 0
        assert st["ms_query_main"] <= st["ms_query"]
        assert st["ms_build_mean"] > 0 and st["ms_query_mean"] > 0
        assert 0 < st["ms_query_main_mean"] <= st["ms_query_mean"]
        if subset:
            # Query preparation (sort by position, row offsets) runs before
            # the kernel, so the kernel is strictly part of the query.
            assert st["ms_query_main"] < st["ms_query"]
        ct.reset_timing()
        x, y, _, _, _ = w.tick(0)
        run(ct, x, y, k)
        ct.sync()
        assert ct.stats()["timed_ticks"] == 1


def test_timing_off_reports_zero():
    w = workloads.uniform_10k()
    x, y, _, _, k = w.tick(0)
    with binding.Context(len(x), len(x), k) as c:
        run(c, x, y, k)
        c.sync()
        st = c.stats()
        assert st["ms_build"] == 0 and st["ms_query_main"] == 0 and st["timed_ticks"] == 0


def test_query_time_without_waiting():
    w = workloads.uniform_10k()
    x, y, _, _, k = w.tick(0)
    with binding.Context(len(x), len(x), k, timing=True) as c:
        for _ in range(3):
            run(c, x, y, k)
        c.sync()
        st = c.stats()
        last = c.query_time(0)
        assert last == st["ms_query"] and last > 0
        assert c.query_time(1) > 0 and c.query_time(2) > 0
        with pytest.raises(binding.MknnError):
            c.query_time(3)      # only three queries so far
    with binding.Context(len(x), len(x), k) as c:
        run(c, x, y, k)
        c.sync()
        with pytest.raises(binding.MknnError):
            c.query_time(0)      # timing off


def test_work_counters_and_node_count():
    """MKNN_FLAG_COUNTERS: per query, one count per wavefront (64 queries
    each with 64-query tiles; 8 each with the automatic tiles of a launch
    this small), at least one leaf swept and one candidate per wavefront,
    totals that restart with reset_timing, and results bit-equal to a
    context without counters.  The node count equals the number of distinct
    quadrants on the paths from the root to every leaf of the oracle's
    index."""
    from tests.helpers import family
    import oracle
    x, y = family("clustered", 30000, 48)
    n, k, th, L = len(x), 16, 32, 16
    exp = oracle.build_index(x, y, th, L)
    quads = set()
    for lev, pre in zip(exp["leaf_level"].tolist(), exp["leaf_prefix"].tolist()):
        for l in range(lev + 1):
            quads.add((l, pre >> (2 * (lev - l))))
    with binding.Context(n, n, k, leaf_capacity=th, max_level=L, counters=True) as c, \
            binding.Context(n, n, k, leaf_capacity=th, max_level=L) as p:
        c.set_schedule(tile_queries=64)
        rows = []
        for ctx in (c, p):
            run(ctx, x, y, k)
            rows.append(ctx.fetch())
        for u, v in zip(rows[0][:3], rows[1][:3]):
            assert np.array_equal(np.asarray(u).view(np.uint8), np.asarray(v).view(np.uint8))
        st = c.stats()
        say(st)
        waves = -(-n // 64)
        assert st["nodes"] == len(quads)
        assert st["nq"] == n
        assert st["wavefronts"] == waves
        assert st["wave_leaf_sweeps"] >= waves and st["wave_candidate_steps"] >= waves
        assert st["wave_node_visits"] > 0 and st["wave_merges"] >= waves
        c.reset_timing()
        issuers = np.arange(0, n, 3, dtype=np.int32)
        c.query(k=k, issuers=torch.from_numpy(issuers).cuda())
        c.sync()
        assert c.stats()["wavefronts"] == -(-len(issuers) // 64)
        # Automatic tiles: 30,000 queries fit the GPU's resident wavefronts
        # in one round even at 8 queries per wavefront.
        c.set_schedule(tile_queries=0)
        c.reset_timing()
        c.query(k=k)
        assert_same = [np.asarray(a).view(np.uint8) for a in c.fetch()[:3]]
        for u, v in zip(assert_same, rows[1][:3]):
            assert np.array_equal(u, np.asarray(v).view(np.uint8))
        assert c.stats()["wavefronts"] == -(-n // 8)
