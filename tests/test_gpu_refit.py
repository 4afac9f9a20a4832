"""GPU: index reuse across ticks (refit ticks).  The objects keep the last
full build's order, leaves and node tables; each leaf's box becomes the
bounding box of its objects' current positions, queries prune inner nodes
with boxes grown by the objects' drift, and must still return exactly the
oracle's answer on the current positions."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding, workloads
from tests.helpers import family, f32

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


def same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


def check(got, exp):
    assert np.array_equal(got[2], exp[2])
    assert np.array_equal(got[0], exp[0]) and same_bits(got[1], exp[1])


@pytest.mark.parametrize("L", [16, 12])
def test_refit_ticks_moving_clusters(L):
    w = workloads.clustered_1m(n=200_000, ticks=6)
    k = 32
    with binding.Context(w.n, w.n, k, leaf_capacity=32, max_level=L) as c:
        for t in range(w.ticks):
            x, y, _, _, _ = w.tick(t)
            say("refit clustered_200k L=%d tick %d" % (L, t))
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            if t == 0:
                c.advance_tick()
            else:
                c.refit_tick()
            c.query(k=k)
            got = c.fetch()
            st = c.stats()
            assert st["refits"] == t
            assert (st["drift"] > 0) == (t > 0)
            check(got, oracle.knn(x, y, k=k, th=32, threads=16))


@pytest.mark.parametrize("sweep,k", [("lane", 24), ("group", 64), ("wave", 40)])
def test_refit_every_sweep_flavour(sweep, k):
    """Refit ticks with each sweep flavour: leaf boxes are the bounding boxes
    of the objects' current positions, inner boxes the build's quadrants
    grown by the drift.  Objects drift over several ticks (leaves spread
    past their quadrants); all queries, a subset and free centres each
    match brute force."""
    w = workloads.clustered_1m(n=20_000, ticks=5)
    rng = np.random.default_rng(11)
    with binding.Context(w.n, w.n, k, leaf_capacity=16, max_level=14) as c:
        c.set_schedule(sweep=sweep)
        for t in range(w.ticks):
            x, y, _, _, _ = w.tick(t)
            say("refit every flavour: %s k=%d tick %d" % (sweep, k, t))
            c.load_positions(x, y)
            if t == 0:
                c.advance_tick()
            else:
                c.refit_tick()
            c.query(k=k)
            check(c.fetch(), oracle.brute_knn(x, y, k=k, threads=16))
            iss = rng.integers(0, w.n, 1500).astype(np.int32)
            c.query(issuers=iss, k=k)
            check(c.fetch(), oracle.brute_knn(x, y, issuers=iss, k=k, threads=16))
            qx = rng.random(1000, dtype=np.float32)
            qy = rng.random(1000, dtype=np.float32)
            c.query_points(qx, qy, k=k)
            check(c.fetch(), oracle.brute_knn_points(x, y, qx, qy, k=k, threads=16))
        assert c.stats()["refits"] == w.ticks - 1


def test_refit_after_large_moves_and_all_query_kinds():
    x0, y0 = family("clustered", 20_000, 3)
    rng = np.random.default_rng(5)
    with binding.Context(len(x0), len(x0), 24, leaf_capacity=16) as c:
        c.load_positions(x0, y0)
        c.advance_tick()
        for step in range(3):
            # A tenth of the objects jump anywhere; the rest jitter.
            x, y = x0.copy(), y0.copy()
            jump = rng.random(len(x)) < 0.1
            x[jump] = rng.random(jump.sum(), dtype=np.float32)
            y[jump] = rng.random(jump.sum(), dtype=np.float32)
            x = f32(np.clip(x + rng.uniform(-1e-3, 1e-3, len(x)), 0, 1 - 2 ** -24))
            y = f32(np.clip(y + rng.uniform(-1e-3, 1e-3, len(y)), 0, 1 - 2 ** -24))
            say("refit large moves step %d" % step)
            c.load_positions(x, y)
            c.refit_tick()
            c.query(k=24)
            check(c.fetch(), oracle.brute_knn(x, y, k=24, threads=16))
            iss = rng.integers(0, len(x), 3000).astype(np.int32)
            ks = rng.integers(1, 25, 3000).astype(np.int32)
            c.query(issuers=iss, ks=ks)
            g = c.fetch()
            e = oracle.brute_knn(x, y, issuers=iss, ks=ks, threads=16)
            assert np.array_equal(g[3], e[3])
            check(g, e)
            qx = rng.random(2000, dtype=np.float32)
            qy = rng.random(2000, dtype=np.float32)
            c.query_points(qx, qy, k=7)
            check(c.fetch(), oracle.brute_knn_points(x, y, qx, qy, k=7, threads=16))


def test_refit_state_errors():
    x, y = family("uniform", 300, 1)
    with binding.Context(400, 400, 8) as c:
        c.load_positions(x, y)
        with pytest.raises(binding.MknnError) as e:
            c.refit_tick()
        assert e.value.code == -3
        c.advance_tick()
        c.load_positions(f32(np.append(x, 0.5)), f32(np.append(y, 0.5)))
        with pytest.raises(binding.MknnError) as e:
            c.refit_tick()
        assert e.value.code == -3
        c.load_positions(x, y)
        c.refit_tick()
        c.query(k=8)
        check(c.fetch(), oracle.brute_knn(x, y, k=8))


def test_reuse_policy_stays_exact():
    w = workloads.clustered_1m(n=100_000, ticks=8)
    pol = binding.ReusePolicy(factor=1.5)
    kinds = []
    with binding.Context(w.n, w.n, 16, leaf_capacity=16, timing=True) as c:
        for t in range(w.ticks):
            x, y, _, _, _ = w.tick(t)
            kinds.append(pol.tick(c, x, y))
            c.query(k=16)
            check(c.fetch(), oracle.knn(x, y, k=16, th=16, threads=16))
    say("policy ticks:", kinds)
    assert kinds[0] == "build" and "refit" in kinds


def jittered(x0, y0, rng, amp):
    x = f32(np.clip(x0 + rng.uniform(-amp, amp, len(x0)), 0, 1 - 2 ** -24))
    y = f32(np.clip(y0 + rng.uniform(-amp, amp, len(y0)), 0, 1 - 2 ** -24))
    return x, y


def test_refit_across_epoch_wrap():
    """Refit ticks whose tags cross the wrap from 2^24 - 1 to 1: the drift of
    each refit must be the one its queries use (a refit that lost its drift
    to a larger word of an earlier epoch would prune with unpadded boxes)."""
    x0, y0 = family("clustered", 20_000, 71)
    rng = np.random.default_rng(72)
    k = 16
    with binding.Context(len(x0), len(x0), k, leaf_capacity=16) as c:
        c.set_epochs(2 ** 24 - 3, 2 ** 24 - 2)
        c.load_positions(x0, y0)
        c.advance_tick()
        for step in range(5):
            x, y = jittered(x0, y0, rng, 3e-3 * (5 - step))
            say("refit across the epoch wrap, step %d" % step)
            c.load_positions(x, y)
            c.refit_tick()
            c.query(k=k)
            check(c.fetch(), oracle.brute_knn(x, y, k=k, threads=16))
            assert c.stats()["drift"] > 0


def test_refit_graphs_replayed_out_of_order():
    """Refit ticks captured as graphs and replayed in another order than
    captured, with eager ticks between: every replay is exact."""
    x0, y0 = family("clustered", 30_000, 73)
    rng = np.random.default_rng(74)
    k = 12
    pos = [jittered(x0, y0, rng, amp) for amp in (4e-3, 1e-3, 2e-3)]
    exp = [oracle.brute_knn(x, y, k=k, threads=16) for x, y in pos]
    dev = [(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()) for x, y in pos]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c = binding.Context(len(x0), len(x0), k, leaf_capacity=16, stream=s.cuda_stream)
        d0 = (torch.from_numpy(x0).cuda(), torch.from_numpy(y0).cuda())
        c.load_positions(*d0)
        c.advance_tick()
        c.query(k=k)
        c.sync()
        graphs = []
        for t in range(len(pos)):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                c.load_positions(*dev[t])
                c.refit_tick()
                c.query(k=k)
            graphs.append(g)
        for t in (2, 0, 1, 2, 1, 0):
            say("replay refit graph %d" % t)
            graphs[t].replay()
            check(c.fetch(), exp[t])
            # An eager refit tick between replays (later tags than every graph).
            c.load_positions(*dev[(t + 1) % len(pos)])
            c.refit_tick()
            c.query(k=k)
            check(c.fetch(), exp[(t + 1) % len(pos)])
        del graphs
        c.close()
