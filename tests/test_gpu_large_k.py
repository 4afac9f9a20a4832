"""GPU parity of the one-query-per-wavefront sweep ("coalesced writes",
Sec. 4.2.1): lists up to k = 1024, and the same flavour at small k, bit for
bit against the oracle (brute force, Definition 1) through the C ABI.
Also the schedule calls that switch flavour, leaf capacity and maximum
level between ticks."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding, workloads
from tests.helpers import FAMILIES, check_invariants, check_rows_vectorized, f32, family
from tests.test_gpu_parity import assert_rows_equal, same, same_bits, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    yield


def run(x, y, k=None, issuers=None, ks=None, th=0, L=0, k_max=None, wave=False,
        device_inputs=False):
    n = len(x)
    nq = n if issuers is None else len(issuers)
    if k_max is None:
        k_max = int(k) if ks is None else int(np.max(ks))
    with binding.Context(max(n, 1), max(nq, 1), k_max, leaf_capacity=th, max_level=L,
                         sweep_wave=wave) as c:
        if device_inputs:
            c.load_positions(torch.from_numpy(f32(x)).cuda(), torch.from_numpy(f32(y)).cuda())
            iss = None if issuers is None else torch.from_numpy(np.asarray(issuers, np.int32)).cuda()
            kk = None if ks is None else torch.from_numpy(np.asarray(ks, np.int32)).cuda()
        else:
            c.load_positions(x, y)
            iss, kk = issuers, ks
        c.advance_tick()
        c.query(k=k, issuers=iss, ks=kk, nq=nq)
        return c.fetch()


@pytest.mark.parametrize("kind", FAMILIES)
def test_large_k_families(kind):
    x, y = family(kind, 3000, 61)
    for k in (129, 256, 300, 512, 1024):
        exp = oracle.brute_knn(x, y, k=k, threads=16)
        for th in (7, 64, 2048):
            say("%s k=%d th=%d" % (kind, k, th))
            assert_rows_equal(run(x, y, k=k, th=th), exp, "%s k=%d th=%d" % (kind, k, th))


@pytest.mark.parametrize("kind", FAMILIES)
def test_wave_flavour_small_k(kind):
    x, y = family(kind, 2500, 62)
    for k in (1, 8, 13, 32, 64, 65, 128):
        exp = oracle.brute_knn(x, y, k=k, threads=16)
        for th in (1, 64, 1000):
            say("wave %s k=%d th=%d" % (kind, k, th))
            assert_rows_equal(run(x, y, k=k, th=th, wave=True), exp,
                              "wave %s k=%d th=%d" % (kind, k, th))


@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 300, 1030])
def test_large_k_beyond_n(n):
    x, y = family("uniform", n, 63)
    # k at and past the n - 1 others, within the 1024 limit.
    for k in sorted({min(v, 1024) for v in (1, max(1, n - 1), n, n + 5, 1024)}):
        exp = oracle.brute_knn(x, y, k=k)
        for L in (16, 12):
            say("n=%d k=%d L=%d" % (n, k, L))
            assert_rows_equal(run(x, y, k=k, th=4, L=L, wave=True), exp,
                              "n=%d k=%d L=%d" % (n, k, L))


def test_large_k_ties_duplicates_denormals():
    side = 48
    iy, ix = np.divmod(np.arange(side * side), side)
    x = (ix * 2.0 ** -6).astype(np.float32)
    y = (iy * 2.0 ** -6).astype(np.float32)
    for k in (200, 700):
        say("lattice k=%d" % k)
        assert_rows_equal(run(x, y, k=k, th=10), oracle.brute_knn(x, y, k=k, threads=16))
    # Every object at one point: the k smallest other ids, d2 = 0.
    x = np.full(1500, 0.375, np.float32)
    y = np.full(1500, 0.625, np.float32)
    got = run(x, y, k=1024, th=3)
    assert_rows_equal(got, oracle.brute_knn(x, y, k=1024, threads=16))
    assert got[0][7].tolist() == [i for i in range(1025) if i != 7]
    # Denormal distances rank.
    x = (np.arange(400) * 2.0 ** -80).astype(np.float32)
    y = np.zeros(400, np.float32)
    got = run(x, y, k=300, th=5)
    assert_rows_equal(got, oracle.brute_knn(x, y, k=300))


@pytest.mark.parametrize("device_inputs", [False, True])
def test_large_variable_k_subset(device_inputs):
    x, y = family("clustered", 6000, 64)
    rng = np.random.default_rng(65)
    iss = rng.choice(len(x), 2500, replace=False).astype(np.int32)
    ks = rng.choice([1, 7, 64, 129, 500, 1024], 2500).astype(np.int32)
    exp = oracle.brute_knn(x, y, issuers=iss, ks=ks, threads=16)
    got = run(x, y, issuers=iss, ks=ks, th=48, k_max=1024, device_inputs=device_inputs)
    assert_rows_equal(got, exp, "variable k up to 1024")
    check_invariants(x, y, iss, ks, got[0], got[1], got[2], offsets=got[3])


def test_large_k_free_centres():
    x, y = family("clustered", 5000, 66)
    rng = np.random.default_rng(67)
    qx = rng.random(700, dtype=np.float32)
    qy = rng.random(700, dtype=np.float32)
    ex = rng.integers(-1, len(x), 700).astype(np.int32)
    exp = oracle.brute_knn_points(x, y, qx, qy, exclude=ex, k=600, threads=16)
    with binding.Context(len(x), 700, 600, leaf_capacity=32) as c:
        c.load_positions(x, y)
        c.advance_tick()
        c.query_points(qx, qy, exclude=ex, k=600)
        got = c.fetch()
    assert_rows_equal(got, exp, "free centres k=600")


def test_clustered_100k_k512_sampled():
    """A larger snapshot at k = 512 (the top of the paper's k study): 1,000
    sampled rows against brute force, and every row's invariants."""
    w = workloads.clustered_1m(n=100_000, ticks=1)
    x, y, _, _, _ = w.tick(0)
    k = 512
    say("clustered 100k k=%d" % k)
    with binding.Context(len(x), len(x), k, leaf_capacity=256) as c:
        c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
        c.advance_tick()
        c.query(k=k)
        ids, d2, cnt, _ = c.fetch()
    rng = np.random.default_rng(68)
    sample = rng.choice(len(x), 1000, replace=False).astype(np.int32)
    bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
    assert same(ids[sample], bi) and same_bits(d2[sample], bd) and same(cnt[sample], bc)
    for lo in range(0, len(x), 20000):
        rows = np.arange(lo, min(lo + 20000, len(x)))
        check_rows_vectorized(x, y, rows, ids[rows], d2[rows], cnt[rows], k)


def test_schedule_switches_between_ticks():
    """Leaf capacity, maximum level and sweep flavour changed between ticks
    of one context: every tick equals the oracle; invalid schedules are
    refused and change nothing."""
    x, y = family("clustered", 8000, 69)
    k = 40
    exp = oracle.brute_knn(x, y, k=k, threads=16)
    with binding.Context(len(x), len(x), 256, leaf_capacity=16, max_level=16) as c:
        assert c.schedule() == {"leaf_capacity": 16, "max_level": 16, "sweep": "auto",
                                "group_k": False, "tile_queries": 0}
        for th, L, sweep in ((16, 16, "auto"), (64, 12, "wave"), (200, 8, "lane"),
                             (32, 16, "wave"), (16, 13, "lane")):
            c.set_schedule(leaf_capacity=th, max_level=L, sweep=sweep)
            c.load_positions(x, y)
            c.advance_tick()
            c.query(k=k)
            say("schedule th=%d L=%d %s" % (th, L, sweep))
            assert_rows_equal(c.fetch(), exp, "th=%d L=%d %s" % (th, L, sweep))
            assert c.stats()["leaf_capacity"] == th
        # k above 128 in the lane setting still runs (wave flavour).
        c.query(k=200)
        assert_rows_equal(c.fetch(), oracle.brute_knn(x, y, k=200, threads=16), "k=200")
        before = c.schedule()
        for bad in ({"leaf_capacity": 0}, {"max_level": 17}, {"max_level": 0},
                    {"tile_queries": 12}, {"tile_queries": 128}):
            with pytest.raises(binding.MknnError) as e:
                c.set_schedule(**bad)
            assert e.value.code == -1
        with pytest.raises(binding.MknnError) as e:
            c.set_schedule(leaf_capacity=1)   # node tables sized for 16
        assert e.value.code == -4
        assert c.schedule() == before


def test_autotune_schedule():
    x, y = family("clustered", 20000, 70)
    k = 16
    exp = oracle.brute_knn(x, y, k=k, threads=16)
    with binding.Context(len(x), len(x), k, leaf_capacity=16, max_level=16, timing=True) as c:
        def tick(i):
            c.load_positions(x, y)
            c.advance_tick()
            c.query(k=k)
        best, times = binding.autotune_schedule(c, tick, (16, 64), max_levels=(12, 16),
                                                sweeps=("lane", "wave"), repeats=1, rounds=1)
        say("autotuned", best, times)
        assert best == c.schedule()
        assert best["leaf_capacity"] in (16, 64) and best["max_level"] in (12, 16)
        assert best["sweep"] in ("lane", "wave")
        assert len(times) >= 4
        tick(0)
        assert_rows_equal(c.fetch(), exp, "after autotuning")
