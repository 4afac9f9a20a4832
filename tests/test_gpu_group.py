"""GPU parity of the group-per-query sweep (MKNN_SWEEP_GROUP: a query's list
spread over a group of k/16 lanes, Sec. 4.2.1's coalesced-writes flavour),
bit for bit against the oracle (brute force, Definition 1) through the C
ABI: every list size from 32 to 1024 keys (groups of 2 to 64 lanes), the
input families, k past n - 1, duplicates and denormals, subsets with
variable k (host and device inputs, one pass and per k class), free
centres, refit ticks, and the autotuner choosing among the flavours."""
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


def run(x, y, k=None, issuers=None, ks=None, th=0, L=0, k_max=None, device_inputs=False,
        group_k=False):
    n = len(x)
    nq = n if issuers is None else len(issuers)
    if k_max is None:
        k_max = int(k) if ks is None else int(np.max(ks))
    with binding.Context(max(n, 1), max(nq, 1), k_max, leaf_capacity=th, max_level=L) as c:
        c.set_schedule(sweep="group", group_k=group_k)
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
def test_group_families_every_list_size(kind):
    x, y = family(kind, 2500, 91)
    for k in (1, 8, 31, 32, 33, 64, 65, 128, 129, 256, 512, 1024):
        exp = oracle.brute_knn(x, y, k=k, threads=16)
        for th in (7, 96):
            say("group %s k=%d th=%d" % (kind, k, th))
            assert_rows_equal(run(x, y, k=k, th=th), exp, "group %s k=%d th=%d" % (kind, k, th))


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 300])
def test_group_k_beyond_n(n):
    x, y = family("uniform", n, 92)
    for k in sorted({1, max(1, n - 1), n, n + 5, 64, 130}):
        exp = oracle.brute_knn(x, y, k=k)
        for L in (16, 9):
            say("group n=%d k=%d L=%d" % (n, k, L))
            assert_rows_equal(run(x, y, k=k, th=4, L=L), exp, "n=%d k=%d L=%d" % (n, k, L))


def test_group_ties_duplicates_denormals():
    side = 48
    iy, ix = np.divmod(np.arange(side * side), side)
    x = (ix * 2.0 ** -6).astype(np.float32)
    y = (iy * 2.0 ** -6).astype(np.float32)
    for k in (40, 200):
        say("group lattice k=%d" % k)
        assert_rows_equal(run(x, y, k=k, th=10), oracle.brute_knn(x, y, k=k, threads=16))
    x = np.full(900, 0.375, np.float32)
    y = np.full(900, 0.625, np.float32)
    got = run(x, y, k=128, th=3)
    assert_rows_equal(got, oracle.brute_knn(x, y, k=128, threads=16))
    assert got[0][11].tolist() == [i for i in range(129) if i != 11]
    x = (np.arange(500) * 2.0 ** -80).astype(np.float32)
    y = np.zeros(500, np.float32)
    assert_rows_equal(run(x, y, k=64, th=5), oracle.brute_knn(x, y, k=64))


@pytest.mark.parametrize("device_inputs,group_k", [(False, False), (True, False), (False, True)])
def test_group_variable_k_subset(device_inputs, group_k):
    x, y = family("clustered", 6000, 93)
    rng = np.random.default_rng(94)
    iss = rng.choice(len(x), 2500, replace=False).astype(np.int32)
    ks = rng.choice([1, 8, 16, 32, 64, 100, 128], 2500).astype(np.int32)
    exp = oracle.brute_knn(x, y, issuers=iss, ks=ks, threads=16)
    got = run(x, y, issuers=iss, ks=ks, th=48, k_max=128, device_inputs=device_inputs,
              group_k=group_k)
    assert_rows_equal(got, exp, "group variable k (group_k=%s)" % group_k)
    check_invariants(x, y, iss, ks, got[0], got[1], got[2], offsets=got[3])


def test_group_free_centres():
    x, y = family("clustered", 5000, 95)
    rng = np.random.default_rng(96)
    qx = rng.random(700, dtype=np.float32)
    qy = rng.random(700, dtype=np.float32)
    ex = rng.integers(-1, len(x), 700).astype(np.int32)
    for k in (20, 64, 300):
        exp = oracle.brute_knn_points(x, y, qx, qy, exclude=ex, k=k, threads=16)
        with binding.Context(len(x), 700, k, leaf_capacity=32) as c:
            c.set_schedule(sweep="group")
            c.load_positions(x, y)
            c.advance_tick()
            c.query_points(qx, qy, exclude=ex, k=k)
            got = c.fetch()
        say("group free centres k=%d" % k)
        assert_rows_equal(got, exp, "group free centres k=%d" % k)


def test_group_refit_ticks():
    w = workloads.clustered_1m(n=40_000, ticks=4)
    k = 64
    with binding.Context(w.n, w.n, k, leaf_capacity=64) as c:
        c.set_schedule(sweep="group")
        for t in range(4):
            x, y, _, _, _ = w.tick(t)
            c.load_positions(x, y)
            if t == 0:
                c.advance_tick()
            else:
                c.refit_tick()
            c.query(k=k)
            ids, d2, cnt, _ = c.fetch()
            rng = np.random.default_rng(97 + t)
            sample = rng.choice(w.n, 400, replace=False).astype(np.int32)
            bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
            say("group refit tick %d" % t)
            assert same(ids[sample], bi) and same_bits(d2[sample], bd) and same(cnt[sample], bc)


def test_group_clustered_100k_sampled():
    w = workloads.clustered_1m(n=100_000, ticks=1)
    x, y, _, _, _ = w.tick(0)
    for k in (64, 128):
        with binding.Context(len(x), len(x), k, leaf_capacity=96) as c:
            c.set_schedule(sweep="group")
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            c.advance_tick()
            c.query(k=k)
            ids, d2, cnt, _ = c.fetch()
        rng = np.random.default_rng(98)
        sample = rng.choice(len(x), 1000, replace=False).astype(np.int32)
        bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
        say("group clustered 100k k=%d" % k)
        assert same(ids[sample], bi) and same_bits(d2[sample], bd) and same(cnt[sample], bc)
        for lo in range(0, len(x), 25000):
            rows = np.arange(lo, min(lo + 25000, len(x)))
            check_rows_vectorized(x, y, rows, ids[rows], d2[rows], cnt[rows], k)


def test_autotuner_takes_the_group_flavour_into_account():
    x, y = family("clustered", 20000, 99)
    k = 64
    exp = oracle.brute_knn(x, y, k=k, threads=16)
    with binding.Context(len(x), len(x), k, leaf_capacity=32, max_level=16, timing=True) as c:
        def tick(i):
            c.load_positions(x, y)
            c.advance_tick()
            c.query(k=k)
        best, times = binding.autotune_schedule(c, tick, (32, 64), sweeps=("lane", "group"),
                                                repeats=1, rounds=1)
        say("autotuned", best, times)
        assert best["sweep"] in ("lane", "group")
        assert any("sweep=group" in key for key in times)
        tick(0)
        assert_rows_equal(c.fetch(), exp, "after autotuning")
