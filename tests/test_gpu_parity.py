"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element and bit for bit (ids, d2 bit patterns, counts).

The bar is exact: both sides compute d2 = fl(fl(dx*dx) + fl(dy*dy)) in fp32
with no contraction and order by (d2, id), so any difference is a bug."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding, workloads
from tests.helpers import FAMILIES, check_invariants, f32, family

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


def same(a, b):
    return np.array_equal(np.asarray(a), np.asarray(b))


def same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


def assert_rows_equal(got, exp, what=""):
    gi, gd, gc, go = got
    ei, ed, ec, eo = exp
    assert same(gc, ec), "counts differ %s" % what
    if not same(gi, ei) or not same_bits(gd, ed):
        gi2 = np.asarray(gi).reshape(len(gc), -1) if go is None else gi
        ei2 = np.asarray(ei).reshape(len(ec), -1) if eo is None else ei
        bad = np.nonzero(np.any(gi2 != ei2, axis=1))[0] if go is None else []
        raise AssertionError("rows differ %s: first bad rows %s\n got %s\n exp %s" % (
            what, bad[:5], gi2[bad[:1]] if len(bad) else "", ei2[bad[:1]] if len(bad) else ""))
    if go is not None or eo is not None:
        assert same(go, eo)


def gpu_knn(x, y, k=None, issuers=None, ks=None, th=0, L=0, k_max=None, device_inputs=False,
            group_k=False):
    n = len(x)
    nq = n if issuers is None else len(issuers)
    if k_max is None:
        k_max = int(k) if ks is None else int(np.max(ks))
    with binding.Context(max(n, 1), max(nq, 1), k_max, leaf_capacity=th, max_level=L,
                         group_k=group_k) as c:
        if device_inputs:
            c.load_positions(torch.from_numpy(f32(x)).cuda(), torch.from_numpy(f32(y)).cuda())
        else:
            c.load_positions(x, y)
        c.advance_tick()
        if device_inputs:
            iss = None if issuers is None else torch.from_numpy(np.asarray(issuers, np.int32)).cuda()
            kk = None if ks is None else torch.from_numpy(np.asarray(ks, np.int32)).cuda()
            c.query(k=k, issuers=iss, ks=kk, nq=nq)
        else:
            c.query(k=k, issuers=issuers, ks=ks, nq=nq)
        return c.fetch()


# ---------------------------------------------------------------------------
# The benchmark workloads
# ---------------------------------------------------------------------------

def test_uniform_10k_full_parity():
    w = workloads.uniform_10k()
    x, y, _, _, k = w.tick(0)
    say("uniform_10k: n=%d k=%d" % (len(x), k))
    got = gpu_knn(x, y, k=k)
    exp = oracle.knn(x, y, k=k, threads=16)
    assert_rows_equal(got, exp, "vs quadtree oracle")
    bru = oracle.brute_knn(x, y, k=k, threads=16)
    assert_rows_equal(got, bru, "vs brute force")
    check_invariants(x, y, None, None, got[0], got[1], got[2], k=k)


def test_clustered_1m_all_ticks_full_parity():
    """The benchmark's 1M-object workload, every tick, every query, in the
    configuration bench.py times (leaf capacity 64, maximum level 12, one
    context advanced tick after tick): the whole result against the oracle, and
    2,000 sampled queries per tick against brute force."""
    w = workloads.clustered_1m()
    k = w.k
    with binding.Context(w.n, w.n, k, leaf_capacity=64, k_hint=k, max_level=12) as c:
        for t in range(w.ticks):
            x, y, _, _, _ = w.tick(t)
            say("clustered_1m tick %d" % t)
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            c.advance_tick()
            c.query(k=k)
            got = c.fetch()
            exp = oracle.knn(x, y, k=k, threads=16)
            assert_rows_equal(got, exp, "tick %d" % t)
            # The oracle itself checked against brute force on 2,000 queries.
            rng = np.random.default_rng(11 + t)
            sample = rng.choice(w.n, 2000, replace=False).astype(np.int32)
            bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
            assert same(got[0][sample], bi) and same_bits(got[1][sample], bd)
            assert np.array_equal(got[2][sample], bc)


# ---------------------------------------------------------------------------
# Families, k and leaf capacity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", FAMILIES)
def test_families_many_k_and_th(kind):
    x, y = family(kind, 3000, 21)
    for k in (1, 8, 13, 32, 33, 64, 128):
        exp = oracle.brute_knn(x, y, k=k, threads=16)
        for th in (1, 7, 64, 1000):
            say("%s k=%d th=%d" % (kind, k, th))
            got = gpu_knn(x, y, k=k, th=th)
            assert_rows_equal(got, exp, "%s k=%d th=%d" % (kind, k, th))


@pytest.mark.parametrize("L", [1, 3, 8, 12, 13, 16])
def test_max_level(L):
    x, y = family("clustered", 2500, 22)
    exp = oracle.brute_knn(x, y, k=16, threads=16)
    for th in (2, 40):
        say("L=%d th=%d" % (L, th))
        assert_rows_equal(gpu_knn(x, y, k=16, th=th, L=L), exp, "L=%d th=%d" % (L, th))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 129, 300])
def test_small_n_and_k_beyond_n(n):
    x, y = family("uniform", n, 23)
    for k in sorted({1, 2, max(1, n - 1), n, n + 5, 32}):
        if k > binding.MKNN_K_LIMIT:
            continue
        exp = oracle.brute_knn(x, y, k=k)
        for L in (16, 12):  # the default, and the benchmark's three-pass sort
            say("n=%d k=%d L=%d" % (n, k, L))
            assert_rows_equal(gpu_knn(x, y, k=k, th=4, L=L), exp, "n=%d k=%d L=%d" % (n, k, L))


def test_ties_lattice_duplicates_and_denormals():
    side = 64
    iy, ix = np.divmod(np.arange(side * side), side)
    x = (ix * 2.0 ** -6).astype(np.float32)
    y = (iy * 2.0 ** -6).astype(np.float32)
    for k in (4, 8, 32, 36, 128):
        say("lattice k=%d" % k)
        assert_rows_equal(gpu_knn(x, y, k=k, th=10), oracle.brute_knn(x, y, k=k, threads=16))
    x = np.full(500, 0.375, np.float32)
    y = np.full(500, 0.625, np.float32)
    got = gpu_knn(x, y, k=10, th=3)
    assert_rows_equal(got, oracle.brute_knn(x, y, k=10))
    assert got[0][7].tolist() == [0, 1, 2, 3, 4, 5, 6, 8, 9, 10]
    x = f32([0.0, 2.0 ** -69, 2.0 ** -70, 2.0 ** -71])
    y = f32([0.0, 0.0, 0.0, 0.0])
    got = gpu_knn(x, y, k=3, th=1)
    assert got[0][0].tolist() == [3, 2, 1], "denormal d2 must be kept"
    assert_rows_equal(got, oracle.brute_knn(x, y, k=3))


# ---------------------------------------------------------------------------
# Index parity (Sec. 4.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["uniform", "clustered", "duplicates", "boundary"])
@pytest.mark.parametrize("th,L", [(1, 16), (5, 4), (2, 7), (3, 12), (8, 13), (64, 16), (384, 16),
                                  (5000, 16)])
def test_index_matches_oracle(kind, th, L):
    x, y = family(kind, 5000, 24)
    exp = oracle.build_index(x, y, th, L)
    with binding.Context(len(x), len(x), 8, leaf_capacity=th, max_level=L) as c:
        c.load_positions(x, y)
        c.advance_tick()
        got = c.index()
        deepest = c.stats()["deepest_level"]
    for key in ("codes", "ids", "leaf_level", "leaf_prefix", "leaf_begin", "leaf_end"):
        assert same(got[key], exp[key]), key
    assert deepest == int(np.max(exp["leaf_level"]))


def test_deepest_level_per_build():
    """The deepest leaf level is that of the latest build, also when it is
    shallower than an earlier build's (the statistic is tagged with the
    build's epoch, so an older, larger value does not stick)."""
    deep = family("clustered", 20000, 25)
    flat = family("uniform", 20000, 26)
    with binding.Context(20000, 20000, 8, leaf_capacity=4, max_level=16) as c:
        for (x, y), th in ((deep, 4), (flat, 4), (deep, 4), (flat, 4)):
            c.set_leaf_capacity(th)
            c.load_positions(x, y)
            c.advance_tick()
            exp = oracle.build_index(x, y, th, 16)
            assert c.stats()["deepest_level"] == int(np.max(exp["leaf_level"]))


def test_sort_tile_size_boundary():
    """The radix sort switches to larger tiles at 2^21 keys; one context
    sized above the switch sorts n just below, at and above it (its
    workspace was sized for the largest tile count any n up to its capacity
    needs): the order equals the oracle's, sampled rows equal brute force."""
    cap = (1 << 21) + 4097
    rng = np.random.default_rng(31)
    with binding.Context(cap, cap, 4, leaf_capacity=32) as c:
        for n in ((1 << 21) - 1, 1 << 21, cap):
            x = rng.random(n, dtype=np.float32)
            y = rng.random(n, dtype=np.float32)
            say("sort tile boundary: n=%d" % n)
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            c.advance_tick()
            got = c.index()
            exp = oracle.build_index(x, y, 32, 16)
            assert same(got["codes"], exp["codes"]) and same(got["ids"], exp["ids"])
            c.query(k=4)
            sample = np.sort(rng.choice(n, 100, replace=False)).astype(np.int32)
            gi, gd, gc = c.fetch_rows(sample, 4)
            bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=4, threads=16)
            assert same(gi, bi) and same_bits(gd, bd) and same(gc, bc)


# ---------------------------------------------------------------------------
# Query subsets, variable k, device inputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("device_inputs", [False, True])
def test_subset_and_variable_k(device_inputs):
    x, y = family("clustered", 6000, 25)
    rng = np.random.default_rng(5)
    iss = rng.choice(6000, 2500, replace=False).astype(np.int32)
    ks = rng.choice([1, 8, 16, 32, 64], 2500).astype(np.int32)
    say("subset+variable k, device=%s" % device_inputs)
    got = gpu_knn(x, y, issuers=iss, ks=ks, device_inputs=device_inputs)
    exp = oracle.brute_knn(x, y, issuers=iss, ks=ks, threads=16)
    assert_rows_equal(got, exp, "variable k")
    got = gpu_knn(x, y, k=16, issuers=iss, device_inputs=device_inputs)
    exp = oracle.brute_knn(x, y, issuers=iss, k=16, threads=16)
    assert_rows_equal(got, exp, "subset")
    got = gpu_knn(x, y, ks=np.full(6000, 7, np.int32), device_inputs=device_inputs)
    exp = oracle.brute_knn(x, y, ks=np.full(6000, 7, np.int32), threads=16)
    assert_rows_equal(got, exp, "all objects, ks array")


@pytest.mark.parametrize("group_k", [False, True])
@pytest.mark.parametrize("device_inputs", [False, True])
def test_variable_k_every_class(device_inputs, group_k):
    """Variable k spanning all five selection-list classes (k up to 128), in
    one pass sized for the largest k or (MKNN_FLAG_GROUP_K) grouped by
    class with each class at its own list size; rows come back in query
    order either way."""
    x, y = family("duplicates", 9000, 41)
    rng = np.random.default_rng(8)
    for issuers in (None, rng.choice(9000, 4000, replace=False).astype(np.int32)):
        nq = 9000 if issuers is None else len(issuers)
        ks = rng.integers(1, 129, nq).astype(np.int32)
        ks[rng.random(nq) < 0.3] = 8          # a crowded class
        say("variable k, all classes, subset=%s device=%s" % (issuers is not None, device_inputs))
        got = gpu_knn(x, y, issuers=issuers, ks=ks, th=24, device_inputs=device_inputs,
                      group_k=group_k)
        exp = oracle.knn(x, y, issuers=issuers, ks=ks, th=24, threads=16)
        assert_rows_equal(got, exp, "variable k, every class")
    # Only two classes present (host ks launch only those).
    ks = np.where(rng.random(9000) < 0.5, 3, 40).astype(np.int32)
    got = gpu_knn(x, y, ks=ks, th=24, device_inputs=device_inputs, group_k=group_k)
    assert_rows_equal(got, oracle.knn(x, y, ks=ks, th=24, threads=16), "two classes")


def test_subset_orders_radix_and_owner_table():
    """Subset queries are ordered by a radix sort of their positions when
    they are fewer than one per 64 objects, else through a table of the
    issuers' positions (repeated issuers listed after the others).  Both
    orders, either side of the switch, with and without repeats, many more
    queries than objects, every object in shuffled order, and calls in a row
    on one context (the table clears itself after each call), each row
    against the oracle."""
    n = 20_000
    x, y = family("clustered", n, 27)
    rng = np.random.default_rng(27)
    # The switch: ceil(n / 64) = 313 <= nq + 1.
    cases = [
        ("radix, distinct", rng.choice(n, 311, replace=False)),
        ("table, distinct", rng.choice(n, 312, replace=False)),
        ("table, distinct, more", rng.choice(n, 700, replace=False)),
        ("table, repeats", rng.integers(0, n, 8000)),
        ("table, more queries than objects", rng.integers(0, n, 50_000)),
        ("table, every object shuffled", rng.permutation(n)),
        ("radix, repeats", np.array([7, 7, 19_999, 0, 7] * 40)),
    ]
    with binding.Context(n, 50_000, 24) as c:
        c.load_positions(x, y)
        c.advance_tick()
        for rnd in range(2):
            for what, iss in cases:
                iss = np.asarray(iss, np.int32)
                ks = rng.choice([1, 5, 12, 24], len(iss)).astype(np.int32)
                say("subset order: %s (%d queries), call %d" % (what, len(iss), rnd))
                c.query(k=12, issuers=iss)
                assert_rows_equal(c.fetch(), oracle.knn(x, y, issuers=iss, k=12, threads=16), what)
                c.query(issuers=iss, ks=ks)
                assert_rows_equal(c.fetch(), oracle.knn(x, y, issuers=iss, ks=ks, threads=16),
                                  what + ", variable k")


def test_repeated_issuers_and_empty_query():
    x, y = family("uniform", 800, 26)
    iss = np.array([5, 5, 799, 0, 5], np.int32)
    assert_rows_equal(gpu_knn(x, y, k=9, issuers=iss), oracle.brute_knn(x, y, issuers=iss, k=9))
    with binding.Context(800, 800, 8) as c:
        c.load_positions(x, y)
        c.advance_tick()
        c.query(k=8, issuers=np.zeros(0, np.int32), nq=0)
        ids, d2, cnt, _ = c.fetch()
        assert ids.shape == (0, 8) and cnt.shape == (0,)


# ---------------------------------------------------------------------------
# Determinism and independence from the index parameters
# ---------------------------------------------------------------------------

def test_results_do_not_depend_on_th_or_L_and_repeat_bitwise():
    w = workloads.clustered_1m(n=200_000, ticks=1)
    x, y, _, _, k = w.tick(0)
    ref = None
    for th, L in ((384, 16), (32, 16), (8, 12), (2048, 16), (100, 6)):
        say("independence th=%d L=%d" % (th, L))
        got = gpu_knn(x, y, k=k, th=th, L=L)
        if ref is None:
            ref = got
            again = gpu_knn(x, y, k=k, th=th, L=L)
            assert_rows_equal(again, ref, "repeat")
        else:
            assert_rows_equal(got, ref, "th=%d L=%d" % (th, L))
    rng = np.random.default_rng(3)
    sample = rng.choice(len(x), 300, replace=False).astype(np.int32)
    bi, bd, _, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
    assert same(ref[0][sample], bi) and same_bits(ref[1][sample], bd)


def test_many_ticks_in_one_context():
    w = workloads.clustered_1m(n=50_000, ticks=4)
    with binding.Context(w.n, w.n, 32, leaf_capacity=48) as c:
        for t in range(w.ticks):
            x, y, _, _, _ = w.tick(t)
            c.load_positions(x, y)
            c.advance_tick()
            c.query(k=32)
            assert_rows_equal(c.fetch(), oracle.knn(x, y, k=32, threads=16), "tick %d" % t)
            c.query(k=5)   # a second query on the same index
            assert_rows_equal(c.fetch(), oracle.knn(x, y, k=5, threads=16), "k=5 tick %d" % t)


def test_subset_queries_across_ticks_sizes_and_refits():
    """Issuer subsets on consecutive ticks of one context: every build
    needs the objects' sorted positions again, object counts change between
    builds, and a refit tick keeps the last build's order."""
    rng = np.random.default_rng(31)
    with binding.Context(30_000, 5_000, 16, leaf_capacity=24) as c:
        for t, (n, refit) in enumerate(((30_000, False), (30_000, False), (20_000, False),
                                         (20_000, True), (30_000, False))):
            if refit:  # the last build's objects, moved a little
                x = np.clip(x + rng.uniform(-1e-4, 1e-4, n), 0, 0.999).astype(np.float32)
            else:
                x, y = family("clustered", n, 40 + t)
            iss = rng.choice(n, 4000, replace=False).astype(np.int32)
            ks = rng.integers(1, 17, len(iss)).astype(np.int32)
            c.load_positions(x, y)
            if refit:
                c.refit_tick()
            else:
                c.advance_tick()
            c.query(issuers=torch.from_numpy(iss).cuda(), ks=torch.from_numpy(ks).cuda())
            say("subset tick %d n=%d refit=%s" % (t, n, refit))
            assert_rows_equal(c.fetch(), oracle.knn(x, y, issuers=iss, ks=ks, threads=16),
                              "subset tick %d" % t)


# ---------------------------------------------------------------------------
# Boundary behaviour
# ---------------------------------------------------------------------------

def test_errors_and_state():
    x, y = family("uniform", 100, 27)
    with binding.Context(100, 100, 16) as c:
        with pytest.raises(binding.MknnError) as e:
            c.advance_tick()
        assert e.value.code == -3
        bad = x.copy()
        bad[3] = 1.0
        with pytest.raises(binding.MknnError) as e:
            c.load_positions(bad, y)
        assert e.value.code == -2
        c.load_positions(x, y)
        with pytest.raises(binding.MknnError) as e:
            c.query(k=4)
        assert e.value.code == -3
        c.advance_tick()
        for kk in (0, 17):
            with pytest.raises(binding.MknnError) as e:
                c.query(k=kk)
            assert e.value.code == -1
        with pytest.raises(binding.MknnError) as e:
            c.query(k=4, issuers=np.array([100], np.int32))
        assert e.value.code == -1
        with pytest.raises(binding.MknnError) as e:
            c.load_positions(np.zeros(101, np.float32), np.zeros(101, np.float32))
        assert e.value.code == -4
        # Device input with a NaN: reported at the next synchronisation.
        dx = torch.from_numpy(x).cuda()
        dx[7] = float("nan")
        c.load_positions(dx, torch.from_numpy(y).cuda())
        c.advance_tick()
        with pytest.raises(binding.MknnError) as e:
            c.sync()
        assert e.value.code == -2
        c.load_positions(x, y)
        c.advance_tick()
        c.query(k=4, issuers=torch.tensor([1, 500, 2], dtype=torch.int32).cuda())
        with pytest.raises(binding.MknnError) as e:
            c.fetch()
        assert e.value.code == -1
        c.query(k=4)
        ids, d2, cnt, _ = c.fetch()
        assert_rows_equal((ids, d2, cnt, None), oracle.brute_knn(x, y, k=4))


def test_borrowed_torch_stream():
    x, y = family("clustered", 4000, 28)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with binding.Context(4000, 4000, 16, stream=s.cuda_stream) as c:
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            c.advance_tick()
            c.query(k=16)
            got = c.fetch()
    assert_rows_equal(got, oracle.brute_knn(x, y, k=16, threads=16))
