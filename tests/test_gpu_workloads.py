"""GPU parity on the larger workloads: the road-graph workload (4M objects,
half of them querying with k in {8,16,32,64}), the 16M-object, k=128
workload and a 64M-object snapshot.  Full comparison where the oracle
finishes in seconds, sampled brute force and per-row invariants
elsewhere."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding, workloads
from tests.helpers import check_rows_vectorized

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    yield


def bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def rows_block(ctx, r0, r1, k):
    """Rows [r0, r1) of a uniform-k result, copied from the device in one
    piece per array."""
    hip = binding._hip()
    ids_p, d2_p, cnt_p, _ = ctx.result_device_ptrs()
    ctx.sync()
    m = r1 - r0
    ids = np.empty((m, k), np.int32)
    d2 = np.empty((m, k), np.float32)
    cnt = np.empty(m, np.int32)
    for dst, src, size, off in ((ids, ids_p, 4 * k * m, 4 * k * r0), (d2, d2_p, 4 * k * m, 4 * k * r0),
                                (cnt, cnt_p, 4 * m, 4 * r0)):
        rc = hip.hipMemcpy(dst.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(src + off),
                           ctypes.c_size_t(size), 2)
        assert rc == 0
    return ids, d2, cnt


def test_network_4m_all_ticks():
    """The road-graph workload in the benchmark's stored configuration (leaf
    capacity 128, maximum level 12, 4M objects, a fresh half of them querying
    each tick with k in {8,16,32,64}): all 20 ticks on the GPU, the whole
    result against the oracle on ticks 0, 10 and 19, and 1,000 sampled
    queries per tick against brute force."""
    w = workloads.network_4m()
    with binding.Context(w.n, w.n // 2 + 1, 64, leaf_capacity=128, k_hint=64, max_level=12) as c:
        for t in range(w.ticks):
            x, y, iss, ks, _ = w.tick(t)
            print("network_4m tick %d: %d queries" % (t, len(iss)), flush=True)
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            c.advance_tick()
            c.query(issuers=torch.from_numpy(iss).cuda(), ks=torch.from_numpy(ks).cuda())
            gi, gd, gc, go = c.fetch()
            if t in (0, 10, 19):
                ei, ed, ec, eo = oracle.knn(x, y, issuers=iss, ks=ks, threads=16)
                assert np.array_equal(go, eo) and np.array_equal(gc, ec)
                assert np.array_equal(gi, ei) and np.array_equal(bits(gd), bits(ed))
            rng = np.random.default_rng(100 + t)
            sample = np.sort(rng.choice(len(iss), 1000, replace=False))
            bi, bd, bc, bo = oracle.brute_knn(x, y, issuers=iss[sample], ks=ks[sample],
                                              threads=16)
            assert np.array_equal(gc[sample], bc)
            for j, q in enumerate(sample):
                g = slice(go[q], go[q + 1])
                b = slice(bo[j], bo[j + 1])
                assert np.array_equal(gi[g], bi[b]) and np.array_equal(bits(gd[g]), bits(bd[b]))


def test_mixed_16m_k128_ticks_0_50_99():
    """The 16M-object, k = 128 workload in the benchmark's stored
    configuration (leaf capacity 384), ticks 0, 50 and 99: 200 sampled queries per tick
    against brute force, and every per-row invariant on a block of 65,536
    consecutive rows (all rows would be 16 GB of results)."""
    w = workloads.mixed_16m()
    k = 128
    with binding.Context(w.n, w.n, k, leaf_capacity=384, k_hint=k) as c:
        for t in (0, 50, 99):
            x, y, _, _, _ = w.tick(t)
            print("mixed_16m tick %d" % t, flush=True)
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            c.advance_tick()
            c.query(k=k)
            rng = np.random.default_rng(5 + t)
            sample = np.sort(rng.choice(w.n, 200, replace=False)).astype(np.int32)
            gi, gd, gc = c.fetch_rows(sample, k)
            bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
            assert np.array_equal(gc, bc)
            assert np.array_equal(gi, bi) and np.array_equal(bits(gd), bits(bd))
            r0 = int(rng.integers(0, w.n - 65536))
            ids, d2, cnt = rows_block(c, r0, r0 + 65536, k)
            check_rows_vectorized(x, y, np.arange(r0, r0 + 65536), ids, d2, cnt, k)


def test_maximum_size_64m_sampled():
    """64M objects (positions on the device), k = 8: the largest snapshot the
    tests build; rows checked against brute force on a sample."""
    n = 64_000_000
    rng = np.random.default_rng(77)
    dx = torch.rand(n, generator=torch.Generator().manual_seed(5)).cuda()
    dy = torch.rand(n, generator=torch.Generator().manual_seed(6)).cuda()
    x, y = dx.cpu().numpy(), dy.cpu().numpy()
    print("maximum size: %d objects" % n, flush=True)
    with binding.Context(n, n, 8, leaf_capacity=32) as c:
        c.load_positions(dx, dy)
        c.advance_tick()
        c.query(k=8)
        sample = np.sort(rng.choice(n, 100, replace=False)).astype(np.int32)
        gi, gd, gc = c.fetch_rows(sample, 8)
    bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=8, threads=16)
    assert np.array_equal(gc, bc)
    assert np.array_equal(gi, bi) and np.array_equal(bits(gd), bits(bd))
