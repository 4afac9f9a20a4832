"""GPU parity on the larger workloads: the road-graph workload (4M objects,
half of them querying with k in {8,16,32,64}) and the 16M-object, k=128
workload.  Full comparison where the oracle finishes in seconds, sampled
brute force elsewhere."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding, workloads

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


def test_network_4m_variable_k_subset():
    w = workloads.network_4m(ticks=2)
    with binding.Context(w.n, w.n // 2 + 1, 64, leaf_capacity=32) as c:
        for t in range(2):
            x, y, iss, ks, _ = w.tick(t)
            print("network_4m tick %d: %d queries" % (t, len(iss)), flush=True)
            c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
            c.advance_tick()
            c.query(issuers=torch.from_numpy(iss).cuda(), ks=torch.from_numpy(ks).cuda())
            gi, gd, gc, go = c.fetch()
            if t == 0:
                ei, ed, ec, eo = oracle.knn(x, y, issuers=iss, ks=ks, threads=16)
                assert np.array_equal(go, eo) and np.array_equal(gc, ec)
                assert np.array_equal(gi, ei) and np.array_equal(bits(gd), bits(ed))
            else:
                rng = np.random.default_rng(t)
                sample = rng.choice(len(iss), 300, replace=False)
                bi, bd, bc, bo = oracle.brute_knn(x, y, issuers=iss[sample], ks=ks[sample],
                                                  threads=16)
                for j, q in enumerate(sample):
                    g = slice(go[q], go[q + 1])
                    b = slice(bo[j], bo[j + 1])
                    assert np.array_equal(gi[g], bi[b]) and np.array_equal(bits(gd[g]), bits(bd[b]))


def test_mixed_16m_k128_sampled():
    w = workloads.mixed_16m(ticks=2)
    k = 128
    x, y, _, _, _ = w.tick(1)
    with binding.Context(w.n, w.n, k, leaf_capacity=1536) as c:
        print("mixed_16m tick 1", flush=True)
        c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
        c.advance_tick()
        c.query(k=k)
        rng = np.random.default_rng(5)
        sample = np.sort(rng.choice(w.n, 200, replace=False)).astype(np.int32)
        gi, gd, gc = c.fetch_rows(sample, k)
    bi, bd, bc, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
    assert np.array_equal(gc, bc)
    assert np.array_equal(gi, bi) and np.array_equal(bits(gd), bits(bd))


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
