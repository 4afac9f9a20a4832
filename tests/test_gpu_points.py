"""GPU parity of queries with free centres (Definition 1: q = (x, y, k)
anywhere in the square, optionally excluding one object), through the C
ABI, against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding, workloads
from tests.helpers import FAMILIES, f32, family

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


def centres(nq, seed, x, y, scale=1.0):
    rng = np.random.default_rng([23, seed, nq])
    qx, qy = rng.random(nq, dtype=np.float32), rng.random(nq, dtype=np.float32)
    on = rng.random(nq) < 0.3
    pick = rng.integers(0, len(x), nq)
    if scale != 1.0:
        qx, qy = (qx * scale).astype(np.float32), (qy * scale).astype(np.float32)
    qx[on], qy[on] = x[pick[on]], y[pick[on]]
    qx[rng.random(nq) < 0.05] = 0.0
    qy[rng.random(nq) < 0.05] = np.float32(1.0 - 2.0 ** -24)
    ex = np.where(on & (rng.random(nq) < 0.7), pick, -1).astype(np.int32)
    return f32(qx), f32(qy), ex


def gpu_points(x, y, qx, qy, exclude=None, k=None, ks=None, th=0, L=0, device=False):
    n, nq = len(x), len(qx)
    k_max = int(k) if ks is None else int(np.max(ks))
    with binding.Context(max(n, 1), max(nq, 1), k_max, leaf_capacity=th, max_level=L) as c:
        c.load_positions(x, y)
        c.advance_tick()
        if device:
            t = lambda a, dt=torch.float32: None if a is None else torch.from_numpy(np.asarray(a)).to(dt).cuda()
            c.query_points(t(qx), t(qy), t(exclude, torch.int32), k=k, ks=t(ks, torch.int32))
        else:
            c.query_points(qx, qy, exclude, k=k, ks=ks)
        return c.fetch()


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("k,th", [(1, 1), (8, 7), (13, 64), (32, 16), (64, 1000)])
def test_points_families(kind, k, th):
    x, y = family(kind, 700, 31)
    scale = 2.0 ** -64 if kind == "tiny_scale" else 1.0
    qx, qy, ex = centres(300, 1, x, y, scale)
    say("points %s k=%d th=%d" % (kind, k, th))
    for excl in (None, ex):
        ei, ed, ec, _ = oracle.knn_points(x, y, qx, qy, exclude=excl, k=k, th=5)
        # At L = 12 the objects are sorted by their top 24 code bits only, so
        # the centres' placement searches a partly sorted sequence.
        for L in (0, 12):
            gi, gd, gc, _ = gpu_points(x, y, qx, qy, excl, k=k, th=th, L=L)
            assert np.array_equal(gc, ec)
            assert np.array_equal(gi, ei) and same_bits(gd, ed)


def test_points_on_objects_equal_issuer_queries():
    x, y = family("clustered", 5000, 3)
    rng = np.random.default_rng(4)
    iss = rng.integers(0, len(x), 2000).astype(np.int32)
    ks = rng.integers(1, 49, 2000).astype(np.int32)
    with binding.Context(len(x), 2000, 48, leaf_capacity=24) as c:
        c.load_positions(x, y)
        c.advance_tick()
        c.query(issuers=iss, ks=ks)
        a = c.fetch()
        c.query_points(x[iss], y[iss], iss, ks=ks)
        b = c.fetch()
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_points_device_inputs_variable_k_and_order():
    x, y = family("duplicates", 3000, 8)
    qx, qy, ex = centres(1500, 2, x, y)
    ks = np.random.default_rng(3).integers(1, 33, 1500).astype(np.int32)
    g = gpu_points(x, y, qx, qy, ex, ks=ks, th=12, device=True)
    e = oracle.knn_points(x, y, qx, qy, exclude=ex, ks=ks, th=12)
    assert np.array_equal(g[3], e[3]) and np.array_equal(g[2], e[2])
    assert np.array_equal(g[0], e[0]) and same_bits(g[1], e[1])


def test_points_small_n_counts():
    for n in (1, 2, 3):
        x, y = family("uniform", n, 40 + n)
        qx, qy = f32([0.5, 0.25, x[0]]), f32([0.5, 0.75, y[0]])
        ex = np.array([-1, n - 1, 0], np.int32)
        gi, gd, gc, _ = gpu_points(x, y, qx, qy, ex, k=4)
        ei, ed, ec, _ = oracle.brute_knn_points(x, y, qx, qy, exclude=ex, k=4)
        assert np.array_equal(gc, ec) and np.array_equal(gi, ei) and same_bits(gd, ed)


def test_points_clustered_200k_sampled():
    w = workloads.clustered_1m(n=200_000, ticks=1)
    x, y, _, _, _ = w.tick(0)
    qx, qy, ex = centres(100_000, 6, x, y)
    say("points clustered_200k: 100k centres")
    gi, gd, gc, _ = gpu_points(x, y, qx, qy, ex, k=32, th=64)
    ei, ed, ec, _ = oracle.knn_points(x, y, qx, qy, exclude=ex, k=32, threads=16)
    assert np.array_equal(gc, ec)
    assert np.array_equal(gi, ei) and same_bits(gd, ed)


def test_points_errors():
    x, y = family("uniform", 100, 5)
    with binding.Context(100, 100, 16) as c:
        c.load_positions(x, y)
        c.advance_tick()
        with pytest.raises(binding.MknnError) as e:
            c.query_points(f32([0.5, 1.0]), f32([0.5, 0.5]), k=2)
        assert e.value.code == -2
        with pytest.raises(binding.MknnError) as e:
            c.query_points(f32([0.5]), f32([0.5]), np.array([100], np.int32), k=2)
        assert e.value.code == -1
        dq = torch.tensor([0.5, float("nan")], dtype=torch.float32).cuda()
        c.query_points(dq, torch.tensor([0.5, 0.5]).cuda(), k=2)
        with pytest.raises(binding.MknnError) as e:
            c.fetch()
        assert e.value.code == -2
        c.query_points(f32([0.5]), f32([0.5]), k=2)
        gi, gd, gc, _ = c.fetch()
        ei, ed, ec, _ = oracle.brute_knn_points(x, y, f32([0.5]), f32([0.5]), k=2)
        assert np.array_equal(gi, ei) and same_bits(gd, ed)
