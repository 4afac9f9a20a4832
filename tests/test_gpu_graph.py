"""GPU: the tick captured as a HIP graph and replayed gives the eager
result on every replay; switching the leaf capacity between ticks changes
nothing in the results."""
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


def test_graph_replays_match_eager():
    w = workloads.clustered_1m(n=120_000, ticks=3)
    k = 32
    s = torch.cuda.Stream()
    dev = []
    for t in range(w.ticks):
        x, y, _, _, _ = w.tick(t)
        dev.append((torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()))
    with torch.cuda.stream(s):
        # The benchmark's maximum level (a three-pass sort) for the captured
        # context, the default for the other one.
        ctx = binding.Context(w.n, w.n, k, leaf_capacity=32, max_level=12, stream=s.cuda_stream)
        other = binding.Context(w.n, w.n, 8, leaf_capacity=16, stream=s.cuda_stream)
        eager = []
        for t in range(w.ticks):
            ctx.load_positions(*dev[t])
            ctx.advance_tick()
            ctx.query(k=k, nq=w.n)
            eager.append(ctx.fetch())
        graphs = []
        for t in range(w.ticks):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                ctx.load_positions(*dev[t])
                ctx.advance_tick()
                ctx.query(k=k, nq=w.n)
            graphs.append(g)
        for rep in range(3):
            for t in (2, 0, 1):
                graphs[t].replay()
                ids, d2, cnt, _ = ctx.fetch()   # synchronises between replays
                assert np.array_equal(ids, eager[t][0]), (rep, t)
                assert np.array_equal(bits(d2), bits(eager[t][1])), (rep, t)
                assert np.array_equal(cnt, eager[t][2])
                # eager work between replays: another context on the same
                # stream, and an eager query of the same shape on this one
                # (the host-side description of the results -- nq, k --
                # is that of the last call made on the host)
                other.load_positions(*dev[(t + 1) % w.ticks])
                other.advance_tick()
                other.query(k=5, nq=w.n)
                other.sync()
                ctx.query(k=k, nq=w.n)
                ctx.sync()
        del graphs
        ctx.close()
        other.close()
    x, y, _, _, _ = w.tick(1)
    sample = np.arange(0, w.n, 997, dtype=np.int32)
    bi, bd, _, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
    assert np.array_equal(eager[1][0][sample], bi) and np.array_equal(bits(eager[1][1][sample]), bits(bd))


def test_leaf_capacity_switch_between_ticks():
    w = workloads.clustered_1m(n=80_000, ticks=2)
    x, y, _, _, _ = w.tick(1)
    exp = oracle.knn(x, y, k=16, threads=16)
    with binding.Context(w.n, w.n, 16, leaf_capacity=8) as c:
        c.load_positions(x, y)
        for th in (8, 40, 300, 8):
            c.set_leaf_capacity(th)
            c.advance_tick()
            c.query(k=16)
            ids, d2, cnt, _ = c.fetch()
            assert np.array_equal(ids, exp[0]) and np.array_equal(bits(d2), bits(exp[1])), th
            assert c.stats()["leaf_capacity"] == th
        with pytest.raises(binding.MknnError) as e:
            c.set_leaf_capacity(2)
        assert e.value.code == -4
        with pytest.raises(binding.MknnError) as e:
            c.set_leaf_capacity(0)
        assert e.value.code == -1


def test_replayed_graph_reports_bad_device_coordinate():
    """A bad device coordinate seen by a replayed graph is reported at the
    next synchronisation even after later eager ticks, and once reported the
    context carries on."""
    w = workloads.clustered_1m(n=20_000, ticks=1)
    x, y, _, _, _ = w.tick(0)
    k = 8
    exp = oracle.brute_knn(x, y, k=k, threads=16)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dx, dy = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
        c = binding.Context(w.n, w.n, k, leaf_capacity=16, stream=s.cuda_stream)
        c.load_positions(dx, dy)
        c.advance_tick()
        c.query(k=k)
        c.sync()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            c.load_positions(dx, dy)
            c.advance_tick()
            c.query(k=k)
        # eager ticks after the capture move the context's tags on
        for _ in range(2):
            c.load_positions(x, y)
            c.advance_tick()
            c.query(k=k)
        c.sync()
        dx[5] = 2.0
        g.replay()
        with pytest.raises(binding.MknnError) as e:
            c.sync()
        assert e.value.code == -2
        dx[5] = float(x[5])
        g.replay()
        ids, d2, cnt, _ = c.fetch()
        assert np.array_equal(ids, exp[0]) and np.array_equal(bits(d2), bits(exp[1]))
        del g
        c.close()
