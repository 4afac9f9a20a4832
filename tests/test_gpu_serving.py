"""GPU: serving many scenes with continuous batching.  Every tick computed
in the mix (overlapping with other scenes' ticks, under an HBM budget that
forces evictions and waiting) equals, bit for bit, the oracle's answer for
that tick and the same tick computed alone.  The mix holds scenes from 10k
objects up to one of 2M objects (the largest scene size of the serving
workload), with k in {8, 32}."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding, serving, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    yield


def make_scenes(count, lo, hi, ticks, seed, extra=()):
    """count scenes of log-uniform size in [lo, hi], then one scene per
    (n, k) in extra; host positions are kept for the oracle."""
    rng = np.random.default_rng(seed)
    sizes = [(int(round(np.exp(rng.uniform(np.log(lo), np.log(hi))))), int(rng.choice([8, 32])))
             for _ in range(count)] + list(extra)
    scenes, host = [], {}
    for sid, (n, k) in enumerate(sizes):
        w = workloads.clustered_1m(n=n, ticks=ticks)
        pos = []
        for t in range(ticks):
            x, y, _, _, _ = w.tick(t)
            host[(sid, t)] = (x, y)
            pos.append((torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()))
        scenes.append(serving.Scene(sid, pos, k, leaf_capacity=16))
    return scenes, host


def alone(scene, tick):
    with binding.Context(scene.n, scene.n, scene.k, leaf_capacity=16) as c:
        x, y = scene.positions[tick]
        c.load_positions(x, y)
        c.advance_tick()
        c.query(k=scene.k, nq=scene.n)
        return c.fetch()


def test_mix_equals_oracle_and_alone_under_budget():
    scenes, host = make_scenes(7, 10_000, 200_000, 3, seed=1, extra=[(2_000_000, 32)])
    total = sum(s.footprint for s in scenes)
    budget = max(max(s.footprint for s in scenes), total // 3)
    got = {}

    def keep(r):
        got[(r.scene.sid, r.tick)] = r.scene.ctx.fetch()

    srv = serving.Server(scenes, hbm_budget=budget, slots=4, on_complete=keep)
    arrivals = serving.poisson_arrivals([s.sid for s in scenes], 3, rate=2000.0, seed=2)
    done = srv.run(arrivals)
    srv.close()
    assert len(done) == len(arrivals) == len(got)
    assert srv.evictions > 0
    summary = serving.summarize(done, {s.sid: s for s in scenes})
    print(summary, "admissions", srv.admissions, "evictions", srv.evictions, flush=True)
    for s in scenes:
        for t in range(3):
            print("scene %d (n=%d, k=%d) tick %d" % (s.sid, s.n, s.k, t), flush=True)
            g = got.pop((s.sid, t))
            x, y = host[(s.sid, t)]
            e = oracle.knn(x, y, k=s.k, threads=16)
            assert np.array_equal(e[0], g[0]), ("oracle ids", s.sid, t)
            assert np.array_equal(e[1].view(np.uint32), g[1].view(np.uint32)), ("oracle d2", s.sid, t)
            assert np.array_equal(e[2], g[2]), ("oracle counts", s.sid, t)
            a = alone(s, t)
            assert np.array_equal(a[0], g[0]), (s.sid, t)
            assert np.array_equal(a[1].view(np.uint32), g[1].view(np.uint32)), (s.sid, t)
            assert np.array_equal(a[2], g[2])
