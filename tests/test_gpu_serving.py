"""GPU: serving many scenes with continuous batching.  Every tick computed
in the mix (overlapping with other scenes' ticks, under an HBM budget that
forces evictions and waiting) equals, bit for bit, the same tick computed
alone."""
import numpy as np
import pytest

from paper_1412_6170_amd import binding, serving, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    yield


def make_scenes(count, lo, hi, ticks, seed):
    rng = np.random.default_rng(seed)
    scenes = []
    for sid in range(count):
        n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        k = int(rng.choice([8, 32]))
        w = workloads.clustered_1m(n=n, ticks=ticks)
        pos = []
        for t in range(ticks):
            x, y, _, _, _ = w.tick(t)
            pos.append((torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()))
        scenes.append(serving.Scene(sid, pos, k, leaf_capacity=16))
    return scenes


def alone(scene, tick):
    with binding.Context(scene.n, scene.n, scene.k, leaf_capacity=16) as c:
        x, y = scene.positions[tick]
        c.load_positions(x, y)
        c.advance_tick()
        c.query(k=scene.k, nq=scene.n)
        return c.fetch()


def test_mix_equals_alone_under_budget():
    scenes = make_scenes(8, 10_000, 200_000, 3, seed=1)
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
            a = alone(s, t)
            g = got[(s.sid, t)]
            assert np.array_equal(a[0], g[0]), (s.sid, t)
            assert np.array_equal(a[1].view(np.uint32), g[1].view(np.uint32)), (s.sid, t)
            assert np.array_equal(a[2], g[2])
