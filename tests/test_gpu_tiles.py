"""GPU parity of the lane flavour's query tiles (mknn_schedule.tile_queries:
64, 32, 16 or 8 queries per wavefront, or automatic), bit for bit against
the oracle (brute force, Definition 1): every tile size over the input
families and sizes that fill one round of wavefronts or several, ragged
last tiles, issuer subsets with variable k, free centres, per-class
launches, and the automatic choice."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding
from tests.helpers import family
from tests.test_gpu_parity import assert_rows_equal, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("kind,n,seed", [("clustered", 70_001, 301), ("uniform", 5_003, 302),
                                         ("duplicates", 777, 303), ("uniform", 2, 304)])
def test_every_tile_size(kind, n, seed):
    x, y = family(kind, n, seed)
    for k in (8, 32, 64):
        exp = oracle.brute_knn(x, y, k=k, threads=16)
        with binding.Context(n, n, k, leaf_capacity=24) as c:
            c.load_positions(x, y)
            c.advance_tick()
            for tq in (0, 8, 16, 32, 64):
                c.set_schedule(sweep="lane", tile_queries=tq)
                c.query(k=k)
                say("tiles %s n=%d k=%d tq=%d" % (kind, n, k, tq))
                assert_rows_equal(c.fetch(), exp, "%s n=%d k=%d tq=%d" % (kind, n, k, tq))


@pytest.mark.parametrize("group_k", [False, True])
def test_subsets_variable_k_and_classes(group_k):
    x, y = family("clustered", 20_000, 305)
    rng = np.random.default_rng(306)
    iss = rng.choice(len(x), 3001, replace=False).astype(np.int32)
    ks = rng.choice([1, 5, 8, 16, 30, 32], len(iss)).astype(np.int32)
    exp = oracle.brute_knn(x, y, issuers=iss, ks=ks, threads=16)
    with binding.Context(len(x), len(iss), 32, leaf_capacity=32) as c:
        c.load_positions(x, y)
        c.advance_tick()
        for tq in (0, 8, 32):
            c.set_schedule(sweep="lane", tile_queries=tq, group_k=group_k)
            c.query(issuers=iss, ks=ks)
            say("tiles subset tq=%d group_k=%s" % (tq, group_k))
            assert_rows_equal(c.fetch(), exp, "subset tq=%d group_k=%s" % (tq, group_k))


def test_free_centres():
    x, y = family("clustered", 9000, 307)
    rng = np.random.default_rng(308)
    m = 1234
    qx = rng.random(m, dtype=np.float32)
    qy = rng.random(m, dtype=np.float32)
    ex = rng.integers(-1, len(x), m).astype(np.int32)
    exp = oracle.brute_knn_points(x, y, qx, qy, exclude=ex, k=16, threads=16)
    with binding.Context(len(x), m, 16, leaf_capacity=32) as c:
        c.load_positions(x, y)
        c.advance_tick()
        for tq in (0, 8, 16, 64):
            c.set_schedule(sweep="lane", tile_queries=tq)
            c.query_points(qx, qy, exclude=ex, k=16)
            say("tiles free centres tq=%d" % tq)
            assert_rows_equal(c.fetch(), exp, "free centres tq=%d" % tq)
