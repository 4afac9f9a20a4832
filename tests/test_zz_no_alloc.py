"""GPU tests of the no-allocation entry point (mknn_knn_noalloc), called
through the C ABI: its rows equal, bit for bit, those of the context path
it is a variant of (mknn_load_positions, mknn_advance_tick, mknn_query with
every object querying, mknn_fetch), on calls in a row whose second input is
smaller than the first, so stale contents of the shared scratch array
would show; for lane lists and wavefront lists; plus the host-checked
errors and the device status word.  The oracle (Definition 1) checks the
small inputs too."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding
from tests.helpers import family

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


def context_rows(x, y, k, th):
    with binding.Context(len(x), len(x), k, leaf_capacity=th, max_level=16) as c:
        c.load_positions(x, y)
        c.advance_tick()
        c.query(k=k)
        ids, d2, cnt, _ = c.fetch()
    return ids, d2, cnt


def noalloc_rows(x, y, k, th):
    """Outputs are pre-filled with garbage, so rows the call does not write
    would show."""
    n = len(x)
    dx = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    dy = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    ids = torch.full((n * k,), -7, dtype=torch.int32, device="cuda")
    d2 = torch.full((n * k,), 7.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    binding.knn_noalloc(dx, dy, k, ids, d2, cnt, st, leaf_capacity=th)
    torch.cuda.synchronize()
    return (ids.cpu().numpy().reshape(n, k), d2.cpu().numpy().reshape(n, k), cnt.cpu().numpy(),
            int(st.cpu().item()))


def assert_same(got, exp, what):
    gi, gd, gc = got[:3]
    ei, ed, ec = exp[:3]
    assert np.array_equal(gi, ei), what + ": ids differ"
    assert np.array_equal(gd.view(np.uint32), ed.view(np.uint32)), what + ": d2 differ"
    assert np.array_equal(gc, ec), what + ": counts differ"


@pytest.mark.parametrize("k,th", [(8, 0), (32, 16), (64, 32), (200, 64)])
def test_noalloc_equals_context_path_on_calls_in_a_row(k, th):
    cases = (("clustered", 60000, 81), ("uniform", 7000, 82), ("duplicates", 3000, 83))
    for kind, n, seed in cases:
        x, y = family(kind, n, seed)
        say("noalloc %s n=%d k=%d th=%d" % (kind, n, k, th))
        got = noalloc_rows(x, y, k, th)
        assert got[3] == 0, "status %d" % got[3]
        assert_same(got, context_rows(x, y, k, th), "%s n=%d k=%d" % (kind, n, k))
        if n <= 7000:
            oi, od, oc, _ = oracle.brute_knn(x, y, k=k, threads=16)
            assert_same(got, (oi, od, oc), "oracle %s n=%d k=%d" % (kind, n, k))


def test_noalloc_largest_size_then_tiny():
    x, y = family("clustered", binding.NOALLOC_MAX_N, 84)
    say("noalloc n=%d k=16" % len(x))
    got = noalloc_rows(x, y, 16, 0)
    assert got[3] == 0
    assert_same(got, context_rows(x, y, 16, 0), "largest n")
    for n in (1, 2, 5):
        x, y = family("uniform", n, 85)
        got = noalloc_rows(x, y, 4, 0)
        assert got[3] == 0
        assert_same(got, oracle.brute_knn(x, y, k=4)[:3], "n=%d" % n)


def test_noalloc_errors_and_status():
    n, k = 1000, 8
    x, y = family("uniform", n, 86)
    dx = torch.from_numpy(x).cuda()
    dy = torch.from_numpy(y).cuda()
    ids = torch.empty(n * k, dtype=torch.int32, device="cuda")
    d2 = torch.empty(n * k, dtype=torch.float32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    L = binding.lib()
    vp = binding._vp
    args = [vp(dx.data_ptr()), vp(dy.data_ptr()), n, k, 0, vp(ids.data_ptr()),
            vp(d2.data_ptr()), vp(cnt.data_ptr()), vp(st.data_ptr()), None]
    for i, bad in ((3, 0), (3, 1025), (4, -1), (2, -1), (5, None)):
        a = list(args)
        a[i] = bad
        assert L.mknn_knn_noalloc(*a) == -1
    a = list(args)
    a[2] = binding.NOALLOC_MAX_N + 1
    assert L.mknn_knn_noalloc(*a) == -4
    a = list(args)
    a[4] = 1   # a leaf capacity of 1 needs node tables larger than the array
    a[2] = binding.NOALLOC_MAX_N
    big = torch.zeros(binding.NOALLOC_MAX_N, dtype=torch.float32, device="cuda")
    a[0] = a[1] = vp(big.data_ptr())
    assert L.mknn_knn_noalloc(*a) == -4
    # n = 0: nothing to do, status 0.
    a = list(args)
    a[2] = 0
    assert L.mknn_knn_noalloc(*a) == 0
    torch.cuda.synchronize()
    assert int(st.cpu().item()) == 0
    # A coordinate outside [0,1) is found on the device: status MKNN_E_RANGE.
    bx = dx.clone()
    bx[17] = 1.5
    st.fill_(99)
    binding.knn_noalloc(bx, dy, k, ids, d2, cnt, st)
    torch.cuda.synchronize()
    assert int(st.cpu().item()) == -2
    # The next good call is exact again.
    got = noalloc_rows(x, y, k, 0)
    assert got[3] == 0
    assert_same(got, context_rows(x, y, k, 0), "after a bad call")
