"""GPU: parts of the C ABI the binding's own calls do not reach --
mknn_fetch into device buffers (uniform k, whose row offsets the library
writes from the host, and variable k) and the device memory mknn_create
takes against mknn_footprint."""
import ctypes

import numpy as np
import pytest

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


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def fetch_to_device(ctx):
    nq, ne = ctx.result_size()
    ids = torch.full((max(ne, 1),), -7, dtype=torch.int32, device="cuda")
    d2 = torch.full((max(ne, 1),), -7.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((max(nq, 1),), -7, dtype=torch.int32, device="cuda")
    off = torch.full((nq + 1,), -7, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    rc = binding.lib().mknn_fetch(ctx._h, ptr(ids), ptr(d2), ptr(cnt), ptr(off),
                                  binding.MKNN_DEVICE)
    assert rc == 0, binding.lib().mknn_last_error(ctx._h)
    return (ids[:ne].cpu().numpy(), d2[:ne].cpu().numpy(), cnt[:nq].cpu().numpy(),
            off.cpu().numpy())


def same_bytes(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                          np.ascontiguousarray(b).view(np.uint8))


@pytest.mark.parametrize("variable_k", [False, True])
def test_fetch_into_device_buffers(variable_k):
    n, k = 6000, 16
    x, y = family("clustered", n, 51)
    rng = np.random.default_rng(52)
    say("api: device fetch, variable k=%s" % variable_k)
    with binding.Context(n, n, k) as c:
        c.load_positions(x, y)
        c.advance_tick()
        if variable_k:
            iss = rng.permutation(n)[:2500].astype(np.int32)
            ks = rng.integers(1, k + 1, len(iss)).astype(np.int32)
            c.query(issuers=iss, ks=ks)
        else:
            c.query(k=k)
        hi, hd, hc, ho = c.fetch()
        di, dd, dc, do = fetch_to_device(c)
    assert same_bytes(np.ravel(hi), di) and same_bytes(np.ravel(hd), dd) and same_bytes(hc, dc)
    if variable_k:
        assert same_bytes(ho, do)
    else:
        assert np.array_equal(do, np.arange(n + 1, dtype=np.int64) * k)


def test_create_takes_the_reported_footprint():
    n, k, th = 4_000_000, 32, 64
    fp = binding.footprint(n_max=n, k_max=k, leaf_capacity=th)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    c = binding.Context(n, n, k, leaf_capacity=th)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    c.close()
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    taken, given_back = free0 - free1, free2 - free1
    say("api: footprint %d B, create took %d B, destroy gave back %d B" % (fp, taken, given_back))
    # Large buffers are mapped in whole 2 MiB pages, which the footprint
    # counts; the few small ones may come from memory the runtime holds.
    # The runtime may keep a few MiB mapped after buffers are freed (by
    # earlier tests of the same process, or by this one), and a later
    # create can take its buffers from there.
    held = 16 << 20
    assert fp - held <= taken <= fp + (4 << 20)
    assert given_back >= taken - held


def test_readme_python_example():
    """The Python usage example in README.md runs as written and returns
    the exact rows."""
    import os
    import re
    import oracle
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "README.md")).read()
    block = re.search(r"```python\n(.*?)```", text, re.S).group(1)
    n = 3000
    x, y = family("clustered", n, 53)
    env = {"n": n, "x": x, "y": y}
    exec(compile(block, "README.md", "exec"), env)
    ei, ed, ec, _ = oracle.brute_knn(x, y, k=32, threads=16)
    assert np.array_equal(env["ids"], ei) and np.array_equal(env["counts"], ec)
    assert same_bytes(env["d2"], ed)


def test_autotuner_picks_a_timed_candidate_and_results_stay_exact():
    """binding.autotune_leaf_capacity times every candidate with the
    library's events, returns the fastest, leaves the context at it, and
    the ticks before and after tuning give the exact rows (the leaf
    capacity changes only the time)."""
    import oracle
    from paper_1412_6170_amd import workloads
    w = workloads.clustered_1m(n=60_000, ticks=4)
    k = 16
    dev = []
    for t in range(w.ticks):
        x, y, _, _, _ = w.tick(t)
        dev.append((x, y, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()))
    cands = (16, 64, 256)
    with binding.Context(w.n, w.n, k, leaf_capacity=min(cands), timing=True) as c:
        def run_tick(i):
            _, _, xd, yd = dev[i % len(dev)]
            c.load_positions(xd, yd)
            c.advance_tick()
            c.query(k=k)

        best, times = binding.autotune_leaf_capacity(c, run_tick, cands, repeats=2)
        say("api: autotuner chose %d from %s" % (best, times))
        assert best in cands and set(times) == set(cands)
        assert all(v > 0 for v in times.values()) and times[best] == min(times.values())
        run_tick(1)
        ids, d2, cnt, _ = c.fetch()
        assert c.stats()["leaf_capacity"] == best
    x, y = dev[1][0], dev[1][1]
    sample = np.arange(0, w.n, 101, dtype=np.int32)
    ei, ed, ec, _ = oracle.brute_knn(x, y, issuers=sample, k=k, threads=16)
    assert np.array_equal(ids[sample], ei) and same_bytes(d2[sample], ed)
    assert np.array_equal(cnt[sample], ec)


def test_knn_tick_helper():
    import oracle
    x, y = family("duplicates", 2500, 54)
    rng = np.random.default_rng(55)
    iss = rng.permutation(2500)[:700].astype(np.int32)
    ks = rng.integers(1, 20, len(iss)).astype(np.int32)
    got = binding.knn_tick(x, y, issuers=iss, ks=ks)
    exp = oracle.brute_knn(x, y, issuers=iss, ks=ks, threads=16)
    for u, v in zip(got[:3], exp[:3]):
        assert same_bytes(np.asarray(u), np.asarray(v))
    assert np.array_equal(got[3], exp[3])


def test_two_contexts_on_two_host_threads():
    """Separate contexts are independent: two host threads, each with its
    own context, run ticks at the same time and both get the exact rows."""
    import threading
    import oracle
    inputs = [family(kind, 8000, 56 + i) for i, kind in enumerate(("clustered", "uniform"))]
    got = [None, None]
    errors = []

    def worker(i):
        try:
            x, y = inputs[i]
            with binding.Context(len(x), len(x), 8) as c:
                for _ in range(3):
                    c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
                    c.advance_tick()
                    c.query(k=8)
                    got[i] = c.fetch()
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in threads) and not errors, errors
    for i, (x, y) in enumerate(inputs):
        ei, ed, ec, _ = oracle.brute_knn(x, y, k=8, threads=16)
        assert np.array_equal(got[i][0], ei) and same_bytes(got[i][1], ed)
        assert np.array_equal(got[i][2], ec)
