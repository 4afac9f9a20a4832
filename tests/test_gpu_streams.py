"""GPU: device inputs produced on the caller's current torch stream.  A
context runs on a stream of its own, so the binding must make that stream
wait for the work already enqueued on the caller's stream before the
library reads the inputs.  Here the caller's stream is held busy by a
bounded spin kernel and the inputs are written after it: reading them
early would index stale positions or issuers and give the wrong rows."""
import numpy as np
import pytest

import oracle
from paper_1412_6170_amd import binding
from tests.helpers import family

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPIN_CYCLES = 20_000_000   # a few ms to a few hundred ms of one busy kernel


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    yield


def say(*a):
    print(*a, flush=True)


def bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def test_positions_written_on_the_current_stream():
    n, k = 5000, 8
    x0, y0 = family("uniform", n, 41)
    x1, y1 = family("clustered", n, 42)
    xd, yd = torch.from_numpy(x0).cuda(), torch.from_numpy(y0).cuda()
    x1d, y1d = torch.from_numpy(x1).cuda(), torch.from_numpy(y1).cuda()
    torch.cuda.synchronize()
    say("streams: positions written after a spin on the current stream")
    with binding.Context(n, n, k) as c:
        assert c.stream.cuda_stream != torch.cuda.current_stream().cuda_stream
        torch.cuda._sleep(SPIN_CYCLES)
        xd.copy_(x1d)
        yd.copy_(y1d)
        c.load_positions(xd, yd)
        c.advance_tick()
        c.query(k=k)
        ids, d2, cnt, _ = c.fetch()
    ei, ed, ec, _ = oracle.brute_knn(x1, y1, k=k, threads=16)
    assert np.array_equal(cnt, ec)
    assert np.array_equal(ids, ei) and np.array_equal(bits(d2), bits(ed))


def test_issuers_written_on_the_current_stream():
    n, k = 5000, 8
    x, y = family("uniform", n, 43)
    rng = np.random.default_rng(44)
    first = rng.permutation(n)[:1000].astype(np.int32)
    second = rng.permutation(n)[:1000].astype(np.int32)
    iss = torch.from_numpy(first).cuda()
    iss2 = torch.from_numpy(second).cuda()
    torch.cuda.synchronize()
    say("streams: issuers written after a spin on the current stream")
    with binding.Context(n, n, k) as c:
        c.load_positions(x, y)
        c.advance_tick()
        torch.cuda._sleep(SPIN_CYCLES)
        iss.copy_(iss2)
        c.query(k=k, issuers=iss)
        ids, d2, cnt, _ = c.fetch()
    ei, ed, ec, _ = oracle.brute_knn(x, y, issuers=second, k=k, threads=16)
    assert np.array_equal(cnt, ec)
    assert np.array_equal(ids, ei) and np.array_equal(bits(d2), bits(ed))


def test_stream_handles():
    """A null handle gets a stream of its own (the library would otherwise
    create one the binding cannot order against); a raw handle of a torch
    stream runs the context on that stream."""
    x, y = family("uniform", 300, 45)
    with binding.Context(300, 300, 4, stream=torch.cuda.current_stream().cuda_stream) as c:
        if torch.cuda.current_stream().cuda_stream == 0:
            assert c.stream.cuda_stream != 0
        c.load_positions(x, y)
        c.advance_tick()
        c.query(k=4)
        a = c.fetch()
    s = torch.cuda.Stream()
    with binding.Context(300, 300, 4, stream=s.cuda_stream) as c:
        assert c.stream.cuda_stream == s.cuda_stream
        c.load_positions(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
        c.advance_tick()
        c.query(k=4)
        b = c.fetch()
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(np.asarray(u).view(np.uint8), np.asarray(v).view(np.uint8))


def test_host_inputs_may_be_reused_when_the_call_returns():
    """Host arrays are read before a query call returns, even while the
    context's stream is still busy with earlier work: the caller may
    overwrite them at once."""
    n, k = 5000, 8
    x, y = family("uniform", n, 46)
    rng = np.random.default_rng(47)
    iss = rng.permutation(n)[:1000].astype(np.int32)
    first = iss.copy()
    cx = rng.random(700, dtype=np.float32)
    cy = rng.random(700, dtype=np.float32)
    centres = (cx.copy(), cy.copy())
    say("streams: host inputs overwritten right after the call")
    with binding.Context(n, n, k) as c:
        c.load_positions(x, y)
        c.advance_tick()
        with torch.cuda.stream(c.stream):
            torch.cuda._sleep(SPIN_CYCLES)
        c.query(k=k, issuers=iss)
        iss[:] = rng.permutation(n)[:1000]
        ids, d2, cnt, _ = c.fetch()
        ei, ed, ec, _ = oracle.brute_knn(x, y, issuers=first, k=k, threads=16)
        assert np.array_equal(cnt, ec)
        assert np.array_equal(ids, ei) and np.array_equal(bits(d2), bits(ed))
        with torch.cuda.stream(c.stream):
            torch.cuda._sleep(SPIN_CYCLES)
        c.query_points(cx, cy, k=k)
        cx[:] = 0.5
        cy[:] = 0.5
        pids, pd2, pcnt, _ = c.fetch()
    ei, ed, ec, _ = oracle.brute_knn_points(x, y, centres[0], centres[1], k=k)
    assert np.array_equal(pcnt, ec)
    assert np.array_equal(pids, ei) and np.array_equal(bits(pd2), bits(ed))
