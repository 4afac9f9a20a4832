"""CPU: the vectorized per-row invariant check used on the largest GPU
workloads accepts the oracle's exact answer and rejects planted mistakes
(a swapped pair, a d2 off by one ulp, the issuer in its own row, a
duplicate, a wrong count)."""
import numpy as np
import pytest

import oracle
from tests.helpers import check_rows_vectorized, family


@pytest.fixture(scope="module")
def exact():
    x, y = family("clustered", 1500, 3)
    k = 16
    ids, d2, cnt, _ = oracle.knn(x, y, k=k, th=32)
    return x, y, k, ids, d2, cnt


def test_accepts_the_exact_answer(exact):
    x, y, k, ids, d2, cnt = exact
    check_rows_vectorized(x, y, np.arange(len(x)), ids, d2, cnt, k)
    check_rows_vectorized(x, y, np.arange(100, 400), ids[100:400], d2[100:400], cnt[100:400], k)


def plant(exact, how):
    x, y, k, ids, d2, cnt = exact
    ids, d2, cnt = ids.copy(), d2.copy(), cnt.copy()
    r = 77
    if how == "swap":
        ids[r, [3, 4]] = ids[r, [4, 3]]
        d2[r, [3, 4]] = d2[r, [4, 3]]
    elif how == "ulp":
        d2[r, 5] = np.nextafter(d2[r, 5], np.float32(np.inf))
    elif how == "self":
        ids[r, k - 1] = r
    elif how == "dup":
        ids[r, 6] = ids[r, 5]
        d2[r, 6] = d2[r, 5]
    elif how == "count":
        cnt[r] -= 1
    return x, y, k, ids, d2, cnt


@pytest.mark.parametrize("how", ["swap", "ulp", "self", "dup", "count"])
def test_rejects_planted_mistakes(exact, how):
    x, y, k, ids, d2, cnt = plant(exact, how)
    with pytest.raises(AssertionError):
        check_rows_vectorized(x, y, np.arange(len(x)), ids, d2, cnt, k)


def test_families_replay_across_processes():
    """Every input family draws the same values in a fresh interpreter (the
    seed must not depend on Python's per-process string hash)."""
    import hashlib
    import os
    import subprocess
    import sys

    from tests.helpers import FAMILIES

    def digest_here():
        h = hashlib.sha256()
        for kind in FAMILIES:
            x, y = family(kind, 257, 9)
            h.update(x.tobytes())
            h.update(y.tobytes())
        return h.hexdigest()

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import hashlib\nfrom tests.helpers import FAMILIES, family\nh = hashlib.sha256()\n"
            "for kind in FAMILIES:\n    x, y = family(kind, 257, 9)\n"
            "    h.update(x.tobytes())\n    h.update(y.tobytes())\nprint(h.hexdigest())\n")
    outs = set()
    for salt in ("1", "2"):
        env = dict(os.environ, PYTHONHASHSEED=salt)
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, check=True,
                           capture_output=True, text=True)
        outs.add(r.stdout.strip())
    assert outs == {digest_here()}
