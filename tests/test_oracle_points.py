"""Pins of the oracle's free-centre queries (Definition 1: a query is
q = (x, y, k) with any centre in the square; one object may be excluded).
Checks against the numpy definition, against the issuer-centred searches
(which are pinned on their own) and against closed forms."""
import numpy as np
import pytest

import oracle
from helpers import FAMILIES, family, f32


def same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


def centres(kind, nq, seed, x, y):
    """Free centres: uniform, plus some exactly on objects and on the
    square's edges."""
    rng = np.random.default_rng([11, seed, nq])
    qx, qy = rng.random(nq, dtype=np.float32), rng.random(nq, dtype=np.float32)
    on = rng.random(nq) < 0.3
    pick = rng.integers(0, len(x), nq)
    qx[on], qy[on] = x[pick[on]], y[pick[on]]
    edge = rng.random(nq) < 0.1
    qx[edge] = 0.0
    if kind == "tiny_scale":
        qx, qy = (qx * 2.0 ** -64).astype(np.float32), (qy * 2.0 ** -64).astype(np.float32)
    return f32(qx), f32(qy), pick, on


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("k", [1, 8, 33])
def test_points_c_brute_equals_numpy(kind, k):
    x, y = family(kind, 150, 3)
    qx, qy, pick, on = centres(kind, 40, 1, x, y)
    ex = np.where(on, pick, -1).astype(np.int32)
    for excl in (None, ex):
        ci, cd, cc, _ = oracle.brute_knn_points(x, y, qx, qy, exclude=excl, k=k)
        ni, nd, nc = oracle.brute_knn_points_numpy(x, y, qx, qy, exclude=excl, k=k)
        assert np.array_equal(ci, ni) and same_bits(cd, nd) and np.array_equal(cc, nc)


@pytest.mark.parametrize("kind", FAMILIES)
def test_points_on_objects_equal_issuer_queries(kind):
    """A free centre on object s with s excluded is the query issued by s."""
    x, y = family(kind, 300, 5)
    rng = np.random.default_rng(9)
    iss = rng.integers(0, len(x), 60).astype(np.int32)
    ks = rng.integers(1, 40, 60).astype(np.int32)
    pi, pd, pc, po = oracle.brute_knn_points(x, y, x[iss], y[iss], exclude=iss, ks=ks)
    bi, bd, bc, bo = oracle.brute_knn(x, y, issuers=iss, ks=ks)
    assert np.array_equal(po, bo) and np.array_equal(pc, bc)
    assert np.array_equal(pi, bi) and same_bits(pd, bd)
    qi, qd, qc, qo = oracle.knn_points(x, y, x[iss], y[iss], exclude=iss, ks=ks, th=6)
    assert np.array_equal(qi, bi) and same_bits(qd, bd) and np.array_equal(qc, bc)


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("th,L", [(1, 16), (4, 4), (16, 16), (64, 8), (2000, 16)])
def test_points_quadtree_equals_brute(kind, th, L):
    x, y = family(kind, 400, 2)
    qx, qy, pick, on = centres(kind, 80, 4, x, y)
    ex = np.where(on, pick, -1).astype(np.int32)
    for excl in (None, ex):
        bi, bd, bc, _ = oracle.brute_knn_points(x, y, qx, qy, exclude=excl, k=9)
        qi, qd, qc, _ = oracle.knn_points(x, y, qx, qy, exclude=excl, k=9, th=th, L=L)
        assert np.array_equal(qi, bi) and same_bits(qd, bd) and np.array_equal(qc, bc)


def test_points_square_corners_closed_form():
    """Four objects on the corners of a square centred on the query are all
    at d2 = 2 * 0.25^2 = 0.125 (exact); the tie goes by id.  A fifth object
    is farther, at a d2 that exposes the fp32 rounding of 0.9."""
    x = f32([0.75, 0.25, 0.5, 0.25, 0.75])
    y = f32([0.25, 0.75, 0.9, 0.25, 0.75])
    ids, d2, cnt, _ = oracle.brute_knn_points(x, y, f32([0.5]), f32([0.5]), k=5)
    assert list(ids[0]) == [0, 1, 3, 4, 2]
    assert list(d2[0][:4]) == [0.125] * 4
    # 0.5 - fl(0.9) is exact (Sterbenz), then one rounded square; x adds 0.
    dy = np.float32(0.5) - np.float32(0.9)
    assert d2[0][4] == np.float32(dy * dy) and d2[0][4] != np.float32(0.16)
    ids, _, cnt, _ = oracle.brute_knn_points(x, y, f32([0.5]), f32([0.5]), exclude=[1], k=3)
    assert list(ids[0]) == [0, 3, 4] and cnt[0] == 3


def test_points_without_exclusion_keep_the_object_on_the_centre():
    x, y = family("uniform", 50, 1)
    ids, d2, cnt, _ = oracle.brute_knn_points(x, y, x[[7]], y[[7]], k=3)
    assert ids[0][0] == 7 and d2[0][0] == 0.0 and cnt[0] == 3


def test_points_counts_and_padding():
    x, y = f32([0.1, 0.2]), f32([0.1, 0.2])
    ids, d2, cnt, _ = oracle.brute_knn_points(x, y, f32([0.5, 0.5]), f32([0.5, 0.5]),
                                              exclude=[-1, 0], k=4)
    assert list(cnt) == [2, 1]
    assert list(ids[0]) == [1, 0, -1, -1] and list(ids[1]) == [1, -1, -1, -1]
    assert np.isinf(d2[1][1:]).all()
    ids, _, cnt, _ = oracle.knn_points(f32([0.3]), f32([0.3]), f32([0.3]), f32([0.3]),
                                       exclude=[0], k=2, th=1)
    assert cnt[0] == 0 and list(ids[0]) == [-1, -1]


def test_points_validation():
    x, y = family("uniform", 10, 1)
    with pytest.raises(oracle.OracleError) as e:
        oracle.brute_knn_points(x, y, f32([1.0]), f32([0.5]), k=1)
    assert e.value.code == -2
    with pytest.raises(oracle.OracleError) as e:
        oracle.brute_knn_points(x, y, f32([0.5]), f32([0.5]), exclude=[10], k=1)
    assert e.value.code == -1
