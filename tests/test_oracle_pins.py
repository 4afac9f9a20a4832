"""Pins for the CPU oracle: closed forms, brute force on tiny inputs, the
paper's worked example of the leaf order, and invariants.  None of these
re-run the oracle's own formulas; each would fail for a plausible mistake
(a dropped term, a wrong sign or index, a fused multiply-add, flushed
denormals, a wrong tie-break, a wrong split rule)."""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.helpers import FAMILIES, check_invariants, f32, family

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def same(a, b):
    return np.array_equal(np.asarray(a), np.asarray(b))


def same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


# --------------------------------------------------------------------------
# Arithmetic: fp32, no contraction, denormals kept (Definition 1's distance)
# --------------------------------------------------------------------------

def _round_f32(fr):
    """Round an exact rational to the nearest float32 (ties to even)."""
    f = np.float32(float(fr))
    lo, hi = (np.nextafter(f, np.float32(-np.inf)), f) if Fraction(float(f)) > fr else \
        (f, np.nextafter(f, np.float32(np.inf)))
    dlo, dhi = fr - Fraction(float(lo)), Fraction(float(hi)) - fr
    if dlo < dhi:
        return lo
    if dhi < dlo:
        return hi
    return lo if (int(lo.view(np.uint32)) & 1) == 0 else hi


def test_sq_dist_is_not_fused():
    """Find operands where fma(dx,dx,fl(dy*dy)) rounds differently from
    fl(fl(dx*dx)+fl(dy*dy)); the oracle must give the unfused value."""
    rng = np.random.default_rng(3)
    found = 0
    for _ in range(20000):
        q = rng.random(2, dtype=np.float32)
        p = rng.random(2, dtype=np.float32)
        dx = Fraction(float(_round_f32(Fraction(float(q[0])) - Fraction(float(p[0])))))
        dy = Fraction(float(_round_f32(Fraction(float(q[1])) - Fraction(float(p[1])))))
        ay = Fraction(float(_round_f32(dy * dy)))
        ax = Fraction(float(_round_f32(dx * dx)))
        unfused = _round_f32(ax + ay)
        fused = _round_f32(dx * dx + ay)
        if unfused != fused:
            got = oracle.sq_dist(q[0], q[1], p[0], p[1])
            assert got.view(np.uint32) == unfused.view(np.uint32)
            found += 1
            if found >= 5:
                break
    assert found >= 5


def test_sq_dist_keeps_denormals():
    tiny = np.float32(2.0 ** -70)
    got = oracle.sq_dist(0.0, 0.0, tiny, 0.0)
    assert got == np.float32(2.0 ** -140) and got > 0
    # Ranking must see the denormal difference: id 2 is nearer than id 1.
    x = f32([0.0, 2.0 ** -69, 2.0 ** -70])
    y = f32([0.0, 0.0, 0.0])
    ids, d2, cnt, _ = oracle.knn(x, y, k=2, th=1)
    assert ids[0].tolist() == [2, 1]
    ids, d2, cnt, _ = oracle.brute_knn(x, y, k=2)
    assert ids[0].tolist() == [2, 1]


def test_sq_dist_sign_and_terms():
    # Both terms present and differences taken, not sums.
    assert oracle.sq_dist(0.75, 0.5, 0.5, 0.25) == np.float32(0.125)
    assert oracle.sq_dist(0.5, 0.25, 0.75, 0.5) == np.float32(0.125)
    assert oracle.sq_dist(0.5, 0.5, 0.5, 0.25) == np.float32(0.0625)
    assert oracle.sq_dist(0.5, 0.5, 0.25, 0.5) == np.float32(0.0625)


# --------------------------------------------------------------------------
# Morton codes and the index (Sec. 4.1)
# --------------------------------------------------------------------------

def test_morton_known_values():
    s = 1.0 / 65536
    assert oracle.lib().oracle_morton(s, 0.0) == 1          # x cell 1 -> bit 0
    assert oracle.lib().oracle_morton(0.0, s) == 2          # y cell 1 -> bit 1
    assert oracle.lib().oracle_morton(1 - s, 0.0) == 0x55555555
    assert oracle.lib().oracle_morton(0.0, 1 - s) == 0xAAAAAAAA
    assert oracle.lib().oracle_morton(0.5, 0.0) == 1 << 30  # level-1 quadrant 1
    assert oracle.lib().oracle_morton(0.0, 0.5) == 2 << 30  # level-1 quadrant 2
    assert oracle.lib().oracle_morton(0.5, 0.5) == 3 << 30


def test_morton_roundtrip_and_ancestor():
    rng = np.random.default_rng(5)
    cx = rng.integers(0, 65536, 4000)
    cy = rng.integers(0, 65536, 4000)
    codes = oracle.morton_codes((cx / 65536).astype(np.float32), (cy / 65536).astype(np.float32))
    bx = np.zeros_like(cx)
    by = np.zeros_like(cy)
    for b in range(16):
        bx |= ((codes.astype(np.int64) >> (2 * b)) & 1) << b
        by |= ((codes.astype(np.int64) >> (2 * b + 1)) & 1) << b
    assert same(bx, cx) and same(by, cy)
    # Ancestor at level l: the quadrant of the 2^l grid holding the point.
    for lev in (1, 3, 8, 15):
        anc = codes.astype(np.int64) >> (2 * (16 - lev))
        gx = cx >> (16 - lev)
        gy = cy >> (16 - lev)
        ax = np.zeros_like(gx)
        ay = np.zeros_like(gy)
        for b in range(lev):
            ax |= ((anc >> (2 * b)) & 1) << b
            ay |= ((anc >> (2 * b + 1)) & 1) << b
        assert same(ax, gx) and same(ay, gy)


def test_validation_rejects_out_of_square():
    for bad in ([1.0], [-0.5], [np.nan], [np.inf]):
        with pytest.raises(oracle.OracleError) as e:
            oracle.validate(f32(bad), f32([0.0]))
        assert e.value.code == -2
    oracle.validate(f32([-0.0, 0.0, np.float32(1 - 2 ** -24)]), f32([0.0, 0.5, 0.25]))


def _check_index(x, y, th, L):
    ix = oracle.build_index(x, y, th, L)
    n = len(x)
    codes, ids = ix["codes"], ix["ids"]
    # A permutation of the objects, sorted by (Morton code at level L, id):
    # the level-L code is the level-16 code without its 2(16-L) low bits.
    assert same(np.sort(ids), np.arange(n))
    lcode = codes.astype(np.uint64) >> np.uint64(2 * (16 - L))
    key = lcode << np.uint64(32) | ids.astype(np.uint64)
    assert np.all(key[1:] > key[:-1])
    if L == 16:
        full = codes.astype(np.uint64) << np.uint64(32) | ids.astype(np.uint64)
        assert np.all(full[1:] > full[:-1])
    # Leaves tile [0, n) in order and share their quadrant prefix.
    beg, end, lev, pre = ix["leaf_begin"], ix["leaf_end"], ix["leaf_level"], ix["leaf_prefix"]
    if n:
        assert beg[0] == 0 and end[-1] == n and same(beg[1:], end[:-1])
        assert np.all(end > beg)
    c64 = codes.astype(np.int64)
    for b, e, l_, p in zip(beg, end, lev, pre):
        shift = 2 * (16 - l_)
        pref = (c64[b:e] >> shift) if l_ > 0 else np.zeros(e - b, np.int64)
        assert np.all(pref == p)
        # No other object lies in the leaf's quadrant (it is the whole run).
        full = (c64 >> shift) if l_ > 0 else np.zeros(n, np.int64)
        assert np.count_nonzero(full == p) == e - b
        # Split rule: at most th unless at L; the parent held more than th.
        assert (e - b) <= th or l_ == L
        if l_ > 0:
            parent = c64 >> (2 * (16 - l_ + 1)) if l_ > 1 else np.zeros(n, np.int64)
            assert np.count_nonzero(parent == (p >> 2)) > th
    # Prefixes in Morton order along the leaves.
    z = [int(p) << (2 * (16 - int(l_))) if l_ > 0 else 0 for p, l_ in zip(pre, lev)]
    assert z == sorted(z)
    return ix


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("th,L", [(1, 16), (4, 4), (16, 16), (64, 1), (8, 12), (3, 13), (3000, 16)])
def test_index_structure(kind, th, L):
    x, y = family(kind, 700, 1)
    _check_index(x, y, th, L)


def _parse_pairs(s):
    return [tuple(int(v) for v in m) for m in re.findall(r"\((\d+),(\d+)\)", s)]


def test_paper_worked_example_leaf_order():
    """Fig. 2 / Sec. 4.2.2 example: with quadrants 1 and 2 split at level 1,
    the leaves in z'' order and the left/right sub-visits from (2,5)."""
    gold = {}
    with open(os.path.join(GOLDEN, "worked_example_leaves.txt")) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            gold[k.strip()] = _parse_pairs(v)
    # th = 3: quadrants 1 and 2 get one object in each level-2 child (4 > 3:
    # split), quadrants 0 and 3 get two objects each (kept as leaves).
    pts = []
    q = 0.25
    for qx0, qy0 in ((0.5, 0.0), (0.0, 0.5)):           # level-1 quadrants 1, 2
        for cx, cy in ((0, 0), (1, 0), (0, 1), (1, 1)):  # their four children
            pts.append((qx0 + cx * q + 0.1, qy0 + cy * q + 0.1))
    pts += [(0.1, 0.1), (0.3, 0.2), (0.6, 0.6), (0.8, 0.9)]  # quadrants 0 and 3
    x = f32([p[0] for p in pts])
    y = f32([p[1] for p in pts])
    ix = _check_index(x, y, 3, 16)
    lev, pre = ix["leaf_level"], ix["leaf_prefix"]
    l_deep = int(lev.max())
    assert l_deep == 2
    labels = [(int(l_), int(p) * 4 ** (l_deep - int(l_))) for l_, p in zip(lev, pre)]
    assert labels == gold["leaves"]
    i = labels.index(gold["start"][0])
    assert labels[i + 1:] == gold["right"]
    assert labels[:i][::-1] == gold["left"]


def test_paper_leaf_capacity_rule():
    # Sec. 6, study S2: th = 192 for k < 32, 12k for 32 <= k <= 128 (the
    # paper's 384 at k = 32, Sec. 6 query-rate study), 2048 for larger k.
    assert oracle.default_leaf_capacity(8) == 192
    assert oracle.default_leaf_capacity(31) == 192
    assert oracle.default_leaf_capacity(32) == 384
    assert oracle.default_leaf_capacity(128) == 1536
    assert oracle.default_leaf_capacity(129) == 2048


# --------------------------------------------------------------------------
# Whole result: brute force (the definition) on tiny inputs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("k", [1, 2, 7, 8, 32])
def test_c_brute_equals_numpy_definition(kind, k):
    x, y = family(kind, 600, 2)
    ni, nd, nc = oracle.brute_knn_numpy(x, y, k=k)
    ci, cd, cc, _ = oracle.brute_knn(x, y, k=k, threads=4)
    assert same(ni, ci) and same_bits(nd, cd) and same(nc, cc)


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("th,L", [(1, 16), (4, 4), (16, 16), (64, 8), (2000, 16), (5, 1)])
def test_quadtree_oracle_equals_brute(kind, th, L):
    x, y = family(kind, 900, 3)
    for k in (1, 8, 33, 64):
        bi, bd, bc, _ = oracle.brute_knn(x, y, k=k, threads=4)
        qi, qd, qc, _ = oracle.knn(x, y, k=k, th=th, L=L, threads=4)
        assert same(bi, qi) and same_bits(bd, qd) and same(bc, qc), (kind, th, L, k)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 40])
def test_small_n_and_large_k(n):
    x, y = family("uniform", n, 4)
    for k in (1, n - 1, n, n + 5):
        if k < 1:
            continue
        ni, nd, nc = oracle.brute_knn_numpy(x, y, k=k)
        qi, qd, qc, _ = oracle.knn(x, y, k=k, th=2)
        assert same(ni, qi) and same_bits(nd, qd) and same(nc, qc)
        assert np.all(qc == min(k, n - 1))


def test_subset_and_variable_k():
    x, y = family("clustered", 1500, 5)
    rng = np.random.default_rng(9)
    iss = rng.choice(1500, 400, replace=False).astype(np.int32)
    ks = rng.choice([1, 8, 16, 32, 64], 400).astype(np.int32)
    bi, bd, bc, bo = oracle.brute_knn(x, y, issuers=iss, ks=ks)
    qi, qd, qc, qo = oracle.knn(x, y, issuers=iss, ks=ks, th=24)
    assert same(bi, qi) and same_bits(bd, qd) and same(bc, qc) and same(bo, qo)
    for q in (0, 17, 399):
        s, kq = iss[q], ks[q]
        ni, nd, nc = oracle.brute_knn_numpy(x, y, issuers=[s], k=int(kq))
        assert same(ni[0], qi[qo[q]:qo[q + 1]]) and same_bits(nd[0], qd[qo[q]:qo[q + 1]])
    check_invariants(x, y, iss, ks, qi, qd, qc, offsets=qo)


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------

def _lattice_expected(ix0, iy0, side, k):
    """Neighbours of lattice point (ix0, iy0) by exact integer squared norm,
    ties by row-major id; d2 = norm * 2^-14 exactly (spacing 2^-7)."""
    cand = []
    r = 8
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dx == 0 and dy == 0:
                continue
            ix, iy = ix0 + dx, iy0 + dy
            if 0 <= ix < side and 0 <= iy < side:
                cand.append((dx * dx + dy * dy, iy * side + ix))
    cand.sort()
    return cand[:k]


def test_lattice_shells_and_id_ties():
    side = 128
    iy, ix = np.divmod(np.arange(side * side), side)
    x = (ix * 2.0 ** -7).astype(np.float32)
    y = (iy * 2.0 ** -7).astype(np.float32)
    with open(os.path.join(GOLDEN, "lattice_shells.txt")) as f:
        cum = [int(v) for line in f if line.startswith("cumulative")
               for v in line.split(":")[1].split()]
    assert cum == [4, 8, 12, 20, 24, 28, 36]
    s = 64 * side + 64
    for k in (4, 8, 12, 20, 24, 28, 32, 36):
        ids, d2, cnt, _ = oracle.knn(x, y, issuers=[s], k=k, th=48)
        exp = _lattice_expected(64, 64, side, k)
        assert ids[0].tolist() == [e[1] for e in exp]
        assert same_bits(d2[0], np.array([e[0] * 2.0 ** -14 for e in exp], np.float32))
    # k = 32: the 28 points through norm 9 plus the 4 lowest ids at norm 10,
    # i.e. offsets (dx,dy) = (-1,-3), (+1,-3), (-3,-1), (+3,-1).
    ids, _, _, _ = oracle.knn(x, y, issuers=[s], k=32, th=48)
    tail = [(i % side - 64, i // side - 64) for i in ids[0][28:]]
    assert tail == [(-1, -3), (1, -3), (-3, -1), (3, -1)]


def test_all_identical_positions():
    n = 300
    x = np.full(n, 0.375, np.float32)
    y = np.full(n, 0.625, np.float32)
    for th in (1, 16, 1000):
        ids, d2, cnt, _ = oracle.knn(x, y, k=10, th=th)
        for s in (0, 5, 299):
            exp = [j for j in range(n) if j != s][:10]
            assert ids[s].tolist() == exp and np.all(d2[s] == 0)


def test_collinear_closed_form():
    n = 200
    x = (np.arange(n) * 2.0 ** -16).astype(np.float32)
    y = np.full(n, 0.5, np.float32)
    ids, d2, cnt, _ = oracle.knn(x, y, k=6, th=4)
    for s in (0, 1, 100, 199):
        exp = sorted(((m - s) ** 2, m) for m in range(n) if m != s)[:6]
        assert ids[s].tolist() == [e[1] for e in exp]
        assert same_bits(d2[s], np.array([e[0] * 2.0 ** -32 for e in exp], np.float32))
    assert ids[100].tolist() == [99, 101, 98, 102, 97, 103]


def test_degenerate_sizes():
    ids, d2, cnt, _ = oracle.knn(f32([0.5]), f32([0.5]), k=3)
    assert cnt.tolist() == [0] and ids.tolist() == [[-1, -1, -1]] and np.all(np.isinf(d2))
    ids, d2, cnt, _ = oracle.knn(f32([0.5, 0.25]), f32([0.5, 0.5]), k=3)
    assert ids.tolist() == [[1, -1, -1], [0, -1, -1]] and cnt.tolist() == [1, 1]
    assert d2[0][0] == np.float32(0.0625)


# --------------------------------------------------------------------------
# Invariants on a mid-size clustered case (no brute force needed)
# --------------------------------------------------------------------------

def test_invariants_mid_size():
    x, y = family("clustered", 4000, 6)
    ids, d2, cnt, _ = oracle.knn(x, y, k=16, th=40, threads=4)
    check_invariants(x, y, None, None, ids, d2, cnt, k=16)
    # Sampled brute force.
    sample = np.arange(0, 4000, 97)
    ni, nd, nc = oracle.brute_knn_numpy(x, y, issuers=sample, k=16)
    assert same(ni, ids[sample]) and same_bits(nd, d2[sample])


def test_invariant_checker_catches_planted_mistakes():
    """The invariant checker must reject an oracle-style result with a
    planted error (here applied to a copy of the oracle output)."""
    x, y = family("uniform", 500, 7)
    ids, d2, cnt, _ = oracle.knn(x, y, k=8, th=16)
    bad = ids.copy()
    bad[3, [2, 3]] = bad[3, [3, 2]]           # swapped order
    with pytest.raises(AssertionError):
        check_invariants(x, y, None, None, bad, d2, cnt, k=8)
    bad = ids.copy()
    bad[4, 0] = 4                              # self included
    with pytest.raises(AssertionError):
        check_invariants(x, y, None, None, bad, d2, cnt, k=8)
