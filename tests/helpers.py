"""Shared test helpers: small seeded input families and result checks.

The checks here restate properties of the exact k-NN result (Definition 1 of
arXiv 1412.6170 with ties broken by ascending id); they do not call the
oracle, so they can pin it.
"""
import zlib

import numpy as np

CLAMP_HI = np.float32(1.0 - 2.0 ** -24)


def f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def family(kind, n, seed):
    """Tiny input families that stress different parts of the search.  The
    seed mixes in a CRC of the family name (stable across processes, unlike
    Python's salted str hash), so every input replays from its seed."""
    rng = np.random.default_rng([7, seed, n, zlib.crc32(kind.encode()) % 1000])
    if kind == "uniform":
        x, y = rng.random(n, dtype=np.float32), rng.random(n, dtype=np.float32)
    elif kind == "clustered":
        c = rng.random((3, 2))
        w = rng.integers(0, 3, n)
        p = c[w] + rng.normal(0, 0.003, (n, 2))
        x, y = np.clip(p[:, 0], 0, CLAMP_HI), np.clip(p[:, 1], 0, CLAMP_HI)
    elif kind == "duplicates":
        base = rng.random((max(1, n // 7), 2), dtype=np.float32)
        p = base[rng.integers(0, len(base), n)]
        x, y = p[:, 0], p[:, 1]
    elif kind == "lattice":
        side = int(np.ceil(np.sqrt(n)))
        i = rng.permutation(side * side)[:n]
        x, y = (i % side) * np.float32(2.0 ** -6), (i // side) * np.float32(2.0 ** -6)
    elif kind == "collinear":
        x = rng.random(n, dtype=np.float32)
        y = np.full(n, 0.25, np.float32)
    elif kind == "boundary":
        x = rng.random(n, dtype=np.float32)
        y = rng.random(n, dtype=np.float32)
        m = rng.random(n) < 0.4
        x[m] = np.where(rng.random(m.sum()) < 0.5, 0.0, CLAMP_HI)
        m = rng.random(n) < 0.4
        y[m] = np.where(rng.random(m.sum()) < 0.5, 0.0, CLAMP_HI)
    elif kind == "tiny_scale":
        # Coordinates near zero: d2 falls into the fp32 denormal range.
        x = (rng.random(n) * 2.0 ** -64).astype(np.float32)
        y = (rng.random(n) * 2.0 ** -64).astype(np.float32)
    else:
        raise ValueError(kind)
    return f32(x), f32(y)


FAMILIES = ["uniform", "clustered", "duplicates", "lattice", "collinear", "boundary",
            "tiny_scale"]


def sq_dist_np(qx, qy, px, py):
    """fp32 d2 with numpy: every float32 ufunc rounds on its own."""
    dx = np.float32(qx) - np.asarray(px, np.float32)
    dy = np.float32(qy) - np.asarray(py, np.float32)
    return dx * dx + dy * dy


def check_rows_vectorized(x, y, issuers, ids, d2, counts, k):
    """The per-row invariants of check_invariants for a block of uniform-k
    rows, vectorized (no mutual-consistency check, which needs every row):
    count = min(k, n-1), padding, ids in range, no self, no duplicates,
    d2 bit-equal to the fp32 d2 recomputed for each id, keys strictly
    ascending."""
    x, y = f32(x), f32(y)
    n = len(x)
    s = np.asarray(issuers, np.int64)
    c = np.asarray(counts)
    assert np.all(c == min(k, n - 1))
    col = np.arange(k)[None, :]
    real = col < c[:, None]
    assert np.all(ids[~real] == -1) and np.all(np.isinf(d2[~real]))
    vi = np.where(real, ids, 0).astype(np.int64)
    assert np.all((vi >= 0) & (vi < n))
    assert not np.any(real & (vi == s[:, None]))
    dx = x[s][:, None] - x[vi]
    dy = y[s][:, None] - y[vi]
    rec = dx * dx + dy * dy
    assert rec.dtype == np.float32
    assert np.array_equal(np.where(real, rec, np.inf).view(np.uint32),
                          np.where(real, d2, np.inf).view(np.uint32))
    keys = (d2.view(np.uint32).astype(np.uint64) << np.uint64(32)) | vi.astype(np.uint64)
    inc = keys[:, 1:] > keys[:, :-1]
    assert np.all(inc | ~real[:, 1:])  # strictly ascending, hence no duplicates


def check_invariants(x, y, issuers, ks, ids, d2, counts, offsets=None, k=None):
    """Properties every exact result satisfies, for all queries:
    count = min(k, n-1); rows strictly ascending by (d2, id); no self, no
    duplicates; each d2 equals the fp32 d2 recomputed for its id; padding is
    id -1 / d2 +inf; and mutual consistency: d2 is bit-symmetric, so if j is
    in i's row with a key below j's k-th key, i is in j's row."""
    x, y = f32(x), f32(y)
    n = len(x)
    nq = len(counts)
    iss = np.arange(n) if issuers is None else np.asarray(issuers)
    rows = []
    for q in range(nq):
        if offsets is None:
            kq = k
            ri, rd = ids[q], d2[q]
        else:
            kq = int(ks[q])
            ri = ids[offsets[q]:offsets[q + 1]]
            rd = d2[offsets[q]:offsets[q + 1]]
        c = int(counts[q])
        assert c == min(kq, n - 1), (q, c, kq, n)
        assert np.all(ri[c:] == -1) and np.all(np.isinf(rd[c:]))
        vi, vd = ri[:c].astype(np.int64), rd[:c]
        s = int(iss[q])
        assert np.all((vi >= 0) & (vi < n))
        assert s not in set(vi.tolist()), (q, s)
        assert len(set(vi.tolist())) == c
        rec = sq_dist_np(x[s], y[s], x[vi], y[vi])
        assert np.array_equal(rec.view(np.uint32), vd.view(np.uint32)), q
        keys = (vd.view(np.uint32).astype(np.uint64) << np.uint64(32)) | vi.astype(np.uint64)
        assert np.all(keys[1:] > keys[:-1]), q
        rows.append((s, kq, c, keys))
    if issuers is None and offsets is None:
        kth = np.array([r[3][-1] if r[2] == r[1] else np.uint64(2 ** 64 - 1) for r in rows],
                       dtype=np.uint64)
        for s, kq, c, keys in rows:
            for key in keys:
                j = int(key & np.uint64(0xFFFFFFFF))
                mirror = (key & ~np.uint64(0xFFFFFFFF)) | np.uint64(s)
                if mirror < kth[j]:
                    assert s in set((rows[j][3] & np.uint64(0xFFFFFFFF)).astype(np.int64).tolist()), (s, j)
