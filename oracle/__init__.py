"""CPU oracle for the per-tick k-NN join -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports, links or calls it, and
it shares no code with the GPU path.

Contents (each function names the passage of arXiv 1412.6170 it follows):

* ``brute_knn_numpy`` -- Definition 1 (Sec. 2.1) written out in numpy for
  tiny inputs: every other object is a candidate, ranked by the fp32 squared
  distance ``fl(fl(dx*dx) + fl(dy*dy))``, ties by ascending object id.
* ``brute_knn``       -- the same definition in plain C (oracle/mknn_oracle.c),
  optionally split across host threads by query.
* ``knn``             -- the sequential PR-quadtree k-NN of Sec. 4 in plain C:
  index creation (Sec. 4.1) then a pruned depth-first leaf visit (Sec. 4.2).
* ``build_index``     -- that index: Morton codes at level 16, objects sorted
  by (code, id), and the non-empty leaves of the PR-quadtree split at ``th``.
* ``brute_knn_points``, ``knn_points`` -- the same two searches for queries
  with a free centre q = (x, y, k) in [0,1)^2 (Definition 1) and an optional
  excluded object id; ``brute_knn_points_numpy`` writes it out in numpy.
* ``morton_codes``, ``sq_dist`` -- the arithmetic the above rely on.

Result convention (all k-NN entry points): rows in query order, each of
``k`` slots ascending by (d2, id), ``count = min(k, n-1)`` valid entries, the
rest padded with id -1 and d2 +inf.  Variable k uses CSR row offsets.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)

ERRORS = {-1: "invalid argument", -2: "coordinate not finite or outside [0,1)",
          -5: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle error %d: %s" % (code, ERRORS.get(code, "?")))
        self.code = code


def lib():
    """Load (building first if needed) the C oracle."""
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "mknn_oracle.c")
        if (not os.path.exists(_SO)) or os.path.getmtime(_SO) < os.path.getmtime(src):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_SO)
        L.oracle_morton.restype = ctypes.c_uint32
        L.oracle_morton.argtypes = [ctypes.c_float, ctypes.c_float]
        L.oracle_sq_dist.restype = ctypes.c_float
        L.oracle_sq_dist.argtypes = [ctypes.c_float] * 4
        L.oracle_validate.argtypes = [_f32p, _f32p, ctypes.c_int64]
        L.oracle_morton_codes.argtypes = [_f32p, _f32p, ctypes.c_int64, _u32p]
        L.oracle_build_index.argtypes = [
            _f32p, _f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
            _u32p, _i32p, _i32p, _u32p, _i64p, _i64p, ctypes.c_int64, _i64p, _i64p]
        knn_args = [_f32p, _f32p, ctypes.c_int64, _i32p, _i32p, ctypes.c_int64,
                    ctypes.c_int32, _i64p]
        L.oracle_brute_knn.argtypes = knn_args + [_i32p, _f32p, _i32p, ctypes.c_int32]
        L.oracle_knn.argtypes = knn_args + [ctypes.c_int32, ctypes.c_int32,
                                            _i32p, _f32p, _i32p, ctypes.c_int32]
        pts_args = [_f32p, _f32p, ctypes.c_int64, _f32p, _f32p, _i32p, _i32p, ctypes.c_int64,
                    ctypes.c_int32, _i64p]
        L.oracle_brute_knn_points.argtypes = pts_args + [_i32p, _f32p, _i32p, ctypes.c_int32]
        L.oracle_knn_points.argtypes = pts_args + [ctypes.c_int32, ctypes.c_int32,
                                                   _i32p, _f32p, _i32p, ctypes.c_int32]
        _lib = L
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def morton_codes(x, y):
    """Level-16 Morton codes, x cell in the even bits (Sec. 4.1)."""
    x, y = _f32(x), _f32(y)
    out = np.empty(len(x), np.uint32)
    _check(lib().oracle_morton_codes(_ptr(x, _f32p), _ptr(y, _f32p), len(x), _ptr(out, _u32p)))
    return out


def sq_dist(qx, qy, px, py):
    """fl(fl(fl(qx-px)^2) + fl(fl(qy-py)^2)) as the oracle rounds it."""
    return np.float32(lib().oracle_sq_dist(float(np.float32(qx)), float(np.float32(qy)),
                                           float(np.float32(px)), float(np.float32(py))))


def validate(x, y):
    x, y = _f32(x), _f32(y)
    _check(lib().oracle_validate(_ptr(x, _f32p), _ptr(y, _f32p), len(x)))


def default_leaf_capacity(k):
    """Paper's rule for th_quad (Sec. 6, study S2): 192 for k < 32, 12k for
    32 <= k <= 128, 2048 above (the stated ranges overlap; this is the
    reading used throughout)."""
    if k < 32:
        return 192
    if k <= 128:
        return 12 * k
    return 2048


def build_index(x, y, th, L=16):
    """Sorted (code, id) order and the non-empty PR-quadtree leaves."""
    x, y = _f32(x), _f32(y)
    n = len(x)
    codes = np.empty(n, np.uint32)
    ids = np.empty(n, np.int32)
    cap = max(16, 4 * n // max(th, 1) + 64)
    while True:
        lev = np.empty(cap, np.int32)
        pre = np.empty(cap, np.uint32)
        beg = np.empty(cap, np.int64)
        end = np.empty(cap, np.int64)
        nl = ctypes.c_int64(0)
        ne = ctypes.c_int64(0)
        rc = lib().oracle_build_index(_ptr(x, _f32p), _ptr(y, _f32p), n, th, L,
                                      _ptr(codes, _u32p), _ptr(ids, _i32p), _ptr(lev, _i32p),
                                      _ptr(pre, _u32p), _ptr(beg, _i64p), _ptr(end, _i64p),
                                      cap, ctypes.byref(nl), ctypes.byref(ne))
        if rc == -1 and nl.value > cap:
            cap = nl.value
            continue
        _check(rc)
        m = nl.value
        return {"codes": codes, "ids": ids, "leaf_level": lev[:m].copy(),
                "leaf_prefix": pre[:m].copy(), "leaf_begin": beg[:m].copy(),
                "leaf_end": end[:m].copy(), "n_empty_leaves": ne.value}


def _prep_queries(n, issuers, ks, k):
    if issuers is None:
        nq = n
        iss = None
    else:
        iss = np.ascontiguousarray(issuers, dtype=np.int32)
        nq = len(iss)
    if ks is None:
        if k is None or k < 1:
            raise ValueError("k must be >= 1")
        kk = None
        offsets = None
        total = nq * int(k)
    else:
        kk = np.ascontiguousarray(ks, dtype=np.int32)
        if len(kk) != nq:
            raise ValueError("ks must have one entry per query")
        offsets = np.zeros(nq + 1, np.int64)
        np.cumsum(kk, out=offsets[1:])
        total = int(offsets[-1])
        k = 0
    return iss, nq, kk, int(k or 0), offsets, total


def _run(fn, x, y, issuers, ks, k, extra, threads):
    x, y = _f32(x), _f32(y)
    n = len(x)
    iss, nq, kk, ku, offsets, total = _prep_queries(n, issuers, ks, k)
    ids = np.empty(max(total, 1), np.int32)
    d2 = np.empty(max(total, 1), np.float32)
    cnt = np.empty(max(nq, 1), np.int32)
    args = [_ptr(x, _f32p), _ptr(y, _f32p), n, _ptr(iss, _i32p), _ptr(kk, _i32p), nq, ku,
            _ptr(offsets, _i64p)] + extra + [_ptr(ids, _i32p), _ptr(d2, _f32p),
                                             _ptr(cnt, _i32p), int(threads)]
    _check(fn(*args))
    ids, d2, cnt = ids[:total], d2[:total], cnt[:nq]
    if ks is None:
        return ids.reshape(nq, ku), d2.reshape(nq, ku), cnt, None
    return ids, d2, cnt, offsets


def brute_knn(x, y, issuers=None, ks=None, k=None, threads=1):
    """Definition 1 by brute force (C).  Returns (ids, d2, counts, offsets);
    dense [nq, k] rows for uniform k, CSR with ``offsets`` for variable k."""
    return _run(lib().oracle_brute_knn, x, y, issuers, ks, k, [], threads)


def knn(x, y, issuers=None, ks=None, k=None, th=None, L=16, threads=1):
    """Sequential PR-quadtree k-NN (Sec. 4); same contract as brute_knn."""
    if th is None:
        kref = int(k) if ks is None else int(np.max(ks)) if len(ks) else 1
        th = default_leaf_capacity(kref)
    return _run(lib().oracle_knn, x, y, issuers, ks, k, [int(th), int(L)], threads)


def brute_knn_numpy(x, y, issuers=None, k=8):
    """Definition 1 in numpy, uniform k, for tiny inputs.  Every numpy float32
    ufunc rounds its own result, so nothing is fused."""
    x, y = _f32(x), _f32(y)
    n = len(x)
    iss = np.arange(n) if issuers is None else np.asarray(issuers)
    nq = len(iss)
    ids_out = np.full((nq, k), -1, np.int32)
    d2_out = np.full((nq, k), np.inf, np.float32)
    cnt = np.zeros(nq, np.int32)
    all_ids = np.arange(n, dtype=np.int64)
    for r, s in enumerate(iss):
        dx = x[s] - x
        dy = y[s] - y
        d2 = dx * dx + dy * dy
        keep = all_ids != s
        cand_d2 = d2[keep]
        cand_id = all_ids[keep]
        order = np.lexsort((cand_id, cand_d2))[:k]
        m = len(order)
        ids_out[r, :m] = cand_id[order]
        d2_out[r, :m] = cand_d2[order]
        cnt[r] = m
    return ids_out, d2_out, cnt


def _run_points(fn, x, y, qx, qy, exclude, ks, k, extra, threads):
    x, y = _f32(x), _f32(y)
    qx, qy = _f32(qx), _f32(qy)
    n, nq = len(x), len(qx)
    if len(qy) != nq:
        raise ValueError("qx and qy differ in length")
    ex = None if exclude is None else np.ascontiguousarray(exclude, dtype=np.int32)
    if ex is not None and len(ex) != nq:
        raise ValueError("exclude must have one entry per query")
    _, _, kk, ku, offsets, total = _prep_queries(nq, np.zeros(nq, np.int32), ks, k)
    ids = np.empty(max(total, 1), np.int32)
    d2 = np.empty(max(total, 1), np.float32)
    cnt = np.empty(max(nq, 1), np.int32)
    args = [_ptr(x, _f32p), _ptr(y, _f32p), n, _ptr(qx, _f32p), _ptr(qy, _f32p), _ptr(ex, _i32p),
            _ptr(kk, _i32p), nq, ku, _ptr(offsets, _i64p)] + extra + [
                _ptr(ids, _i32p), _ptr(d2, _f32p), _ptr(cnt, _i32p), int(threads)]
    _check(fn(*args))
    ids, d2, cnt = ids[:total], d2[:total], cnt[:nq]
    if ks is None:
        return ids.reshape(nq, ku), d2.reshape(nq, ku), cnt, None
    return ids, d2, cnt, offsets


def brute_knn_points(x, y, qx, qy, exclude=None, ks=None, k=None, threads=1):
    """Definition 1 with free centres (qx[i], qy[i]) by brute force (C);
    object exclude[i] (None or -1: none) is left out.  Rows hold
    min(k, candidates) entries; same layout as brute_knn."""
    return _run_points(lib().oracle_brute_knn_points, x, y, qx, qy, exclude, ks, k, [], threads)


def knn_points(x, y, qx, qy, exclude=None, ks=None, k=None, th=None, L=16, threads=1):
    """Sequential PR-quadtree k-NN (Sec. 4) with free centres; same contract
    as brute_knn_points."""
    if th is None:
        kref = int(k) if ks is None else int(np.max(ks)) if len(ks) else 1
        th = default_leaf_capacity(kref)
    return _run_points(lib().oracle_knn_points, x, y, qx, qy, exclude, ks, k,
                       [int(th), int(L)], threads)


def brute_knn_points_numpy(x, y, qx, qy, exclude=None, k=8):
    """Definition 1 with free centres in numpy, uniform k, tiny inputs."""
    x, y = _f32(x), _f32(y)
    qx, qy = _f32(qx), _f32(qy)
    n, nq = len(x), len(qx)
    ids_out = np.full((nq, k), -1, np.int32)
    d2_out = np.full((nq, k), np.inf, np.float32)
    cnt = np.zeros(nq, np.int32)
    all_ids = np.arange(n, dtype=np.int64)
    for r in range(nq):
        dx = qx[r] - x
        dy = qy[r] - y
        d2 = dx * dx + dy * dy
        keep = all_ids != (-1 if exclude is None else int(exclude[r]))
        cand_d2 = d2[keep]
        cand_id = all_ids[keep]
        order = np.lexsort((cand_id, cand_d2))[:k]
        m = len(order)
        ids_out[r, :m] = cand_id[order]
        d2_out[r, :m] = cand_d2[order]
        cnt[r] = m
    return ids_out, d2_out, cnt
