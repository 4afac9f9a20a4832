"""ctypes binding of libmknn.so (the C ABI in include/mknn.h).

Argument marshalling only: every step of the tick runs in the HIP library.
Host arrays are numpy; device arrays are torch tensors on the context's
device (torch only provides device memory and streams).  A missing library
raises immediately -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmknn.so")

MKNN_OK = 0
MKNN_HOST = 0
MKNN_DEVICE = 1
MKNN_FLAG_TIMING = 1
MKNN_FLAG_COUNTERS = 2
MKNN_FLAG_GROUP_K = 4
MKNN_FLAG_SWEEP_WAVE = 8
MKNN_K_LIMIT = 1024
MKNN_SWEEP_AUTO = 0
MKNN_SWEEP_LANE = 1
MKNN_SWEEP_WAVE = 2
MKNN_SWEEP_GROUP = 3
SWEEPS = {"auto": MKNN_SWEEP_AUTO, "lane": MKNN_SWEEP_LANE, "wave": MKNN_SWEEP_WAVE,
          "group": MKNN_SWEEP_GROUP}
STATUS = {0: "MKNN_OK", -1: "MKNN_E_INVAL", -2: "MKNN_E_RANGE", -3: "MKNN_E_STATE",
          -4: "MKNN_E_CAPACITY", -5: "MKNN_E_NOMEM", -6: "MKNN_E_DEVICE"}


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("leaf_capacity", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("n_max", ctypes.c_int64), ("q_max", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("k_hint", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("tick", ctypes.c_int64), ("n", ctypes.c_int64), ("nq", ctypes.c_int64),
                ("leaves", ctypes.c_int64), ("nodes", ctypes.c_int64),
                ("leaf_capacity", ctypes.c_int32), ("deepest_level", ctypes.c_int32),
                ("ms_build", ctypes.c_float), ("ms_query", ctypes.c_float),
                ("ms_query_main", ctypes.c_float), ("timed_ticks", ctypes.c_int32),
                ("ms_build_mean", ctypes.c_float), ("ms_query_mean", ctypes.c_float),
                ("ms_query_main_mean", ctypes.c_float), ("reserved", ctypes.c_float * 4),
                ("wave_candidate_steps", ctypes.c_int64), ("wave_merges", ctypes.c_int64),
                ("wave_node_visits", ctypes.c_int64), ("wave_leaf_sweeps", ctypes.c_int64),
                ("wavefronts", ctypes.c_int64), ("refits", ctypes.c_int64),
                ("drift", ctypes.c_float), ("reserved2", ctypes.c_float)]


class Schedule(ctypes.Structure):
    _fields_ = [("leaf_capacity", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("sweep", ctypes.c_int32), ("group_k", ctypes.c_int32),
                ("tile_queries", ctypes.c_int32)]


class MknnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def lib():
    """Load libmknn.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmknn.so is not built (run `python -m paper_1412_6170_amd.build`"
                              " or __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "mknn_create": ([ctypes.POINTER(Config), ctypes.POINTER(_vp)], _i32),
            "mknn_destroy": ([_vp], _i32),
            "mknn_load_positions": ([_vp, _vp, _vp, _i64, _i32], _i32),
            "mknn_advance_tick": ([_vp], _i32),
            "mknn_refit_tick": ([_vp], _i32),
            "mknn_query": ([_vp, _vp, _vp, _i64, _i32, _i32], _i32),
            "mknn_query_points": ([_vp, _vp, _vp, _vp, _vp, _i64, _i32, _i32], _i32),
            "mknn_fetch": ([_vp, _vp, _vp, _vp, _vp, _i32], _i32),
            "mknn_result_size": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)], _i32),
            "mknn_result_device": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                    ctypes.POINTER(_vp), ctypes.POINTER(_vp)], _i32),
            "mknn_index_fetch": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64,
                                  ctypes.POINTER(_i64)], _i32),
            "mknn_sync": ([_vp], _i32),
            "mknn_reset_timing": ([_vp], _i32),
            "mknn_query_time": ([_vp, _i32, _i32, ctypes.POINTER(ctypes.c_float)], _i32),
            "mknn_set_leaf_capacity": ([_vp, _i32], _i32),
            "mknn_get_stats": ([_vp, ctypes.POINTER(Stats)], _i32),
            "mknn_last_error": ([_vp], ctypes.c_char_p),
            "mknn_status_str": ([_i32], ctypes.c_char_p),
            "mknn_default_leaf_capacity": ([_i32], _i32),
            "mknn_footprint": ([ctypes.POINTER(Config), ctypes.POINTER(_i64)], _i32),
            "mknn_get_schedule": ([_vp, ctypes.POINTER(Schedule)], _i32),
            "mknn_set_epochs": ([_vp, ctypes.c_uint32, ctypes.c_uint32], _i32),
            "mknn_set_schedule": ([_vp, ctypes.POINTER(Schedule)], _i32),
            "mknn_knn_noalloc": ([_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp], _i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


_hiplib = None


def _hip():
    """The HIP runtime: plain device-to-host copies of result rows, and the
    event that orders a context's stream after its inputs' producer."""
    global _hiplib
    if _hiplib is None:
        h = ctypes.CDLL("libamdhip64.so")
        for name, args in (("hipMemcpy", [_vp, _vp, ctypes.c_size_t, ctypes.c_int]),
                           ("hipEventCreateWithFlags", [ctypes.POINTER(_vp), ctypes.c_uint]),
                           ("hipEventRecord", [_vp, _vp]),
                           ("hipStreamWaitEvent", [_vp, _vp, ctypes.c_uint]),
                           ("hipEventDestroy", [_vp])):
            f = getattr(h, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _hiplib = h
    return _hiplib


# hipEventDisableTiming | hipEventDisableSystemFence: an ordering-only event
# between two streams of one device needs no system-scope release.
_ORDER_EVENT_FLAGS = 0x2 | 0x20000000


NOALLOC_MAX_N = 65536


def knn_noalloc(x, y, k, ids, d2, counts, status=None, leaf_capacity=0, stream=None):
    """mknn_knn_noalloc: one tick (index build, every object querying with
    uniform k) that allocates nothing, writing into the caller's device
    buffers.  x, y: float32 cuda tensors of n coordinates; ids (int32),
    d2 (float32): n * k entries; counts (int32): n entries; status: one
    int32 entry or None.  Runs on `stream` (a torch stream or a raw handle;
    None: torch's current stream).  Raises MknnError on a host-checked
    error; device-detected errors land in status."""
    import torch
    n = int(x.numel())
    for t, dt, cnt in ((x, torch.float32, n), (y, torch.float32, n), (ids, torch.int32, n * k),
                       (d2, torch.float32, n * k), (counts, torch.int32, n)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous() or t.numel() < cnt:
            raise MknnError(-1, "knn_noalloc: bad buffer")
    if status is not None and (not status.is_cuda or status.dtype != torch.int32):
        raise MknnError(-1, "knn_noalloc: bad status buffer")
    if stream is None:
        handle = torch.cuda.current_stream(x.device).cuda_stream
    elif isinstance(stream, torch.cuda.Stream):
        handle = stream.cuda_stream
    else:
        handle = int(stream)
    with torch.cuda.device(x.device):
        rc = lib().mknn_knn_noalloc(_vp(x.data_ptr()), _vp(y.data_ptr()), n, int(k),
                                    int(leaf_capacity), _vp(ids.data_ptr()),
                                    _vp(d2.data_ptr()), _vp(counts.data_ptr()),
                                    _vp(status.data_ptr()) if status is not None else None,
                                    _vp(handle) if handle else None)
    if rc != 0:
        raise MknnError(rc, "mknn_knn_noalloc failed")


def default_leaf_capacity(k):
    return int(lib().mknn_default_leaf_capacity(int(k)))


def make_config(n_max, q_max=None, k_max=32, leaf_capacity=0, max_level=0, k_hint=0, device=0,
                stream=None, timing=False, counters=False, group_k=False, sweep_wave=False):
    cfg = Config()
    cfg.device = device
    cfg.leaf_capacity = int(leaf_capacity)
    cfg.max_level = int(max_level)
    cfg.k_max = int(k_max)
    cfg.n_max = int(n_max)
    cfg.q_max = int(q_max if q_max is not None else n_max)
    cfg.stream = stream
    cfg.k_hint = int(k_hint)
    cfg.flags = ((MKNN_FLAG_TIMING if timing else 0) | (MKNN_FLAG_COUNTERS if counters else 0)
                 | (MKNN_FLAG_GROUP_K if group_k else 0)
                 | (MKNN_FLAG_SWEEP_WAVE if sweep_wave else 0))
    return cfg


def footprint(**kw):
    """Device bytes a context with these settings allocates (no device use)."""
    b = _i64()
    rc = lib().mknn_footprint(ctypes.byref(make_config(**kw)), ctypes.byref(b))
    if rc != 0:
        raise MknnError(rc, "mknn_footprint failed")
    return b.value


def _is_tensor(a):
    return type(a).__module__.startswith("torch")


def _host_ptr(a, dtype):
    return a.ctypes.data_as(_vp) if a is not None else None


class Context:
    """One mknn context: device memory for n_max objects and q_max queries
    of up to k_max neighbours each.

    Work runs on the context's stream: `stream` (a torch stream or a raw
    stream handle), else (None or the null stream) a torch stream of its
    own.  Device inputs may still be being produced on the caller's current
    torch stream: each call that takes them first makes the context's
    stream wait for the work enqueued there so far, and marks them used on
    the context's stream, so that torch's caching allocator does not hand
    their memory out again before the context's stream has passed the
    call."""

    def __init__(self, n_max, q_max=None, k_max=32, leaf_capacity=0, max_level=0, k_hint=0,
                 device=0, stream=None, timing=False, counters=False, group_k=False,
                 sweep_wave=False):
        self._h = None
        self._order_ev = None
        import torch
        if isinstance(stream, torch.cuda.Stream):
            ts = stream
        elif stream:
            ptr = int(stream)
            known = (torch.cuda.current_stream(device), torch.cuda.default_stream(device))
            ts = next((t for t in known if t.cuda_stream == ptr), None)
            if ts is None:
                ts = torch.cuda.ExternalStream(ptr, device=device)
        else:
            ts = None
        if ts is None or not ts.cuda_stream:
            # A null handle would ask the library for a stream of its own;
            # take a torch stream instead, so that it has a torch object.
            ts = torch.cuda.Stream(device=device)   # default priority
        self._tstream = ts
        cfg = make_config(n_max, q_max, k_max, leaf_capacity, max_level, k_hint, device,
                          ts.cuda_stream, timing, counters, group_k, sweep_wave)
        self.cfg = cfg
        h = _vp()
        rc = lib().mknn_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != 0:
            raise MknnError(rc, "mknn_create failed")
        self._h = h
        ev = _vp()
        rc = _hip().hipEventCreateWithFlags(ctypes.byref(ev), _ORDER_EVENT_FLAGS)
        if rc != 0:
            self.close()
            raise MknnError(-6, "hipEventCreateWithFlags failed (%d)" % rc)
        self._order_ev = ev
        self._keep = []

    @property
    def stream(self):
        """The torch stream the context's work runs on."""
        return self._tstream

    def _device_inputs(self, *arrays):
        """Order the context's stream after the caller's current stream and
        mark device inputs as used on the context's stream (see the class
        docstring).  Host arrays need neither: they are read during the
        call."""
        dev = [a for a in arrays if a is not None and _is_tensor(a) and a.is_cuda]
        if not dev:
            return
        import torch
        for a in dev:
            if a.device.index != self.cfg.device:
                raise ValueError("device arrays must be on the context's device (%d)"
                                 % self.cfg.device)
        cur = torch.cuda.current_stream(self.cfg.device)
        # Nothing to wait for when the caller's stream is the context's, or
        # has already finished everything enqueued on it (a capturing
        # stream cannot be asked, so it always gets the event).
        if cur.cuda_stream != self._tstream.cuda_stream and (
                torch.cuda.is_current_stream_capturing() or not cur.query()):
            hip = _hip()
            rc = hip.hipEventRecord(self._order_ev, ctypes.c_void_p(cur.cuda_stream))
            if rc == 0:
                rc = hip.hipStreamWaitEvent(ctypes.c_void_p(self._tstream.cuda_stream),
                                            self._order_ev, 0)
            if rc != 0:
                raise MknnError(-6, "ordering the context's stream after the current "
                                    "stream failed (%d)" % rc)
        for a in dev:
            a.record_stream(self._tstream)

    # -- plumbing ------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise MknnError(rc, lib().mknn_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().mknn_destroy(self._h)
            self._h = None
        if getattr(self, "_order_ev", None):
            _hip().hipEventDestroy(self._order_ev)
            self._order_ev = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _arg(a, dtype):
        """(pointer, where, keepalive) for a host numpy array or a device
        torch tensor."""
        if a is None:
            return None, None, None
        if _is_tensor(a):
            if not a.is_cuda:
                a = a.numpy()
            else:
                import torch
                tdt = {np.float32: torch.float32, np.int32: torch.int32}[dtype]
                if a.dtype != tdt or not a.is_contiguous():
                    raise TypeError("device arrays must be contiguous %s" % tdt)
                return ctypes.c_void_p(a.data_ptr()), MKNN_DEVICE, a
        a = np.ascontiguousarray(a, dtype=dtype)
        return a.ctypes.data_as(_vp), MKNN_HOST, a

    # -- the four verbs ------------------------------------------------------
    def load_positions(self, x, y):
        self._device_inputs(x, y)
        px, wx, kx = self._arg(x, np.float32)
        py, wy, ky = self._arg(y, np.float32)
        if wx != wy:
            raise TypeError("x and y must both be host or both be device arrays")
        n = len(kx)
        if len(ky) != n:
            raise ValueError("x and y differ in length")
        self._check(lib().mknn_load_positions(self._h, px, py, n, wx))
        self._keep = [kx, ky]
        self._n = n

    def advance_tick(self):
        self._check(lib().mknn_advance_tick(self._h))

    def refit_tick(self):
        """Reuse the last full build's index with the current positions
        (exact; leaf boxes are recomputed from the objects, inner node
        boxes grow by the objects' drift since that build)."""
        self._check(lib().mknn_refit_tick(self._h))

    def query(self, k=None, issuers=None, ks=None, nq=None):
        self._device_inputs(issuers, ks)
        pi, wi, ki = self._arg(issuers, np.int32)
        pk, wk, kk = self._arg(ks, np.int32)
        where = wi if wi is not None else (wk if wk is not None else MKNN_HOST)
        if wi is not None and wk is not None and wi != wk:
            raise TypeError("issuers and ks must live in the same place")
        if nq is None:
            if ki is not None:
                nq = len(ki)
            elif kk is not None:
                nq = len(kk)
            else:
                nq = self._n
        self._check(lib().mknn_query(self._h, pi, pk, int(nq), int(k or 0), where))
        self._qkeep = [ki, kk]
        self._last_k = None if ks is not None else int(k)
        self._queried = True

    def query_points(self, qx, qy, exclude=None, k=None, ks=None):
        """Queries with free centres (qx[i], qy[i]) in [0,1)^2; object
        exclude[i] (None or -1: none) is left out.  Arrays are numpy (host)
        or torch CUDA tensors (device), all in the same place."""
        self._device_inputs(qx, qy, exclude, ks)
        px, wx, kx = self._arg(qx, np.float32)
        py, wy, ky = self._arg(qy, np.float32)
        pe, we, ke = self._arg(exclude, np.int32)
        pk, wk, kk = self._arg(ks, np.int32)
        places = {w for w in (wx, wy, we, wk) if w is not None}
        if len(places) > 1:
            raise TypeError("query arrays must all live in the same place")
        where = places.pop() if places else MKNN_HOST
        nq = len(kx)
        if len(ky) != nq or (ke is not None and len(ke) != nq) or (kk is not None and len(kk) != nq):
            raise ValueError("query arrays differ in length")
        self._check(lib().mknn_query_points(self._h, px, py, pe, pk, int(nq), int(k or 0), where))
        self._qkeep = [kx, ky, ke, kk]
        self._last_k = None if ks is not None else int(k)
        self._queried = True

    def result_size(self):
        nq, ne = _i64(), _i64()
        self._check(lib().mknn_result_size(self._h, ctypes.byref(nq), ctypes.byref(ne)))
        return nq.value, ne.value

    def fetch(self):
        """Host copies: (ids, d2, counts, offsets).  Uniform k gives [nq, k]
        arrays and offsets None; variable k gives flat arrays and offsets."""
        nq, ne = self.result_size()
        ids = np.empty(max(ne, 1), np.int32)
        d2 = np.empty(max(ne, 1), np.float32)
        cnt = np.empty(max(nq, 1), np.int32)
        off = np.empty(nq + 1, np.int64)
        self._check(lib().mknn_fetch(self._h, ids.ctypes.data_as(_vp), d2.ctypes.data_as(_vp),
                                     cnt.ctypes.data_as(_vp), off.ctypes.data_as(_vp),
                                     MKNN_HOST))
        ids, d2, cnt = ids[:ne], d2[:ne], cnt[:nq]
        if self._last_k is not None:
            k = self._last_k
            return ids.reshape(nq, k), d2.reshape(nq, k), cnt, None
        return ids, d2, cnt, off

    def fetch_rows(self, rows, k):
        """Host copies of selected rows of a uniform-k result (ids, d2,
        counts), copied row by row from the device."""
        hip = _hip()
        ids_p, d2_p, cnt_p, _ = self.result_device_ptrs()
        self.sync()
        rows = np.asarray(rows, np.int64)
        ids = np.empty((len(rows), k), np.int32)
        d2 = np.empty((len(rows), k), np.float32)
        cnt = np.empty(len(rows), np.int32)
        for i, r in enumerate(rows):
            for dst, src, size, off in ((ids[i], ids_p, 4 * k, 4 * k * int(r)),
                                        (d2[i], d2_p, 4 * k, 4 * k * int(r)),
                                        (cnt[i:i + 1], cnt_p, 4, 4 * int(r))):
                rc = hip.hipMemcpy(dst.ctypes.data_as(_vp), ctypes.c_void_p(src + off),
                                   ctypes.c_size_t(size), 2)  # device to host
                if rc != 0:
                    raise MknnError(-6, "hipMemcpy failed (%d)" % rc)
        return ids, d2, cnt

    def result_device_ptrs(self):
        """Device addresses of the result rows (ids, d2, counts, offsets or
        None).  The rows are complete once the context's stream has passed
        the query: work on another stream that reads them waits for it
        first, e.g. torch.cuda.current_stream().wait_stream(ctx.stream)."""
        ids, d2, cnt, off = _vp(), _vp(), _vp(), _vp()
        self._check(lib().mknn_result_device(self._h, ctypes.byref(ids), ctypes.byref(d2),
                                             ctypes.byref(cnt), ctypes.byref(off)))
        return ids.value, d2.value, cnt.value, off.value

    def sync(self):
        self._check(lib().mknn_sync(self._h))

    def reset_timing(self):
        self._check(lib().mknn_reset_timing(self._h))

    def query_time(self, back=0, wait=False):
        """Device ms of an earlier query (back = 0: the last one enqueued).
        With wait, blocks until that query (only) has finished; without,
        returns None if it has not."""
        ms = ctypes.c_float()
        rc = lib().mknn_query_time(self._h, int(back), 1 if wait else 0, ctypes.byref(ms))
        if rc == -3:  # MKNN_E_STATE: still running
            return None
        self._check(rc)
        return ms.value

    def set_epochs(self, build_epoch, query_epoch):
        """Testing hook: the next index step and query take the tags one
        past these (tags wrap from 2^24 - 1 to 1)."""
        self._check(lib().mknn_set_epochs(self._h, int(build_epoch), int(query_epoch)))

    def set_leaf_capacity(self, th):
        self._check(lib().mknn_set_leaf_capacity(self._h, int(th)))

    def schedule(self):
        """The tuning settings in force: leaf_capacity, max_level, sweep
        ("auto", "lane", "wave" or "group"), group_k and tile_queries (lane
        flavour queries per wavefront, 0 = automatic)."""
        sc = Schedule()
        self._check(lib().mknn_get_schedule(self._h, ctypes.byref(sc)))
        names = {v: k for k, v in SWEEPS.items()}
        return {"leaf_capacity": sc.leaf_capacity, "max_level": sc.max_level,
                "sweep": names[sc.sweep], "group_k": bool(sc.group_k),
                "tile_queries": sc.tile_queries}

    def set_schedule(self, leaf_capacity=None, max_level=None, sweep=None, group_k=None,
                     tile_queries=None):
        """Change tuning settings (None: keep); results never depend on
        them."""
        cur = self.schedule()
        sc = Schedule()
        sc.leaf_capacity = int(cur["leaf_capacity"] if leaf_capacity is None else leaf_capacity)
        sc.max_level = int(cur["max_level"] if max_level is None else max_level)
        sc.sweep = SWEEPS[cur["sweep"] if sweep is None else sweep]
        sc.group_k = int(cur["group_k"] if group_k is None else bool(group_k))
        sc.tile_queries = int(cur["tile_queries"] if tile_queries is None else tile_queries)
        self._check(lib().mknn_set_schedule(self._h, ctypes.byref(sc)))

    def stats_ready(self):
        """True once the context has run a query (stats then describe it)."""
        return getattr(self, "_queried", False)

    def stats(self):
        s = Stats()
        self._check(lib().mknn_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_ if f != "reserved"}

    def index(self):
        """The current index as host arrays (same keys as the oracle's
        build_index, without n_empty_leaves)."""
        st = self.stats()
        n = st["n"]
        cap = max(int(st["leaves"]), 1)
        codes = np.empty(max(n, 1), np.uint32)
        ids = np.empty(max(n, 1), np.int32)
        lev = np.empty(cap, np.int32)
        pre = np.empty(cap, np.uint32)
        beg = np.empty(cap, np.int64)
        end = np.empty(cap, np.int64)
        nl = _i64()
        self._check(lib().mknn_index_fetch(
            self._h, codes.ctypes.data_as(_vp), ids.ctypes.data_as(_vp),
            lev.ctypes.data_as(_vp), pre.ctypes.data_as(_vp), beg.ctypes.data_as(_vp),
            end.ctypes.data_as(_vp), cap, ctypes.byref(nl)))
        m = nl.value
        return {"codes": codes[:n], "ids": ids[:n], "leaf_level": lev[:m], "leaf_prefix": pre[:m],
                "leaf_begin": beg[:m], "leaf_end": end[:m], "nodes": st["nodes"]}


class ReusePolicy:
    """When to rebuild the index (Sec. 4.1: rebuild only when the work of the
    last tick exceeds that of recent ticks by some factor).  The query of a
    tick with a full build is the reference; later ticks refit the index
    while queries stay within ``factor`` times that reference (and at most
    ``max_refits`` ticks in a row), otherwise they rebuild.  The decision
    reads the time of the query two ticks back, waiting for that query only:
    the host stays at most two ticks ahead while the last tick keeps the GPU
    busy (waiting for the last query instead would leave the GPU idle while
    the next tick is enqueued).  Queries older than the last full build are
    ignored.  A tick whose object count differs from the last full build's
    rebuilds (a refit keeps that build's objects).  The caller enqueues one
    query per tick after tick(); the context needs timing=True."""

    def __init__(self, factor=1.15, max_refits=None):
        self.factor = float(factor)
        self.max_refits = max_refits
        self.reference = None
        self.rebuilds = 0
        self.refits = 0
        self._ticks = 0         # ticks enqueued
        self._last_build = -1   # tick of the last full build
        self._streak = 0        # refit ticks in a row
        self._last = None       # latest query time seen since that build
        self._n_built = None    # object count of the last full build

    def tick(self, ctx, x, y):
        """Load the tick's positions and enqueue its index step."""
        q = self._ticks - 2     # the query read below: two ticks back
        if q >= 0 and q >= self._last_build:
            t = ctx.query_time(back=1, wait=True)
            if t is not None:
                if q == self._last_build:
                    self.reference = t
                else:
                    self._last = t
        n = len(x)
        refit = (self._ticks > 0 and n == self._n_built
                 and (self.reference is None or self._last is None
                      or self._last <= self.factor * self.reference)
                 and (self.max_refits is None or self._streak < self.max_refits))
        ctx.load_positions(x, y)
        if refit:
            ctx.refit_tick()
            self.refits += 1
            self._streak += 1
        else:
            ctx.advance_tick()
            self.rebuilds += 1
            self._streak = 0
            self._last_build = self._ticks
            self._last = None
            self._n_built = n
        self._ticks += 1
        return "refit" if refit else "build"


def autotune_leaf_capacity(ctx, run_tick, candidates, repeats=3):
    """Pick the leaf capacity with the shortest device time per tick.

    ctx must have been created with timing enabled and with a leaf capacity
    no larger than min(candidates) (the node tables are sized for it).
    run_tick(i) enqueues tick i (load, advance, query) on the context.  Each
    candidate runs `repeats` ticks after one untimed tick; the mean of the
    library's build + query device times decides.  Results never depend on
    the leaf capacity, only the time does.  Returns (best, {th: ms})."""
    times = {}
    i = 0
    for th in candidates:
        ctx.set_leaf_capacity(th)
        run_tick(i)
        i += 1
        ctx.sync()
        ctx.reset_timing()
        for _ in range(repeats):
            run_tick(i)
            i += 1
        ctx.sync()
        st = ctx.stats()
        times[th] = st["ms_build_mean"] + st["ms_query_mean"]
    best = min(times, key=times.get)
    ctx.set_leaf_capacity(best)
    ctx.sync()
    ctx.reset_timing()
    return best, times


def autotune_schedule(ctx, run_tick, leaf_capacities, max_levels=(), sweeps=(), group_k=(),
                      repeats=3, rounds=2, finalists=1, final_repeats=8):
    """Pick the schedule with the shortest device time per tick, one
    dimension at a time (coordinate descent over leaf capacity, maximum
    level, sweep flavour and k grouping, `rounds` passes; an empty list
    leaves that dimension as it is).  With finalists > 1, the fastest
    `finalists` settings seen are timed again, in two interleaved passes of
    `final_repeats` ticks each, and the lowest mean of those decides:
    settings a few percent apart are otherwise told apart by the noise of
    a few ticks.  Their entries in the returned times are those means.

    ctx must have been created with timing enabled and with node tables
    that fit every candidate (the smallest leaf capacity and the largest
    maximum level).  run_tick(i) enqueues tick i (load, advance, query) on
    the context.  A setting runs one untimed tick, then `repeats` timed
    ticks; the mean of the library's build + query device times decides.
    Results never depend on the schedule, only the time does.  Returns
    (best schedule dict, {str(setting): ms})."""
    times = {}
    i = [0]

    def timed(kw, reps):
        ctx.set_schedule(**kw)
        run_tick(i[0])
        i[0] += 1
        ctx.sync()
        ctx.reset_timing()
        for _ in range(reps):
            run_tick(i[0])
            i[0] += 1
        ctx.sync()
        st = ctx.stats()
        return st["ms_build_mean"] + st["ms_query_mean"]

    def measure(**kw):
        key = tuple(sorted(kw.items()))
        if key not in times:
            times[key] = timed(kw, repeats)
        return times[key]

    best = ctx.schedule()
    dims = [("leaf_capacity", list(leaf_capacities)), ("max_level", list(max_levels)),
            ("sweep", list(sweeps)), ("group_k", [bool(g) for g in group_k])]
    for _ in range(rounds):
        for name, values in dims:
            if not values:
                continue
            trial = {}
            for v in values:
                cand = dict(best, **{name: v})
                trial[v] = measure(**cand)
            best = dict(best, **{name: min(trial, key=trial.get)})
    if finalists > 1 and len(times) > 1:
        top = sorted(times, key=times.get)[:finalists]
        acc = {key: [] for key in top}
        for _ in range(2):
            for key in top:
                acc[key].append(timed(dict(key), final_repeats))
        for key in top:
            times[key] = sum(acc[key]) / len(acc[key])
        best = dict(min(top, key=times.get))
    ctx.set_schedule(**best)
    ctx.sync()
    ctx.reset_timing()
    return best, {", ".join("%s=%s" % kv for kv in k): v for k, v in times.items()}


def knn_tick(x, y, k=None, issuers=None, ks=None, leaf_capacity=0, max_level=0, k_max=None,
             sweep_wave=False):
    """One tick through a fresh context: load, advance, query, fetch."""
    n = len(x)
    nq = n if issuers is None else len(issuers)
    if k_max is None:
        k_max = int(k) if ks is None else int(np.max(ks)) if len(ks) else 1
    with Context(max(n, 1), max(nq, 1), k_max, leaf_capacity=leaf_capacity,
                 max_level=max_level, sweep_wave=sweep_wave) as c:
        c.load_positions(x, y)
        c.advance_tick()
        c.query(k=k, issuers=issuers, ks=ks, nq=nq)
        return c.fetch()
