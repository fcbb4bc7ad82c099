"""Python binding of libddhf (include/ddhf.h), by ctypes.

Argument marshalling only: every step of the sketch update and the restore
runs in the HIP library. The functions keep the C names; ``Sketch`` wraps a
handle for torch callers (pairs as a CUDA tensor, work on torch's current
stream). There is no fallback: if libddhf.so is not built, loading fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddhf.so")

SKETCH_OK = 0
SKETCH_E_INVAL = -1
SKETCH_E_NOMEM = -2
SKETCH_E_HIP = -3
SKETCH_E_CAPACITY = -4
SKETCH_E_SATURATED = -5

DEFAULT_SEED = 0x1803114490000001

EXPORTS = ("sketch_params_default", "sketch_params_check", "sketch_bytes",
           "sketch_create", "sketch_destroy", "sketch_update",
           "sketch_restore", "sketch_restore_noalloc",
           "sketch_reset", "sketch_download", "sketch_upload",
           "sketch_candidates", "sketch_last_error", "sketch_set_option",
           "sketch_update_batch", "sketch_restore_batch", "sketch_restore_batch_begin",
           "sketch_restore_batch_end", "sketch_merge",
           "sketch_plan_create", "sketch_plan_run", "sketch_plan_results",
           "sketch_plan_launches", "sketch_plan_destroy", "sketch_timings")

SKETCH_PLAN_RESET = 1
SKETCH_PLAN_RESTORE = 2

SKETCH_OPT_UPDATE_PATH = 1
SKETCH_OPT_BINNED_MIN_PAIRS = 2
SKETCH_OPT_UPDATE_GRID = 3
SKETCH_OPT_UPDATE_CHECK = 4
SKETCH_OPT_BINNED_ROUND = 5
SKETCH_OPT_SCATTER_PPT = 6
SKETCH_OPT_BINNED_BLOCKS = 7
SKETCH_OPT_TRIM_POOLS = 8
SKETCH_OPT_APPLY_BLOCKS = 9
SKETCH_OPT_TIMING = 10
SKETCH_OPT_CANDIDATES = 11
SKETCH_OPT_BINNED_SAMPLE = 12
SKETCH_OPT_BINNED_REGIONS = 13
SKETCH_OPT_JOIN_BLOCKS = 14

c_u32, c_u64, c_i32, c_sz, c_dbl, c_vp = (ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_int32, ctypes.c_size_t,
                                          ctypes.c_double, ctypes.c_void_p)


class sketch_params_t(ctypes.Structure):
    _fields_ = [("g", c_u32), ("k", c_u32), ("r", c_u32), ("alpha", c_u32),
                ("seed", c_u64), ("device", c_i32)]


class sketch_sp_t(ctypes.Structure):
    _fields_ = [("ip", c_u32), ("sz", c_u32), ("est", c_dbl)]


class sketch_info_t(ctypes.Structure):
    _fields_ = [("zr", c_u64 * 8), ("he_count", c_u32 * 8),
                ("n_partials", c_u64 * 8), ("n_candidates", c_u64),
                ("n_reported", c_u64), ("psi", c_dbl), ("d", c_dbl),
                ("zmin", c_dbl), ("trep", c_dbl), ("zhot", c_u32),
                ("szmax", c_u32)]


class sketch_timings_t(ctypes.Structure):
    _fields_ = [("hot_scan_ms", ctypes.c_float), ("rows_ms", ctypes.c_float),
                ("join_ms", ctypes.c_float), ("estimate_ms", ctypes.c_float),
                ("sort_publish_ms", ctypes.c_float), ("hot_scan_bytes", c_u64),
                ("join_probes", c_u64), ("join_outputs", c_u64), ("estimate_bytes", c_u64),
                ("search", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("lattice_points", c_u64)]


class sketch_update_job_t(ctypes.Structure):
    _fields_ = [("sketch", c_vp), ("d_pairs", c_vp), ("n_pairs", c_sz)]


class sketch_plan_job_t(ctypes.Structure):
    _fields_ = [("sketch", c_vp), ("d_pairs", c_vp), ("n_pairs", c_sz), ("theta", c_dbl)]


class sketch_restore_job_t(ctypes.Structure):
    _fields_ = [("sketch", c_vp), ("theta", c_dbl), ("out", c_vp), ("cap", c_sz),
                ("info", c_vp), ("n_out", c_sz), ("status", ctypes.c_int)]


SP_DTYPE = np.dtype([("ip", "<u4"), ("sz", "<u4"), ("est", "<f8")])
assert SP_DTYPE.itemsize == ctypes.sizeof(sketch_sp_t) == 16


class SketchError(RuntimeError):
    def __init__(self, code: int, msg: str, n_needed: int | None = None):
        super().__init__(f"libddhf status {code}: {msg}")
        self.code = code
        self.n_needed = n_needed


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library. Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        sig = {
            "sketch_params_default": (None, [P(sketch_params_t)]),
            "sketch_params_check": (c_i32, [P(sketch_params_t)]),
            "sketch_bytes": (c_sz, [P(sketch_params_t)]),
            "sketch_create": (c_i32, [P(sketch_params_t), P(c_vp)]),
            "sketch_destroy": (None, [c_vp]),
            "sketch_update": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
            "sketch_restore": (c_i32, [c_vp, c_dbl, c_vp, c_sz, P(c_sz),
                                       P(sketch_info_t), c_vp]),
            "sketch_restore_noalloc": (c_i32, [c_vp, c_dbl, c_vp, c_sz, P(c_sz),
                                               P(sketch_info_t), c_vp]),
            "sketch_reset": (c_i32, [c_vp, c_vp]),
            "sketch_download": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
            "sketch_upload": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
            "sketch_candidates": (c_i32, [c_vp, c_dbl, c_vp, c_sz, P(c_sz), c_vp]),
            "sketch_last_error": (ctypes.c_char_p, []),
            "sketch_set_option": (c_i32, [c_vp, c_i32, ctypes.c_int64]),
            "sketch_update_batch": (c_i32, [c_vp, c_sz, c_vp]),
            "sketch_restore_batch": (c_i32, [c_vp, c_sz, c_vp]),
            "sketch_restore_batch_begin": (c_i32, [c_vp, c_sz, c_vp]),
            "sketch_restore_batch_end": (c_i32, [c_vp, c_sz, c_vp]),
            "sketch_merge": (c_i32, [c_vp, c_vp, c_vp]),
            "sketch_plan_create": (c_i32, [c_vp, c_sz, c_i32, P(c_vp)]),
            "sketch_plan_run": (c_i32, [c_vp, c_vp]),
            "sketch_plan_results": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
            "sketch_plan_launches": (c_sz, [c_vp]),
            "sketch_plan_destroy": (None, [c_vp]),
            "sketch_timings": (c_i32, [c_vp, P(sketch_timings_t)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().sketch_last_error().decode()


def _check(rc: int, n_needed=None) -> None:
    if rc != SKETCH_OK:
        raise SketchError(rc, last_error(), n_needed)


# --------------------------------------------------- C names, thin wrappers

def sketch_set_option(h: int, option: int, value: int) -> None:
    _check(lib().sketch_set_option(h, option, int(value)))


def sketch_params_default() -> sketch_params_t:
    p = sketch_params_t()
    lib().sketch_params_default(ctypes.byref(p))
    return p


def sketch_params_check(p: sketch_params_t) -> int:
    return lib().sketch_params_check(ctypes.byref(p))


def sketch_bytes(p: sketch_params_t) -> int:
    return lib().sketch_bytes(ctypes.byref(p))


def sketch_create(p: sketch_params_t) -> int:
    h = c_vp()
    _check(lib().sketch_create(ctypes.byref(p), ctypes.byref(h)))
    return h.value


def sketch_destroy(h: int) -> None:
    lib().sketch_destroy(h)


def sketch_update(h: int, d_pairs: int, n_pairs: int, stream: int = 0) -> None:
    _check(lib().sketch_update(h, d_pairs, n_pairs, stream))


def sketch_update_batch(jobs, stream: int = 0) -> None:
    """jobs: sequence of (handle, d_pairs, n_pairs)."""
    arr = (sketch_update_job_t * max(1, len(jobs)))()
    for i, (h, ptr, n) in enumerate(jobs):
        arr[i] = sketch_update_job_t(h, ptr, n)
    _check(lib().sketch_update_batch(ctypes.cast(arr, c_vp), len(jobs), stream))


def sketch_reset(h: int, stream: int = 0) -> None:
    _check(lib().sketch_reset(h, stream))


def _host_buf(cap: int, buf=None) -> np.ndarray:
    """A record buffer of at least cap entries: buf when it is large
    enough (a buffer kept across calls avoids a fresh allocation's page
    faults on every restore), else a new one."""
    if buf is not None and len(buf) >= max(cap, 1):
        return buf
    return np.empty(max(cap, 1), dtype=SP_DTYPE)


def _records(buf: np.ndarray, n: int) -> np.ndarray:
    """A copy of the first n records of buf, copied as bytes (numpy copies
    a structured array field by field, several times slower)."""
    out = np.empty(n, dtype=SP_DTYPE)
    if n:
        out.view(np.uint8)[:] = buf[:n].view(np.uint8)
    return out


def sketch_restore(h: int, theta: float, cap: int, stream: int = 0, _fn="sketch_restore",
                   buf=None):
    """Returns (records[:n], info). Raises SketchError (with n_needed on
    CAPACITY). buf: an optional record buffer of at least cap entries to
    write into (the returned records are a copy)."""
    out = _host_buf(cap, buf)                          # the first n are written
    n = c_sz(0)
    info = sketch_info_t()
    rc = getattr(lib(), _fn)(h, float(theta), out.ctypes.data, cap,
                             ctypes.byref(n), ctypes.byref(info), stream)
    if rc != SKETCH_OK:
        err = SketchError(rc, last_error(), n.value)
        err.info = info_dict(info)
        raise err
    return _records(out, n.value), info_dict(info)


def sketch_restore_noalloc(h: int, theta: float, cap: int, stream: int = 0, buf=None):
    """sketch_restore_noalloc: as sketch_restore, on the library's fixed
    per-GPU work array (no allocation inside the call)."""
    return sketch_restore(h, theta, cap, stream, _fn="sketch_restore_noalloc", buf=buf)


class _RestoreJobs:
    """A job array for the batched restore calls and the host buffers its
    entries point at (kept alive together)."""

    def __init__(self, items):
        """items: (handle, theta, cap) or (handle, theta, cap, buffer)."""
        self.n = len(items)
        self.arr = (sketch_restore_job_t * max(1, self.n))()
        self.outs, self.infos = [], []
        for i, item in enumerate(items):
            h, theta, cap = item[:3]
            out = _host_buf(cap, item[3] if len(item) > 3 else None)   # the first n are written
            info = sketch_info_t()
            self.outs.append(out)
            self.infos.append(info)
            self.arr[i] = sketch_restore_job_t(h, float(theta), out.ctypes.data, cap,
                                               ctypes.addressof(info), 0, 0)

    def call(self, fn, stream: int) -> None:
        rc = fn(ctypes.cast(self.arr, c_vp), self.n, stream)
        if rc == SKETCH_E_INVAL and all(self.arr[i].status == 0 for i in range(self.n)):
            raise SketchError(rc, last_error())

    def results(self):
        res = []
        for i in range(self.n):
            st = self.arr[i].status
            recs = _records(self.outs[i], self.arr[i].n_out if st == SKETCH_OK else 0)
            res.append((recs, info_dict(self.infos[i]), st, self.arr[i].n_out))
        return res


def sketch_restore_batch(items, stream: int = 0):
    """items: sequence of (handle, theta, cap). Returns a list of
    (records, info, status, n_needed) per item, in order."""
    jobs = _RestoreJobs(items)
    jobs.call(lib().sketch_restore_batch, stream)
    return jobs.results()


def sketch_restore_batch_begin(items, stream: int = 0) -> _RestoreJobs:
    """items: sequence of (handle, theta, cap). Enqueues the restores and
    returns the pending jobs for sketch_restore_batch_end."""
    jobs = _RestoreJobs(items)
    jobs.call(lib().sketch_restore_batch_begin, stream)
    return jobs


def sketch_restore_batch_end(jobs: _RestoreJobs, stream: int = 0):
    """Waits for the pending restores; results as sketch_restore_batch."""
    jobs.call(lib().sketch_restore_batch_end, stream)
    return jobs.results()


def sketch_plan_create(jobs, flags: int) -> int:
    """jobs: sequence of (handle, d_pairs, n_pairs, theta). Returns the plan."""
    arr = (sketch_plan_job_t * max(1, len(jobs)))()
    for i, (h, ptr, n, theta) in enumerate(jobs):
        arr[i] = sketch_plan_job_t(h, ptr, n, float(theta))
    out = c_vp()
    _check(lib().sketch_plan_create(ctypes.cast(arr, c_vp), len(jobs), flags,
                                    ctypes.byref(out)))
    return out.value


def sketch_plan_run(plan: int, stream: int = 0) -> None:
    _check(lib().sketch_plan_run(plan, stream))


def sketch_plan_results(plan: int, items, stream: int = 0):
    """items: sequence of (handle, cap) or (handle, cap, buffer) in job
    order. Returns a list of (records, info, status, n_needed)."""
    n = len(items)
    arr = (sketch_restore_job_t * max(1, n))()
    outs, infos = [], []
    for i, item in enumerate(items):
        h, cap = item[:2]
        out = _host_buf(cap, item[2] if len(item) > 2 else None)   # the first n are written
        info = sketch_info_t()
        outs.append(out)
        infos.append(info)
        arr[i] = sketch_restore_job_t(h, 0.0, out.ctypes.data, cap, ctypes.addressof(info), 0, 0)
    rc = lib().sketch_plan_results(plan, ctypes.cast(arr, c_vp), n, stream)
    if rc == SKETCH_E_INVAL and all(arr[i].status == 0 for i in range(n)):
        raise SketchError(rc, last_error())
    res = []
    for i in range(n):
        st = arr[i].status
        recs = _records(outs[i], arr[i].n_out if st == SKETCH_OK else 0)
        res.append((recs, info_dict(infos[i]), st, arr[i].n_out))
    return res


def sketch_candidates(h: int, theta: float, cap: int, stream: int = 0) -> np.ndarray:
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    n = c_sz(0)
    rc = lib().sketch_candidates(h, float(theta), out.ctypes.data, cap,
                                 ctypes.byref(n), stream)
    _check(rc, n.value)
    return out[: n.value].copy()


def sketch_timings(h: int) -> dict:
    """Phase times and work of the last restore run with SKETCH_OPT_TIMING."""
    t = sketch_timings_t()
    _check(lib().sketch_timings(h, ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in sketch_timings_t._fields_}


def sketch_merge(dst: int, src: int, stream: int = 0) -> None:
    _check(lib().sketch_merge(dst, src, stream))


def sketch_download(h: int, n_words: int, stream: int = 0) -> np.ndarray:
    out = np.zeros(n_words, dtype=np.uint32)
    _check(lib().sketch_download(h, out.ctypes.data, n_words, stream))
    return out


def sketch_upload(h: int, words: np.ndarray, stream: int = 0) -> None:
    words = np.ascontiguousarray(words, dtype=np.uint32)
    _check(lib().sketch_upload(h, words.ctypes.data, words.size, stream))


def info_dict(info: sketch_info_t) -> dict:
    return {
        "zr": list(info.zr), "he_count": list(info.he_count),
        "n_partials": list(info.n_partials),
        "n_candidates": info.n_candidates, "n_reported": info.n_reported,
        "psi": info.psi, "d": info.d, "zmin": info.zmin, "trep": info.trep,
        "zhot": info.zhot, "szmax": info.szmax,
    }


# ------------------------------------------------------------ torch facade

def _stream_handle(stream, device) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _check_pairs(pairs):
    import torch
    if not isinstance(pairs, torch.Tensor) or not pairs.is_cuda:
        raise TypeError("pairs must be a CUDA tensor")
    if pairs.element_size() != 4 or not pairs.is_contiguous():
        raise TypeError("pairs must be a contiguous 32-bit tensor")
    if pairs.numel() % 2:
        raise ValueError("pairs must hold an even number of words")


def update_batch(items, stream=None) -> None:
    """items: sequence of (Sketch, pairs tensor). One batched update."""
    if not items:
        return
    for _, t in items:
        _check_pairs(t)
    dev = items[0][0].device
    sketch_update_batch([(sk.handle, t.data_ptr(), t.numel() // 2) for sk, t in items],
                        _stream_handle(stream, dev))


def restore_batch(items, stream=None, raise_errors: bool = True):
    """items: sequence of (Sketch, theta). One batched restore; returns
    [(records, info)] in order. CAPACITY jobs are rerun in a second batch.
    Another failed job raises SketchError, or with raise_errors=False comes
    back as (None, info) with info["status"] set (info of a SATURATED job
    still holds its scalars)."""
    if not items:
        return []
    dev = items[0][0].device
    s = _stream_handle(stream, dev)
    res = sketch_restore_batch([(sk.handle, th, sk._cap, sk._buf()) for sk, th in items], s)
    return _collect(items, res, stream, raise_errors)


def _collect(items, res, stream, raise_errors):
    """Per-item results of a batched restore; CAPACITY jobs run again in a
    second (synchronous) batch with room for their lists."""
    out = [None] * len(items)
    retry = []
    for i, ((sk, th), (recs, info, st, need)) in enumerate(zip(items, res)):
        info["status"] = st
        if st == SKETCH_OK:
            out[i] = (recs, info)
        elif st == SKETCH_E_CAPACITY:
            sk._cap = max(int(need) + 64, 2 * sk._cap)
            retry.append(i)
        elif raise_errors:
            raise SketchError(st, f"restore of batch item {i} failed: {last_error()}")
        else:
            out[i] = (None, info)
    if retry:
        again = restore_batch([items[i] for i in retry], stream, raise_errors)
        for i, r in zip(retry, again):
            out[i] = r
    return out


class PendingRestore:
    """Restores enqueued by restore_batch_begin; end() collects them."""

    def __init__(self, items, stream=None):
        self.items = list(items)
        self.dev = self.items[0][0].device if self.items else None
        self.stream = stream
        self.jobs = None
        if self.items:
            self.jobs = sketch_restore_batch_begin(
                [(sk.handle, th, sk._cap, sk._buf()) for sk, th in self.items],
                _stream_handle(stream, self.dev))

    def end(self, raise_errors: bool = True):
        """[(records, info)] in item order, as restore_batch returns them."""
        if not self.items:
            return []
        res = sketch_restore_batch_end(self.jobs, _stream_handle(self.stream, self.dev))
        return _collect(self.items, res, self.stream, raise_errors)


def restore_batch_begin(items, stream=None) -> PendingRestore:
    """items: sequence of (Sketch, theta). Enqueues one batched restore on
    the stream and returns without waiting (sketch_restore_batch_begin)."""
    return PendingRestore(items, stream)


class Plan:
    """A fixed batch's window cycle as one HIP graph (sketch_plan_*).

    items: sequence of (Sketch, pairs tensor, theta). The tensors must stay
    alive and in place while the plan is used; close the plan before its
    sketches."""

    def __init__(self, items, reset: bool = True, restore: bool = True):
        for _, t, _ in items:
            _check_pairs(t)
        self.items = list(items)
        self.device = self.items[0][0].device
        flags = (SKETCH_PLAN_RESET if reset else 0) | (SKETCH_PLAN_RESTORE if restore else 0)
        self.handle = sketch_plan_create(
            [(sk.handle, t.data_ptr(), t.numel() // 2, th) for sk, t, th in self.items], flags)

    @property
    def launches(self) -> int:
        return lib().sketch_plan_launches(self.handle)

    def run(self, stream=None) -> None:
        sketch_plan_run(self.handle, _stream_handle(stream, self.device))

    def results(self, stream=None):
        """[(records, info)] of the last run, in item order."""
        s = _stream_handle(stream, self.device)
        while True:
            res = sketch_plan_results(self.handle, [(sk.handle, sk._cap, sk._buf())
                                                    for sk, _, _ in self.items], s)
            retry = False
            for (sk, _, _), (_, _, st, need) in zip(self.items, res):
                if st == SKETCH_E_CAPACITY:
                    sk._cap = max(int(need) + 64, 2 * sk._cap)
                    retry = True
                elif st != SKETCH_OK:
                    raise SketchError(st, f"plan result failed: {last_error()}")
            if not retry:
                return [(recs, info) for recs, info, _, _ in res]

    def close(self) -> None:
        if self.handle:
            sketch_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sketch_plan_destroy(plan: int) -> None:
    lib().sketch_plan_destroy(plan)


class Sketch:
    """One DDHF sketch on a GPU (r rows of 2^k LEs of g bits)."""

    def __init__(self, g=1024, k=14, r=5, alpha=6, seed=DEFAULT_SEED, device=None):
        import torch
        if device is None:
            device = torch.cuda.current_device()
        elif isinstance(device, torch.device):
            device = device.index or 0
        self.device = int(device)
        self.params = sketch_params_t(g, k, r, alpha, seed, self.device)
        self.words = sketch_bytes(self.params) // 4
        self.handle = sketch_create(self.params)
        self._cap = 1 << 12
        self._outbuf = None

    # pairs: CUDA tensor of 2n 32-bit words (int32/uint32, [n,2] or [2n])
    def update(self, pairs, stream=None) -> None:
        _check_pairs(pairs)
        sketch_update(self.handle, pairs.data_ptr(), pairs.numel() // 2,
                      _stream_handle(stream, pairs.device))

    def set_option(self, option: int, value: int) -> None:
        sketch_set_option(self.handle, option, value)

    def update_ptr(self, d_pairs: int, n_pairs: int, stream: int = 0) -> None:
        sketch_update(self.handle, d_pairs, n_pairs, stream)

    def _buf(self) -> np.ndarray:
        """This handle's host record buffer, at least _cap entries (restores
        write into it; what they return is a copy)."""
        if self._outbuf is None or len(self._outbuf) < max(self._cap, 1):
            self._outbuf = np.empty(max(self._cap, 1), dtype=SP_DTYPE)
        return self._outbuf

    def restore(self, theta: float, stream=None):
        """(records ascending by ip, info dict)."""
        s = _stream_handle(stream, self.device)
        while True:
            try:
                recs, info = sketch_restore(self.handle, theta, self._cap, s, buf=self._buf())
                return recs, info
            except SketchError as e:
                if e.code != SKETCH_E_CAPACITY:
                    raise
                self._cap = max(int(e.n_needed) + 64, 2 * self._cap)

    def restore_noalloc(self, theta: float, stream=None):
        """restore() through sketch_restore_noalloc (records, info)."""
        s = _stream_handle(stream, self.device)
        while True:
            try:
                return sketch_restore_noalloc(self.handle, theta, self._cap, s, buf=self._buf())
            except SketchError as e:
                if e.code != SKETCH_E_CAPACITY or not e.n_needed or e.n_needed <= self._cap:
                    raise
                self._cap = max(int(e.n_needed) + 64, 2 * self._cap)

    def candidates(self, theta: float, stream=None) -> np.ndarray:
        s = _stream_handle(stream, self.device)
        cap = 1 << 14
        while True:
            try:
                return sketch_candidates(self.handle, theta, cap, s)
            except SketchError as e:
                if e.code != SKETCH_E_CAPACITY:
                    raise
                cap = int(e.n_needed) + 64

    def reset(self, stream=None) -> None:
        sketch_reset(self.handle, _stream_handle(stream, self.device))

    def download(self, stream=None) -> np.ndarray:
        return sketch_download(self.handle, self.words, _stream_handle(stream, self.device))

    def upload(self, words: np.ndarray, stream=None) -> None:
        sketch_upload(self.handle, words, _stream_handle(stream, self.device))

    def merge(self, other: "Sketch", stream=None) -> None:
        """OR another monitor's sketch of the same window into this one."""
        sketch_merge(self.handle, other.handle, _stream_handle(stream, self.device))

    def save(self, path: str) -> None:
        """Snapshot: the sketch words and parameters to an .npz file."""
        p = self.params
        np.savez(path, words=self.download(),
                 params=np.array([p.g, p.k, p.r, p.alpha], dtype=np.uint32),
                 seed=np.array([p.seed], dtype=np.uint64))

    @classmethod
    def load(cls, path: str, device=None) -> "Sketch":
        """A sketch restored from a snapshot written by save()."""
        with np.load(path, allow_pickle=False) as z:
            g, k, r, alpha = (int(x) for x in z["params"])
            sk = cls(g, k, r, alpha, int(z["seed"][0]), device=device)
            sk.upload(z["words"])
        return sk

    def close(self) -> None:
        if getattr(self, "handle", None):
            sketch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
