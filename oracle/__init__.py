"""CPU oracle for DDHF super point detection (arXiv 1803.11449).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU product path
never does. It wraps ``ddhf_oracle.c`` (plain C, built with gcc) and shares no
code with the GPU library.

Every function follows the paper directly:
  update         Alg. 1 (Sec. 3.2); update_omp, the same on several threads
  zero_counts    z0 per LE (Alg. 2) and ZR(i) (Sec. 3.3)
  scalars        Lemma 1 with the flow-count estimate of Sec. 3.3, Zmin of
                 Alg. 2, the denominator of eq. (4)
  hot_lists      HE(i), first loop of Alg. 2
  candidates     Algs. 3-4 join (mode "join"), all 2^32 addresses ("brute"),
                 every tuple of hot LEs judged by the address it names
                 ("tuples"), join without the re-hash test ("join_norehash")
  estimate       ULE, SZ (Def. 1) and C by eq. (4)
  restore        Alg. 2 end to end
  exact_cardinality  |CO(a)| per measured host (Sec. 3.1), by sort/unique
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddhf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, E_INVAL, E_NOMEM, E_SATURATED = 0, -1, -2, -5

MODES = {"join": 0, "brute": 1, "tuples": 2, "join_norehash": 3}


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u32, u64, i32, i64, sz, dbl = (ctypes.c_uint32, ctypes.c_uint64,
                                       ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_size_t, ctypes.c_double)
        vp = ctypes.c_void_p
        sig = {
            "orc_check_params": (i32, [u32, u32, u32, u32]),
            "orc_splitmix64": (None, [u64, vp, sz]),
            "orc_hash_coeffs": (None, [u64, vp]),
            "orc_dh": (i32, [u32, u32, u32, u32, u64, u32, vp, vp, sz]),
            "orc_h1": (i32, [u32, u32, u32, u32, u64, vp, vp, sz]),
            "orc_sketch_words": (sz, [u32, u32, u32]),
            "orc_update": (i32, [u32, u32, u32, u32, u64, vp, vp, sz]),
            "orc_update_omp": (i32, [u32, u32, u32, u32, u64, vp, vp, sz, i32]),
            "orc_zero_counts": (i32, [u32, u32, u32, u32, vp, vp, vp]),
            "orc_scalars": (i32, [u32, u32, u32, vp, dbl, vp]),
            "orc_hot_lists": (i32, [u32, u32, u32, u32, vp, dbl, vp, vp]),
            "orc_candidates": (i64, [u32, u32, u32, u32, u64, vp, dbl, i32,
                                     i32, vp, sz]),
            "orc_estimate": (i32, [u32, u32, u32, u32, u64, vp, dbl, vp, sz,
                                   vp, vp]),
            "orc_restore": (i64, [u32, u32, u32, u32, u64, vp, dbl, i32, i32,
                                  vp, vp, vp, sz, vp]),
            "orc_exact_cardinality": (i64, [vp, sz, vp, vp, sz]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def default_threads() -> int:
    """Threads for the parallel parts (the 2^32 scan): the CPU share this
    process may use (affinity, OMP_NUM_THREADS), at most 16."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, min(n, 16))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise OracleError(rc, what)
    return rc


class Params:
    """Sketch parameters: g bits per LE, 2^k LEs per row, r rows, block
    stride alpha (Sec. 3.2-3.3), and the seed the hash coefficients come
    from."""

    def __init__(self, g=1024, k=14, r=5, alpha=6, seed=0x1803114490000001):
        self.g, self.k, self.r, self.alpha = int(g), int(k), int(r), int(alpha)
        self.seed = int(seed)

    def t(self):
        return (self.g, self.k, self.r, self.alpha)

    def words(self) -> int:
        return self.r * (1 << self.k) * (self.g // 32)


def check_params(p: Params) -> bool:
    return lib().orc_check_params(*p.t()) == OK


def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_splitmix64(seed, _ptr(out), n)
    return out


def hash_coeffs(seed: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_hash_coeffs(seed, _ptr(out))
    return out


def dh(p: Params, i: int, a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    out = np.empty_like(a)
    _check(lib().orc_dh(*p.t(), p.seed, i, _ptr(a), _ptr(out), a.size), "dh")
    return out


def h1(p: Params, b) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint32)
    out = np.empty_like(b)
    _check(lib().orc_h1(*p.t(), p.seed, _ptr(b), _ptr(out), b.size), "h1")
    return out


def new_sketch(p: Params) -> np.ndarray:
    return np.zeros(p.words(), dtype=np.uint32)


def as_pairs(pairs) -> np.ndarray:
    """Interleaved uint32 (a,b) pairs as a flat array of 2n words."""
    arr = np.ascontiguousarray(pairs)
    if arr.dtype != np.uint32:
        arr = arr.view(np.uint32) if arr.dtype.itemsize == 4 else arr.astype(np.uint32)
    return np.ascontiguousarray(arr.reshape(-1))


def update(p: Params, sketch: np.ndarray, pairs) -> np.ndarray:
    flat = as_pairs(pairs)
    assert sketch.dtype == np.uint32 and sketch.size == p.words()
    _check(lib().orc_update(*p.t(), p.seed, _ptr(sketch), _ptr(flat),
                            flat.size // 2), "update")
    return sketch


def update_omp(p: Params, sketch: np.ndarray, pairs, nthreads: int | None = None) -> np.ndarray:
    """Alg. 1 on several threads (same sketch as update)."""
    flat = as_pairs(pairs)
    assert sketch.dtype == np.uint32 and sketch.size == p.words()
    _check(lib().orc_update_omp(*p.t(), p.seed, _ptr(sketch), _ptr(flat), flat.size // 2,
                                nthreads or default_threads()), "update_omp")
    return sketch


def build_sketch(p: Params, pairs) -> np.ndarray:
    return update(p, new_sketch(p), pairs)


def zero_counts(p: Params, sketch: np.ndarray):
    z0 = np.zeros(p.r << p.k, dtype=np.uint32)
    zr = np.zeros(p.r, dtype=np.uint64)
    _check(lib().orc_zero_counts(*p.t(), _ptr(sketch), _ptr(z0), _ptr(zr)),
           "zero_counts")
    return z0.reshape(p.r, 1 << p.k), zr


def scalars(p: Params, zr, theta: float) -> dict:
    zr = np.ascontiguousarray(zr, dtype=np.uint64)
    out = np.zeros(4, dtype=np.float64)
    _check(lib().orc_scalars(p.g, p.k, p.r, _ptr(zr), float(theta), _ptr(out)),
           "scalars")
    return {"psi": out[0], "D": out[1], "zmin": out[2], "w": out[3]}


def hot_lists(p: Params, sketch: np.ndarray, theta: float):
    he = np.zeros(p.r << p.k, dtype=np.uint32)
    he_n = np.zeros(8, dtype=np.uint32)
    _check(lib().orc_hot_lists(*p.t(), _ptr(sketch), float(theta), _ptr(he),
                               _ptr(he_n)), "hot_lists")
    he = he.reshape(p.r, 1 << p.k)
    return [he[i, :he_n[i]].copy() for i in range(p.r)]


def candidates(p: Params, sketch: np.ndarray, theta: float, mode="join",
               nthreads: int | None = None) -> np.ndarray:
    nth = nthreads or default_threads()
    cap = 1 << 16
    while True:
        out = np.zeros(cap, dtype=np.uint32)
        n = _check(lib().orc_candidates(*p.t(), p.seed, _ptr(sketch),
                                        float(theta), MODES[mode], nth,
                                        _ptr(out), cap), "candidates")
        if n <= cap:
            return out[:n].copy()
        cap = n


def estimate(p: Params, sketch: np.ndarray, psi: float, ips):
    ips = np.ascontiguousarray(ips, dtype=np.uint32)
    sz = np.zeros(ips.size, dtype=np.uint32)
    c = np.zeros(ips.size, dtype=np.float64)
    _check(lib().orc_estimate(*p.t(), p.seed, _ptr(sketch), float(psi),
                              _ptr(ips), ips.size, _ptr(sz), _ptr(c)),
           "estimate")
    return sz, c


def restore(p: Params, sketch: np.ndarray, theta: float, mode="join",
            nthreads: int | None = None):
    """Alg. 2: returns (ips, sz, C, scalars) ascending by address."""
    nth = nthreads or default_threads()
    cap = 1 << 14
    while True:
        ip = np.zeros(cap, dtype=np.uint32)
        sz = np.zeros(cap, dtype=np.uint32)
        c = np.zeros(cap, dtype=np.float64)
        sc = np.zeros(4, dtype=np.float64)
        n = _check(lib().orc_restore(*p.t(), p.seed, _ptr(sketch), float(theta),
                                     MODES[mode], nth, _ptr(ip), _ptr(sz),
                                     _ptr(c), cap, _ptr(sc)), "restore")
        if n <= cap:
            return (ip[:n].copy(), sz[:n].copy(), c[:n].copy(),
                    {"psi": sc[0], "D": sc[1], "zmin": sc[2], "w": sc[3]})
        cap = n


def exact_cardinality(pairs):
    """(hosts ascending, |CO(host)|) for every measured host."""
    flat = as_pairs(pairs)
    n = flat.size // 2
    cap = max(n, 1)
    host = np.zeros(cap, dtype=np.uint32)
    card = np.zeros(cap, dtype=np.uint32)
    m = _check(lib().orc_exact_cardinality(_ptr(flat), n, _ptr(host),
                                           _ptr(card), cap), "exact_cardinality")
    return host[:m].copy(), card[:m].copy()
