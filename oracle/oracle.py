"""ctypes front end of the CPU oracle in ``imin_oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's
CPU-baseline leg, never by the library. ``build()`` compiles the C file with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "imin_oracle.c")
_LIB = os.path.join(_HERE, "libimin_oracle.so")

AG, GR = 0, 1
IC, LT = 0, 1  # propagation models: independent cascade; linear threshold (triggering)

_lib = None


def build() -> str:
    """Compile the oracle with gcc (plain C99, -O2) next to its source."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-pthread", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    """The oracle library: the build next to the source (rebuilt when older than it), or,
    when IMIN_ORACLE_LIB names a file, that build of the same source as it is (the
    sanitizer builds of ``sanitize.sh``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("IMIN_ORACLE_LIB") or _LIB
    if path == _LIB and (not os.path.exists(_LIB) or
                         os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_philox4x32_10.restype = None
    lib.orc_threshold.argtypes = [ctypes.c_float]
    lib.orc_threshold.restype = ctypes.c_uint32
    lib.orc_edge_live.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_float]
    lib.orc_edge_live.restype = ctypes.c_int
    lib.orc_sample.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P, ctypes.c_uint64,
                               ctypes.c_uint32, P, P]
    lib.orc_sample.restype = ctypes.c_int64
    lib.orc_sample_m.argtypes = lib.orc_sample.argtypes + [ctypes.c_int]
    lib.orc_sample_m.restype = ctypes.c_int64
    lib.orc_lt_trigger.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_int32]
    lib.orc_lt_trigger.restype = ctypes.c_int64
    lib.orc_decrease.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P, ctypes.c_uint32,
                                 ctypes.c_uint64, P, P]
    lib.orc_decrease.restype = ctypes.c_int
    lib.orc_decrease_m.argtypes = lib.orc_decrease.argtypes + [ctypes.c_int]
    lib.orc_decrease_m.restype = ctypes.c_int
    lib.orc_greedy.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, P, P, P, P]
    lib.orc_greedy.restype = ctypes.c_int
    lib.orc_greedy_m.argtypes = lib.orc_greedy.argtypes + [ctypes.c_int]
    lib.orc_greedy_m.restype = ctypes.c_int
    lib.orc_decrease_mt.argtypes = lib.orc_decrease_m.argtypes + [ctypes.c_int]
    lib.orc_decrease_mt.restype = ctypes.c_int
    lib.orc_greedy_mt.argtypes = lib.orc_greedy_m.argtypes + [ctypes.c_int]
    lib.orc_greedy_mt.restype = ctypes.c_int
    lib.orc_lt_bounds.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int32, P]
    lib.orc_lt_bounds.restype = ctypes.c_int64
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph(row_ptr, col, prob):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    prob = np.ascontiguousarray(prob, dtype=np.float32)
    return row_ptr, col, prob


class OracleError(RuntimeError):
    pass


def philox(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def threshold(p: float) -> int:
    return int(_load().orc_threshold(float(p)))


def edge_live(key: int, j: int, e: int, p: float) -> bool:
    return bool(_load().orc_edge_live(key, j, e, float(p)))


def lt_trigger(n, row_ptr, col, w, key: int, j: int, u: int) -> int:
    """LT: the in-edge id u chooses in sample j (its triggering set), or -1."""
    row_ptr, col, w = _graph(row_ptr, col, w)
    r = _load().orc_lt_trigger(n, _ptr(row_ptr), _ptr(col), _ptr(w), key, j, u)
    if r < -1:
        raise OracleError(f"orc_lt_trigger failed: {r}")
    return int(r)


def sample(n, row_ptr, col, prob, seeds, blocked, key: int, j: int, model: int = IC):
    """One sampled graph: (reached count, c[n], idom[n]); see orc_sample."""
    lib = _load()
    row_ptr, col, prob = _graph(row_ptr, col, prob)
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    blk = None if blocked is None else np.ascontiguousarray(blocked, dtype=np.uint8)
    c = np.zeros(n, dtype=np.int32)
    idom = np.zeros(n, dtype=np.int32)
    r = lib.orc_sample_m(n, _ptr(row_ptr), _ptr(col), _ptr(prob), _ptr(S), S.shape[0],
                         _ptr(blk), key, j, _ptr(c), _ptr(idom), model)
    if r < 0:
        raise OracleError(f"orc_sample failed: {r}")
    return int(r), c, idom


def lt_bounds(n, row_ptr, col, w, u: int):
    """LT: the interval upper ends of u's in-edges, ascending edge id (orc_lt_bounds)."""
    row_ptr, col, w = _graph(row_ptr, col, w)
    out = np.zeros(max(1, int(np.count_nonzero(col == u))), dtype=np.uint32)
    k = _load().orc_lt_bounds(n, _ptr(row_ptr), _ptr(col), _ptr(w), u, _ptr(out))
    if k < 0:
        raise OracleError(f"orc_lt_bounds failed: {k}")
    return out[:k].copy()


def decrease(n, row_ptr, col, prob, seeds, blocked, theta: int, key: int, model: int = IC,
             threads: int = 1):
    """Integer decrease counts D[n] and stats (samples, reached, edges scanned, live edges).
    threads > 1: the samples spread over that many host threads (same result)."""
    lib = _load()
    row_ptr, col, prob = _graph(row_ptr, col, prob)
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    blk = None if blocked is None else np.ascontiguousarray(blocked, dtype=np.uint8)
    D = np.zeros(n, dtype=np.uint64)
    st = np.zeros(4, dtype=np.uint64)
    if threads > 1:
        rc = lib.orc_decrease_mt(n, _ptr(row_ptr), _ptr(col), _ptr(prob), _ptr(S), S.shape[0],
                                 _ptr(blk), theta, key, _ptr(D), _ptr(st), model, threads)
    else:
        rc = lib.orc_decrease_m(n, _ptr(row_ptr), _ptr(col), _ptr(prob), _ptr(S), S.shape[0],
                                _ptr(blk), theta, key, _ptr(D), _ptr(st), model)
    if rc != 0:
        raise OracleError(f"orc_decrease failed: {rc}")
    return D, dict(samples=int(st[0]), reached=int(st[1]), edges_scanned=int(st[2]),
                   live_edges=int(st[3]))


def greedy(n, row_ptr, col, prob, seeds, b: int, theta: int, seed: int, mode: int,
           model: int = IC, threads: int = 1):
    """Blocker slots in order, number of decrease calls, summed stats.
    threads > 1: every decrease call spread over that many host threads (same result)."""
    lib = _load()
    row_ptr, col, prob = _graph(row_ptr, col, prob)
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    out = np.zeros(max(b, 1), dtype=np.int32)
    nb = np.zeros(1, dtype=np.int32)
    calls = np.zeros(1, dtype=np.int32)
    st = np.zeros(4, dtype=np.uint64)
    if threads > 1:
        rc = lib.orc_greedy_mt(n, _ptr(row_ptr), _ptr(col), _ptr(prob), _ptr(S), S.shape[0], b,
                               theta, seed, mode, _ptr(out), _ptr(nb), _ptr(calls), _ptr(st),
                               model, threads)
    else:
        rc = lib.orc_greedy_m(n, _ptr(row_ptr), _ptr(col), _ptr(prob), _ptr(S), S.shape[0], b,
                              theta, seed, mode, _ptr(out), _ptr(nb), _ptr(calls), _ptr(st),
                              model)
    if rc != 0:
        raise OracleError(f"orc_greedy failed: {rc}")
    return out[: nb[0]].copy(), int(calls[0]), dict(samples=int(st[0]), reached=int(st[1]),
                                                     edges_scanned=int(st[2]),
                                                     live_edges=int(st[3]))
