"""ctypes binding of libimin (include/imin.h): argument marshalling only.

The functions keep the C names (``imin_graph_create``, ``imin_decrease``, ``imin_spread``,
``imin_greedy``, ``imin_greedy_batch``, ``imin_set_launch``, ``imin_set_small``,
``imin_graph_destroy``, ``imin_server_*``, ``imin_strerror``); ``Graph`` and ``Server`` wrap
them for convenience. Every step
of the estimate runs in the library's HIP kernels; if the library is missing this module
raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimin.so")

IMIN_OK, IMIN_EINVAL, IMIN_ENOMEM, IMIN_EDEVICE, IMIN_ERANGE = 0, -1, -2, -3, -4
IMIN_AG, IMIN_GR = 0, 1
IMIN_IC, IMIN_LT = 0, 1


class IminError(RuntimeError):
    def __init__(self, func: str, status: int):
        super().__init__(f"{func} failed: {status} ({imin_strerror(status)})")
        self.status = status


class imin_stats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_uint64), ("reached", ctypes.c_uint64),
                ("edges_scanned", ctypes.c_uint64), ("live_edges", ctypes.c_uint64),
                ("spilled", ctypes.c_uint64), ("device_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("wave_samples", ctypes.c_uint64),
                ("pack_samples", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class imin_launch(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("quad_limit", ctypes.c_int32),
                ("pick_div", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("pack_per_cu", ctypes.c_int32)]


def _launch(launch):
    """None, a dict with any of the imin_launch fields, or an imin_launch."""
    if launch is None:
        return None
    if isinstance(launch, imin_launch):
        return ctypes.byref(launch)
    return ctypes.byref(imin_launch(**{k: int(v) for k, v in launch.items()}))


class imin_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_active", ctypes.c_int32),
                ("max_theta", ctypes.c_uint32), ("launch", imin_launch)]


class imin_instance(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("S", ctypes.c_void_p), ("nS", ctypes.c_int32),
                ("b", ctypes.c_int32), ("theta", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("blockers", ctypes.c_void_p), ("n_blockers", ctypes.c_void_p),
                ("stats", ctypes.POINTER(imin_stats))]


_lib = None


def load() -> ctypes.CDLL:
    """Load libimin.so (built by ``paper_2302_13529_amd.build``); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; importing it first makes libimin bind to that same
    # runtime instead of loading a second copy into the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2302_13529_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.imin_graph_create.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P,
                                      ctypes.POINTER(ctypes.c_void_p)]
    lib.imin_graph_create.restype = ctypes.c_int
    lib.imin_graph_create_model.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_void_p)]
    lib.imin_graph_create_model.restype = ctypes.c_int
    lib.imin_graph_destroy.argtypes = [P]
    lib.imin_graph_destroy.restype = None
    lib.imin_decrease.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_uint32, ctypes.c_uint64, P,
                                  ctypes.POINTER(imin_stats)]
    lib.imin_decrease.restype = ctypes.c_int
    lib.imin_spread.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(imin_stats)]
    lib.imin_spread.restype = ctypes.c_int
    lib.imin_greedy.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_int, P, P, ctypes.POINTER(imin_stats)]
    lib.imin_greedy.restype = ctypes.c_int
    lib.imin_set_launch.argtypes = [P, ctypes.c_int32, ctypes.c_int64]
    lib.imin_set_launch.restype = ctypes.c_int
    lib.imin_set_small.argtypes = [P, ctypes.c_int32, P]
    lib.imin_set_small.restype = ctypes.c_int
    lib.imin_greedy_batch.argtypes = [ctypes.POINTER(imin_instance), ctypes.c_int32,
                                      ctypes.c_int, P]
    lib.imin_greedy_batch.restype = ctypes.c_int
    lib.imin_server_create.argtypes = [P, ctypes.POINTER(imin_server_config),
                                       ctypes.POINTER(ctypes.c_void_p)]
    lib.imin_server_create.restype = ctypes.c_int
    lib.imin_server_destroy.argtypes = [P]
    lib.imin_server_destroy.restype = None
    lib.imin_server_query_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_uint64)]
    lib.imin_server_query_bytes.restype = ctypes.c_int
    lib.imin_server_submit.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                       ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    lib.imin_server_submit.restype = ctypes.c_int
    lib.imin_server_submit_mode.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_uint64)]
    lib.imin_server_submit_mode.restype = ctypes.c_int
    lib.imin_server_step.argtypes = [P, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
    lib.imin_server_step.restype = ctypes.c_int
    lib.imin_server_completed.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.imin_server_completed.restype = ctypes.c_int
    lib.imin_server_result.argtypes = [P, ctypes.c_uint64, P, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(imin_stats)]
    lib.imin_server_result.restype = ctypes.c_int
    lib.imin_decrease_noalloc.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_uint32,
                                          ctypes.c_uint64, P, ctypes.POINTER(imin_stats)]
    lib.imin_decrease_noalloc.restype = ctypes.c_int
    lib.imin_strerror.argtypes = [ctypes.c_int]
    lib.imin_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def imin_strerror(status: int) -> str:
    return load().imin_strerror(status).decode()


def imin_graph_create(n: int, row_ptr, col, prob, model: int = IMIN_IC) -> int:
    """Returns the opaque handle (an integer address)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    prob = np.ascontiguousarray(prob, dtype=np.float32)
    h = ctypes.c_void_p()
    rc = load().imin_graph_create_model(int(n), int(col.shape[0]), _p(row_ptr), _p(col),
                                        _p(prob), int(model), ctypes.byref(h))
    if rc != IMIN_OK:
        raise IminError("imin_graph_create", rc)
    return h.value


def imin_graph_destroy(handle: int) -> None:
    load().imin_graph_destroy(ctypes.c_void_p(handle))


def imin_set_launch(handle: int, slots: int = 0, extra_cap: int = 0) -> None:
    rc = load().imin_set_launch(ctypes.c_void_p(handle), int(slots), int(extra_cap))
    if rc != IMIN_OK:
        raise IminError("imin_set_launch", rc)


def imin_set_small(handle: int, enable: int = -1, launch=None) -> None:
    rc = load().imin_set_small(ctypes.c_void_p(handle), int(enable), _launch(launch))
    if rc != IMIN_OK:
        raise IminError("imin_set_small", rc)


def imin_decrease(handle: int, n: int, seeds, blocked, theta: int, seed: int):
    """Exact counts D (uint64[n]) and the stats dict of one Algorithm 2 call."""
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    blk = None if blocked is None else np.ascontiguousarray(blocked, dtype=np.uint8)
    if blk is not None and blk.shape[0] != n:
        raise ValueError("blocked must have n entries")
    D = np.zeros(n, dtype=np.uint64)
    st = imin_stats()
    rc = load().imin_decrease(ctypes.c_void_p(handle), _p(S), S.shape[0], _p(blk), int(theta),
                              int(seed) & (2**64 - 1), _p(D), ctypes.byref(st))
    if rc != IMIN_OK:
        raise IminError("imin_decrease", rc)
    return D, st.as_dict()


def imin_decrease_noalloc(handle: int, n: int, seeds, blocked, theta: int, seed: int,
                          d_counts: int):
    """Algorithm 2 into the caller's device buffer of n uint64 (address d_counts), through
    the entry point that allocates nothing; returns the stats dict."""
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    blk = None if blocked is None else np.ascontiguousarray(blocked, dtype=np.uint8)
    if blk is not None and blk.shape[0] != n:
        raise ValueError("blocked must have n entries")
    st = imin_stats()
    rc = load().imin_decrease_noalloc(ctypes.c_void_p(handle), _p(S), S.shape[0], _p(blk),
                                      int(theta), int(seed) & (2**64 - 1),
                                      ctypes.c_void_p(int(d_counts)), ctypes.byref(st))
    if rc != IMIN_OK:
        raise IminError("imin_decrease_noalloc", rc)
    return st.as_dict()


def imin_spread(handle: int, n: int, seeds, blocked, theta: int, seed: int):
    """Expected-spread estimate |S| + reached/theta and the stats dict."""
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    blk = None if blocked is None else np.ascontiguousarray(blocked, dtype=np.uint8)
    if blk is not None and blk.shape[0] != n:
        raise ValueError("blocked must have n entries")
    out = ctypes.c_double()
    st = imin_stats()
    rc = load().imin_spread(ctypes.c_void_p(handle), _p(S), S.shape[0], _p(blk), int(theta),
                            int(seed) & (2**64 - 1), ctypes.byref(out), ctypes.byref(st))
    if rc != IMIN_OK:
        raise IminError("imin_spread", rc)
    return out.value, st.as_dict()


def imin_greedy(handle: int, seeds, b: int, theta: int, seed: int, mode: int):
    """Blocker slots (int32) and the summed stats of AG (mode 0) or GR (mode 1)."""
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    out = np.zeros(max(int(b), 1), dtype=np.int32)
    nb = np.zeros(1, dtype=np.int32)
    st = imin_stats()
    rc = load().imin_greedy(ctypes.c_void_p(handle), _p(S), S.shape[0], int(b), int(theta),
                            int(seed) & (2**64 - 1), int(mode), _p(out), _p(nb),
                            ctypes.byref(st))
    if rc != IMIN_OK:
        raise IminError("imin_greedy", rc)
    return out[: nb[0]].copy(), st.as_dict()


def imin_greedy_batch(problems, mode: int = IMIN_AG, launch=None):
    """AdvancedGreedy or GreedyReplace on many problems at once. ``problems``: sequence of
    (handle, seeds, b, theta, seed); ``launch``: None or a dict of imin_launch fields.
    Returns a list of (blockers, stats dict)."""
    k = len(problems)
    arr = (imin_instance * max(k, 1))()
    keep = []
    outs = []
    for i, (handle, seeds, b, theta, seed) in enumerate(problems):
        S = np.ascontiguousarray(seeds, dtype=np.int32)
        out = np.zeros(max(int(b), 1), dtype=np.int32)
        nb = np.zeros(1, dtype=np.int32)
        st = imin_stats()
        keep += [S, out, nb, st]
        outs.append((out, nb, st))
        arr[i].g = ctypes.c_void_p(handle)
        arr[i].S = _p(S)
        arr[i].nS = S.shape[0]
        arr[i].b = int(b)
        arr[i].theta = int(theta)
        arr[i].seed = int(seed) & (2**64 - 1)
        arr[i].blockers = _p(out)
        arr[i].n_blockers = _p(nb)
        arr[i].stats = ctypes.pointer(st)
    rc = load().imin_greedy_batch(arr, k, int(mode), _launch(launch))
    if rc != IMIN_OK:
        raise IminError("imin_greedy_batch", rc)
    return [(out[: nb[0]].copy(), st.as_dict()) for out, nb, st in outs]


class Graph:
    """A device-resident graph (one ``imin_graph`` handle)."""

    def __init__(self, row_ptr, col, prob, model: int = IMIN_IC):
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.n = int(row_ptr.shape[0] - 1)
        self.model = int(model)
        self.handle = imin_graph_create(self.n, row_ptr, col, prob, model)

    def decrease(self, seeds, blocked=None, theta: int = 1000, seed: int = 0):
        return imin_decrease(self.handle, self.n, seeds, blocked, theta, seed)

    def spread(self, seeds, blocked=None, theta: int = 100000, seed: int = 0):
        return imin_spread(self.handle, self.n, seeds, blocked, theta, seed)

    def greedy(self, seeds, b: int, theta: int, seed: int = 0, mode: int = IMIN_AG):
        return imin_greedy(self.handle, seeds, b, theta, seed, mode)

    def set_launch(self, slots: int = 0, extra_cap: int = 0) -> None:
        imin_set_launch(self.handle, slots, extra_cap)

    def set_small(self, enable: int = -1, launch=None) -> None:
        imin_set_small(self.handle, enable, launch)

    def close(self) -> None:
        if self.handle:
            imin_graph_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A query server on a resident graph (``imin_server_*``): submit (S, b, theta, seed)
    AdvancedGreedy queries, drive it with ``step``, collect finished ones."""

    def __init__(self, graph: Graph, hbm_budget: int = 0, max_active: int = 0,
                 max_theta: int = 0, launch=None):
        cfg = imin_server_config()
        cfg.hbm_budget = int(hbm_budget)
        cfg.max_active = int(max_active)
        cfg.max_theta = int(max_theta)
        if launch:
            for k, v in launch.items():
                setattr(cfg.launch, k, int(v))
        h = ctypes.c_void_p()
        rc = load().imin_server_create(ctypes.c_void_p(graph.handle), ctypes.byref(cfg),
                                       ctypes.byref(h))
        if rc != IMIN_OK:
            raise IminError("imin_server_create", rc)
        self.handle = h.value
        self.graph = graph  # the graph must outlive the server

    def query_bytes(self, n_seeds: int, b: int) -> int:
        out = ctypes.c_uint64()
        rc = load().imin_server_query_bytes(ctypes.c_void_p(self.handle), int(n_seeds), int(b),
                                            ctypes.byref(out))
        if rc != IMIN_OK:
            raise IminError("imin_server_query_bytes", rc)
        return out.value

    def submit(self, seeds, b: int, theta: int, seed: int = 0, mode: int = IMIN_AG) -> int:
        S = np.ascontiguousarray(seeds, dtype=np.int32)
        t = ctypes.c_uint64()
        rc = load().imin_server_submit_mode(ctypes.c_void_p(self.handle), _p(S), S.shape[0],
                                            int(b), int(theta), int(seed) & (2**64 - 1),
                                            int(mode), ctypes.byref(t))
        if rc != IMIN_OK:
            raise IminError("imin_server_submit_mode", rc)
        return t.value

    def step(self):
        """One scheduling step; returns (active, queued) after it."""
        a, q = ctypes.c_int32(), ctypes.c_int32()
        rc = load().imin_server_step(ctypes.c_void_p(self.handle), ctypes.byref(a),
                                     ctypes.byref(q))
        if rc != IMIN_OK:
            raise IminError("imin_server_step", rc)
        return a.value, q.value

    def completed(self, cap: int = 4096):
        out = np.zeros(cap, dtype=np.uint64)
        k = ctypes.c_int32()
        rc = load().imin_server_completed(ctypes.c_void_p(self.handle), _p(out), int(cap),
                                          ctypes.byref(k))
        if rc != IMIN_OK:
            raise IminError("imin_server_completed", rc)
        return [int(x) for x in out[: k.value]]

    def result(self, ticket: int, cap: int):
        """(blockers, stats dict) of a finished query, or None while it is pending."""
        out = np.zeros(max(int(cap), 1), dtype=np.int32)
        nb = ctypes.c_int32()
        st = imin_stats()
        rc = load().imin_server_result(ctypes.c_void_p(self.handle), int(ticket), _p(out),
                                       int(cap), ctypes.byref(nb), ctypes.byref(st))
        if rc == 1:
            return None
        if rc != IMIN_OK:
            raise IminError("imin_server_result", rc)
        return out[: nb.value].copy(), st.as_dict()

    def close(self) -> None:
        if self.handle:
            load().imin_server_destroy(ctypes.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
