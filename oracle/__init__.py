"""Oracle for the parallel bucket heap and parDijkstra (CPU, plain, slow).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the GPU library.  It shares no code
with the HIP path (the seeded generators in ``workloads`` are the only common
module, and they hold none of the method's arithmetic).

* ``PQ``            -- the priority-queue ADT of Section 1.2 (update /
                       bulk update / delete / batched extractMin) as a sorted
                       multiset (``oracle.cpp``).
* ``PQArrays``      -- the same ADT written with numpy arrays (``cur[id]`` plus
                       "the k smallest live (key, id)"), for heap sizes where a
                       std::set per element is too slow.  Pinned against ``PQ``.
* ``dijkstra``      -- binary-heap Dijkstra (Section 1.1), settle order too.
* ``bellman_ford``  -- brute-force Bellman-Ford (Section 1.1) for tiny graphs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(force: bool = False) -> str:
    """Compile oracle.cpp with g++ into liboracle.so (in-tree)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        u64p, u32p = C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)
        L.opq_create.restype = C.c_void_p
        L.opq_create.argtypes = [C.c_uint32]
        L.opq_destroy.argtypes = [C.c_void_p]
        L.opq_bulk_update.restype = C.c_int64
        L.opq_bulk_update.argtypes = [C.c_void_p, u64p, u32p, C.c_uint64]
        L.opq_delete.restype = C.c_int64
        L.opq_delete.argtypes = [C.c_void_p, u32p, C.c_uint64]
        L.opq_extract_min.restype = C.c_uint64
        L.opq_extract_min.argtypes = [C.c_void_p, C.c_uint64, u64p, u32p]
        L.opq_size.restype = C.c_uint64
        L.opq_size.argtypes = [C.c_void_p]
        L.opq_cur.argtypes = [C.c_void_p, u64p]
        L.odijkstra.restype = C.c_int
        L.odijkstra.argtypes = [u64p, u32p, u32p, C.c_uint32, C.c_uint64, C.c_uint32, u64p, u32p,
                                u64p, u64p]
        L.obellman_ford.restype = C.c_int64
        L.obellman_ford.argtypes = [u64p, u32p, u32p, C.c_uint32, C.c_uint64, C.c_uint32, u64p]
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class PQ:
    """Sorted-multiset priority queue over (uint64 key, uint32 id)."""

    def __init__(self, id_capacity: int):
        self.id_capacity = id_capacity
        self._h = lib().opq_create(id_capacity)

    def close(self):
        if self._h:
            lib().opq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bulk_update(self, keys, ids) -> int:
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        assert keys.shape == ids.shape
        r = lib().opq_bulk_update(self._h, _p(keys, C.c_uint64), _p(ids, C.c_uint32), keys.shape[0])
        if r < 0:
            raise ValueError("invalid update (id out of range or key == UINT64_MAX)")
        return int(r)

    def delete(self, ids) -> int:
        """Delete(e) of Section 1.2 for every listed id (absent ids: no-op);
        returns how many elements left the queue."""
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        r = lib().opq_delete(self._h, _p(ids, C.c_uint32), ids.shape[0])
        if r < 0:
            raise ValueError("invalid delete (id out of range)")
        return int(r)

    def extract_min(self, k: int):
        k = int(k)
        cap = min(k, self.size())
        ko = np.empty(cap, np.uint64)
        io = np.empty(cap, np.uint32)
        n = lib().opq_extract_min(self._h, k, _p(ko, C.c_uint64), _p(io, C.c_uint32))
        return ko[:n], io[:n]

    def size(self) -> int:
        return int(lib().opq_size(self._h))

    def cur(self) -> np.ndarray:
        out = np.empty(self.id_capacity, np.uint64)
        lib().opq_cur(self._h, _p(out, C.c_uint64))
        return out


class PQArrays:
    """The same ADT as ``PQ`` on numpy arrays.

    State: ``cur[id]`` (INF = absent).  bulk_update: cur[id] = min(cur[id], key)
    over the batch (np.minimum.at).  extract_min(k): the min(k, size) smallest
    live (key, id) pairs in ascending order, then cur = INF for them.  (key, id)
    is packed as key * 2**id_bits + id when that fits in 64 bits, else sorted
    with lexsort."""

    def __init__(self, id_capacity: int):
        self.cur = np.full(id_capacity, INF, dtype=np.uint64)
        self.id_bits = max(1, int(id_capacity - 1).bit_length())

    def bulk_update(self, keys, ids):
        keys = np.asarray(keys, dtype=np.uint64)
        ids = np.asarray(ids, dtype=np.int64)
        if keys.size and (ids.max() >= self.cur.shape[0] or (keys == INF).any()):
            raise ValueError("invalid update")
        np.minimum.at(self.cur, ids, keys)

    def size(self) -> int:
        return int(np.count_nonzero(self.cur != INF))

    def delete(self, ids) -> int:
        """cur[id] = INF for every listed id; returns how many were live."""
        ids = np.asarray(ids, dtype=np.int64)
        if ids.size and ids.max() >= self.cur.shape[0]:
            raise ValueError("invalid delete")
        u = np.unique(ids)
        n = int(np.count_nonzero(self.cur[u] != INF))
        self.cur[u] = INF
        return n

    def extract_min(self, k: int):
        live = np.nonzero(self.cur != INF)[0]
        keys = self.cur[live]
        k = min(int(k), live.shape[0])
        if k == 0:
            return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
        if keys.size and int(keys.max()) < (1 << (64 - self.id_bits)):
            packed = (keys << np.uint64(self.id_bits)) | live.astype(np.uint64)
            sel = np.argpartition(packed, k - 1)[:k] if k < packed.shape[0] else np.arange(packed.shape[0])
            sel = sel[np.argsort(packed[sel], kind="stable")]
        else:
            sel = np.lexsort((live, keys))[:k]
        ids = live[sel]
        out_k = self.cur[ids].copy()
        self.cur[ids] = INF
        return out_k, ids.astype(np.uint32)


def dijkstra(g, src: int, want_order: bool = False):
    """Distances from ``src`` (uint64, INF = unreachable); optionally the settle
    order and the number of edges scanned."""
    off = np.ascontiguousarray(g.offsets, dtype=np.uint64)
    tg = np.ascontiguousarray(g.targets, dtype=np.uint32)
    w = np.ascontiguousarray(g.weights, dtype=np.uint32)
    dist = np.empty(g.n, np.uint64)
    order = np.empty(g.n, np.uint32) if want_order else None
    ns = C.c_uint64(0)
    nr = C.c_uint64(0)
    r = lib().odijkstra(_p(off, C.c_uint64), _p(tg, C.c_uint32), _p(w, C.c_uint32), g.n, g.m, src,
                        _p(dist, C.c_uint64), _p(order, C.c_uint32) if want_order else None,
                        C.byref(ns), C.byref(nr))
    if r != 0:
        raise ValueError("invalid graph or source")
    if want_order:
        return dist, order[: ns.value], int(nr.value)
    return dist


def bellman_ford(g, src: int):
    off = np.ascontiguousarray(g.offsets, dtype=np.uint64)
    tg = np.ascontiguousarray(g.targets, dtype=np.uint32)
    w = np.ascontiguousarray(g.weights, dtype=np.uint32)
    dist = np.empty(g.n, np.uint64)
    r = lib().obellman_ford(_p(off, C.c_uint64), _p(tg, C.c_uint32), _p(w, C.c_uint32), g.n, g.m, src,
                            _p(dist, C.c_uint64))
    if r < 0:
        raise ValueError("invalid graph or source")
    return dist


def time_dijkstra(g, src: int, budget_s: float = 20.0):
    """Wall time of single-thread oracle Dijkstra on ``g``; repeats the whole run
    until ~budget_s of CPU work (at least once).  Returns (seconds per run, runs)."""
    runs = 0
    t0 = time.perf_counter()
    while True:
        dijkstra(g, src)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / runs * (runs + 1) > budget_s * 1.5:
            break
    return el / runs, runs
