"""Python binding of libpbh.so: the parallel bucket heap (parBucketHeap) and
parDijkstra for MI355X (gfx950).

Argument marshalling only: every step runs in the HIP kernels of the library.
Arrays are torch tensors on the GPU (uint64 data as int64/uint64 tensors,
uint32 data as int32/uint32 tensors); the C entry points of include/pbh.h
receive their device pointers.  There is no CPU fallback: if the library is
not built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbh.so")

PBH_OK, PBH_EINVAL, PBH_ECAPACITY, PBH_ENOMEM, PBH_EDEVICE, PBH_ETIMEOUT, PBH_EINTERNAL = 0, -1, -2, -3, -4, -5, -6


class PBHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


MLP_PARAMS = 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1
MLP_BLOB = MLP_PARAMS + 2 * 8 + 1
K_PLAIN, K_FIXED, K_LEARNED, K_SEQ = 0, 1, 2, 3


class PbhOpts(C.Structure):
    _fields_ = [("engine", C.c_uint32), ("schedule", C.c_uint32), ("reserved", C.c_uint32 * 6)]


ENGINE_AUTO, ENGINE_TEAM, ENGINE_WIDE = 0, 1, 2


class SsspOpts(C.Structure):
    _fields_ = [("d", C.c_uint32), ("team", C.c_uint32), ("schedule", C.c_uint32),
                ("lds_levels", C.c_uint32), ("heap_capacity", C.c_uint64),
                ("k_rule", C.c_uint32), ("k_fixed", C.c_uint32), ("k_max", C.c_uint32), ("k_seq_len", C.c_uint32),
                ("k_seq", C.c_void_p), ("k_model", C.c_void_p),
                ("trace_features", C.c_void_p), ("trace_keys", C.c_void_p), ("trace_ids", C.c_void_p),
                ("trace_count", C.c_void_p), ("trace_query", C.c_void_p), ("trace_every", C.c_uint32),
                ("trace_cap", C.c_uint32), ("stop_key", C.c_uint64), ("max_rounds", C.c_uint32),
                ("d_scale", C.c_uint32), ("k_scale", C.c_float), ("k_every", C.c_uint32),
                ("settle_order", C.c_void_p), ("settle_cap", C.c_uint64), ("profile", C.c_uint32),
                ("deep_level", C.c_uint32)]


class SsspStats(C.Structure):
    _fields_ = [("rounds", C.c_uint64), ("relaxations", C.c_uint64), ("updates", C.c_uint64),
                ("heap_elems", C.c_uint64), ("extracted", C.c_uint64), ("resolves", C.c_uint64 * 16),
                ("levels", C.c_uint32), ("d", C.c_uint32), ("team", C.c_uint32), ("lds_levels", C.c_uint32),
                ("kernel_ms", C.c_double), ("last_key", C.c_uint64), ("level_us", C.c_double * 16),
                ("phase_us", C.c_double * 8)]


class NearFarStats(C.Structure):
    _fields_ = [("relaxations", C.c_uint64), ("phases", C.c_uint32), ("splits", C.c_uint32),
                ("delta", C.c_uint64), ("workgroups", C.c_uint32), ("reserved", C.c_uint32),
                ("kernel_ms", C.c_double)]


class SsspQuery(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("targets", C.c_void_p), ("weights", C.c_void_p), ("m", C.c_uint64),
                ("n", C.c_uint32), ("source", C.c_uint32), ("dist_out", C.c_void_p)]


_lib = None
EXPORTS = ["pbh_create", "pbh_create_ex", "pbh_bulk_update", "pbh_delete", "pbh_extract_min", "pbh_size", "pbh_traffic", "pbh_merge_profile", "pbh_kernel_profile", "pbh_set_profiling", "pbh_destroy",
           "pbh_debug_levels", "sssp", "sssp_ex", "sssp_noalloc", "sssp_batch", "sssp_autotune", "sssp_batch_autotune", "mlp_trace_labels", "mlp_feature_stats",
           "mlp_grad", "mlp_train", "mlp_infer", "sssp_nearfar", "pbh_last_error"]


def lib():
    """Loads libpbh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1908_09378_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        L.pbh_create.argtypes = [C.POINTER(vp), u32, u32]
        L.pbh_create_ex.argtypes = [C.POINTER(vp), u32, u32, C.POINTER(PbhOpts)]
        L.pbh_bulk_update.argtypes = [vp, vp, vp, u64]
        L.pbh_delete.argtypes = [vp, vp, u64]
        L.pbh_extract_min.argtypes = [vp, u64, vp, vp, C.POINTER(u64)]
        L.pbh_size.argtypes = [vp, C.POINTER(u64)]
        L.pbh_traffic.argtypes = [vp, C.POINTER(u64)]
        L.pbh_merge_profile.argtypes = [vp, C.POINTER(u64), C.POINTER(u64), C.POINTER(C.c_double)]
        L.pbh_set_profiling.argtypes = [vp, C.c_int]
        L.pbh_kernel_profile.argtypes = [vp, u32, C.POINTER(u64), C.POINTER(u64), C.POINTER(C.c_double)]
        L.pbh_kernel_name.argtypes = [u32]
        L.pbh_kernel_name.restype = C.c_char_p
        L.pbh_destroy.argtypes = [vp]
        L.pbh_debug_levels.argtypes = [vp, u32, C.POINTER(u32), C.POINTER(C.c_int32), vp, vp, vp, vp, vp]
        L.sssp.argtypes = [vp, vp, vp, u32, u64, u32, vp]
        L.sssp_ex.argtypes = [vp, vp, vp, u32, u64, u32, vp, C.POINTER(SsspOpts), C.POINTER(SsspStats), vp]
        L.sssp_noalloc.argtypes = [vp, vp, vp, u32, u64, u32, vp, C.POINTER(SsspOpts), C.POINTER(SsspStats), vp]
        L.sssp_batch.argtypes = [C.POINTER(SsspQuery), u32, C.POINTER(SsspOpts), C.POINTER(SsspStats), vp]
        L.sssp_autotune.argtypes = [vp, vp, vp, u32, u64, u32, vp, C.POINTER(SsspOpts), vp]
        L.sssp_batch_autotune.argtypes = [C.POINTER(SsspQuery), u32, C.POINTER(SsspOpts), vp]
        L.mlp_trace_labels.argtypes = [vp, vp, vp, u32, vp, vp, u32, vp]
        L.mlp_feature_stats.argtypes = [vp, u32, vp]
        L.mlp_grad.argtypes = [vp, vp, u32, vp, vp, vp]
        L.mlp_train.argtypes = [vp, vp, u32, vp, u32, u32, C.c_float, C.POINTER(C.c_float)]
        L.mlp_infer.argtypes = [vp, u32, vp, u32, vp]
        L.sssp_nearfar.argtypes = [vp, vp, vp, u32, u64, u32, vp, u64, C.POINTER(NearFarStats), vp]
        L.sssp_nearfar_last_error.restype = C.c_char_p
        L.pbh_last_error.restype = C.c_char_p
        for f in EXPORTS[:-1]:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PBH_OK:
        raise PBHError(rc, lib().pbh_last_error().decode())


def _ptr(t, elem_bytes):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("arrays must be GPU tensors")
    if not t.is_contiguous():
        raise ValueError("arrays must be contiguous")
    if t.element_size() != elem_bytes:
        raise ValueError(f"expected {elem_bytes}-byte elements, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _stats_dict(s):
    return dict(rounds=s.rounds, relaxations=s.relaxations, updates=s.updates, heap_elems=s.heap_elems,
                extracted=s.extracted, resolves=list(s.resolves), levels=s.levels, d=s.d, team=s.team,
                lds_levels=s.lds_levels, kernel_ms=s.kernel_ms, last_key=s.last_key, level_us=list(s.level_us),
                phase_us=dict(zip(PHASES, s.phase_us)))


# sssp_stats.phase_us slots (see include/pbh.h)
PHASES = ("drive", "piece", "propose", "extract", "relax", "intake", "other", "wait")


def sssp(offsets, targets, weights, n: int, m: int, source: int, dist_out) -> None:
    """parDijkstra: dist_out[v] = shortest distance from source (UINT64_MAX if
    unreachable); see include/pbh.h."""
    _check(lib().sssp(_ptr(offsets, 8), _ptr(targets, 4), _ptr(weights, 4), n, m, source, _ptr(dist_out, 8)))


def _opts(d=0, team=0, schedule=0, lds_levels=0, heap_capacity=0, k_rule=0, k_fixed=0, k_max=0, k_seq=None,
          k_model=None, trace=None, stop_key=0, max_rounds=0, d_scale=0, k_scale=0.0, settle_order=None, k_every=0,
          profile=0, deep_level=0):
    o = SsspOpts()
    o.profile = profile
    o.deep_level = deep_level
    o.k_every = k_every
    if settle_order is not None:
        o.settle_order, o.settle_cap = _ptr(settle_order, 4), settle_order.numel()
    o.k_scale = k_scale
    o.d, o.team, o.schedule, o.lds_levels, o.heap_capacity = d, team, schedule, lds_levels, heap_capacity
    o.k_rule, o.k_fixed, o.k_max = k_rule, k_fixed, k_max
    o.stop_key, o.max_rounds, o.d_scale = stop_key, max_rounds, d_scale
    if k_seq is not None:
        o.k_seq, o.k_seq_len = _ptr(k_seq, 4), k_seq.numel()
    if k_model is not None:
        if k_model.numel() != MLP_BLOB or k_model.element_size() != 4:
            raise ValueError(f"k_model must hold {MLP_BLOB} float32 values")
        o.k_model = _ptr(k_model, 4)
    if trace is not None:
        f, k, v, cnt, q, every = trace
        o.trace_features, o.trace_keys, o.trace_ids, o.trace_count = _ptr(f, 4), _ptr(k, 8), _ptr(v, 4), _ptr(cnt, 4)
        o.trace_query = _ptr(q, 4) if q is not None else None
        o.trace_every, o.trace_cap = every, f.numel() // 8
    return o


def sssp_ex(offsets, targets, weights, n: int, m: int, source: int, dist_out, *, stream=None, **kw) -> dict:
    """sssp with options (see sssp_opts in include/pbh.h): d, team, schedule,
    lds_levels, heap_capacity, k_rule, k_fixed, k_max, k_seq (int32 tensor),
    k_model (float32 tensor of MLP_BLOB values), trace=(features, keys, ids,
    count, every)."""
    o = _opts(**kw)
    s = SsspStats()
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(lib().sssp_ex(_ptr(offsets, 8), _ptr(targets, 4), _ptr(weights, 4), n, m, source, _ptr(dist_out, 8),
                         C.byref(o), C.byref(s), sp))
    return _stats_dict(s)


def sssp_noalloc(offsets, targets, weights, n: int, m: int, source: int, dist_out, *, stream=None, **kw) -> dict:
    """sssp_ex without device allocation: every buffer comes from the
    library's fixed scratch (sssp_noalloc in include/pbh.h)."""
    o = _opts(**kw)
    s = SsspStats()
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(lib().sssp_noalloc(_ptr(offsets, 8), _ptr(targets, 4), _ptr(weights, 4), n, m, source,
                              _ptr(dist_out, 8), C.byref(o), C.byref(s), sp))
    return _stats_dict(s)


def sssp_nearfar(offsets, targets, weights, n: int, m: int, source: int, dist_out, delta: int = 0, *,
                 stream=None) -> dict:
    """Near-Far (Delta-stepping) baseline: dist_out = shortest distances from
    source; delta = 0 picks mean weight x 64 / mean degree (sssp_nearfar in
    include/pbh.h)."""
    s = NearFarStats()
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = lib().sssp_nearfar(_ptr(offsets, 8), _ptr(targets, 4), _ptr(weights, 4), n, m, source,
                            _ptr(dist_out, 8), delta, C.byref(s), sp)
    if rc != PBH_OK:
        raise PBHError(rc, lib().sssp_nearfar_last_error().decode())
    return dict(relaxations=s.relaxations, phases=s.phases, splits=s.splits, delta=s.delta,
                workgroups=s.workgroups, kernel_ms=s.kernel_ms)


def _tuned(o) -> dict:
    return dict(d=o.d, d_scale=o.d_scale, k_max=o.k_max, team=o.team, k_scale=o.k_scale, k_every=o.k_every)


def sssp_autotune(offsets, targets, weights, n: int, m: int, source: int, dist_out, *, stream=None, **kw) -> dict:
    """Picks d and k_max for this query by timed trials on it (sssp_autotune
    in include/pbh.h); returns {d, d_scale, k_max} to pass to sssp_ex along
    with the other options.  dist_out is scratch."""
    o = _opts(**kw)
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(lib().sssp_autotune(_ptr(offsets, 8), _ptr(targets, 4), _ptr(weights, 4), n, m, source,
                               _ptr(dist_out, 8), C.byref(o), sp))
    return _tuned(o)


def _queries(queries):
    arr = (SsspQuery * max(1, len(queries)))()
    for i, (off, tg, wt, n, m, src, dist) in enumerate(queries):
        arr[i] = SsspQuery(_ptr(off, 8), _ptr(tg, 4) if m else None, _ptr(wt, 4) if m else None, m, n, src,
                           _ptr(dist, 8))
    return arr


def sssp_batch_autotune(queries, *, stream=None, **kw) -> dict:
    """Picks d_scale and k_max for a batch (sssp_batch_autotune in
    include/pbh.h); returns {d, d_scale, k_max} for sssp_batch."""
    arr = _queries(queries)
    o = _opts(**kw)
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(lib().sssp_batch_autotune(arr, len(queries), C.byref(o), sp))
    return _tuned(o)


def sssp_batch(queries, *, stream=None, **kw) -> dict:
    """Many independent parDijkstra queries in one launch.  queries: sequence
    of (offsets, targets, weights, n, m, source, dist_out)."""
    arr = _queries(queries)
    o = _opts(**kw)
    s = SsspStats()
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(lib().sssp_batch(arr, len(queries), C.byref(o), C.byref(s), sp))
    return _stats_dict(s)


class Heap:
    """A parallel bucket heap over ids [0, id_capacity) with bulk size d."""

    def __init__(self, id_capacity: int, d: int, engine: int = ENGINE_AUTO, schedule: int = 0):
        """engine: ENGINE_AUTO, ENGINE_TEAM (one workgroup per operation) or
        ENGINE_WIDE (device-wide steps); schedule 0 = Theorem 1, 1 = on demand."""
        h = C.c_void_p()
        o = PbhOpts(engine, schedule)
        _check(lib().pbh_create_ex(C.byref(h), id_capacity, d, C.byref(o)))
        self._h = h
        self.id_capacity = id_capacity
        self.d = d

    def close(self):
        if getattr(self, "_h", None):
            lib().pbh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bulk_update(self, keys, ids) -> None:
        count = keys.numel()
        if ids.numel() != count:
            raise ValueError("keys and ids differ in length")
        _check(lib().pbh_bulk_update(self._h, _ptr(keys, 8) if count else None,
                                     _ptr(ids, 4) if count else None, count))

    def delete(self, ids) -> None:
        """Delete (Section 1.2) of every id in `ids` (uint32 data, device);
        absent ids are no-ops."""
        count = ids.numel()
        _check(lib().pbh_delete(self._h, _ptr(ids, 4) if count else None, count))

    def extract_min(self, k: int, keys_out, ids_out) -> int:
        if k and (keys_out.numel() < k or ids_out.numel() < k):
            raise ValueError("output arrays shorter than k")
        n = C.c_uint64(0)
        _check(lib().pbh_extract_min(self._h, k, _ptr(keys_out, 8) if k else None,
                                     _ptr(ids_out, 4) if k else None, C.byref(n)))
        return n.value

    def size(self) -> int:
        n = C.c_uint64(0)
        _check(lib().pbh_size(self._h, C.byref(n)))
        return n.value

    def merge_profile(self) -> dict:
        """Device-wide engine: launches, algorithmic bytes and HIP-event ms of
        the merge writing passes so far."""
        a, b, t = C.c_uint64(0), C.c_uint64(0), C.c_double(0)
        _check(lib().pbh_merge_profile(self._h, C.byref(a), C.byref(b), C.byref(t)))
        return dict(launches=a.value, bytes=b.value, ms=t.value)

    def kernel_profile(self) -> dict:
        """Device-wide engine: {kernel name: {launches, bytes, ms}} over the
        launches timed so far (pbh_kernel_profile)."""
        out = {}
        kind = 0
        while True:
            name = lib().pbh_kernel_name(kind)
            if name is None:
                break
            a, b, t = C.c_uint64(0), C.c_uint64(0), C.c_double(0)
            _check(lib().pbh_kernel_profile(self._h, kind, C.byref(a), C.byref(b), C.byref(t)))
            out[name.decode()] = dict(launches=a.value, bytes=b.value, ms=t.value)
            kind += 1
        return out

    def set_profiling(self, on: bool) -> None:
        """Device-wide engine: time each merge writing pass with HIP events."""
        _check(lib().pbh_set_profiling(self._h, 1 if on else 0))

    def traffic(self) -> int:
        """Heap elements read or written by the level operations so far."""
        n = C.c_uint64(0)
        _check(lib().pbh_traffic(self._h, C.byref(n)))
        return n.value

    def debug_levels(self) -> dict:
        import numpy as np
        cap = 16
        q = C.c_uint32(0)
        ell = C.c_int32(0)
        nB = np.zeros(cap, np.uint32)
        nS = np.zeros(cap, np.uint32)
        pk = np.zeros(cap, np.uint64)
        pv = np.zeros(cap, np.uint32)
        rs = np.zeros(cap, np.uint64)
        _check(lib().pbh_debug_levels(self._h, cap, C.byref(q), C.byref(ell), nB.ctypes.data, nS.ctypes.data,
                                      pk.ctypes.data, pv.ctypes.data, rs.ctypes.data))
        k = q.value
        return dict(q=k, ell=ell.value, nB=nB[:k], nS=nS[:k], pk=pk[:k], pv=pv[:k], resolves=rs[:k])


# ---------------------------------------------------------------- learned k
def mlp_trace_labels(trace_keys, trace_ids, trace_query, count: int, dists, labels) -> None:
    """labels[r] = log2(zero-waste pull size) of trace record r; dists: a
    sequence of per-query distance tensors (device)."""
    import torch
    ptrs = torch.tensor([d.data_ptr() for d in dists], dtype=torch.int64, device=labels.device)
    lens = torch.tensor([d.numel() for d in dists], dtype=torch.int32, device=labels.device)
    _check(lib().mlp_trace_labels(_ptr(trace_keys, 8), _ptr(trace_ids, 4), _ptr(trace_query, 4), count,
                                  _ptr(ptrs, 8), _ptr(lens, 4), len(dists), _ptr(labels, 4)))


def mlp_feature_stats(X, blob) -> None:
    _check(lib().mlp_feature_stats(_ptr(X, 4), X.shape[0], _ptr(blob, 4)))


def mlp_infer(X, blob, y, team: int = 256) -> None:
    """The round loop's inference on rows of X (n x 8 float32, device):
    y[r] = scale * network output (k = 2^y before clamping)."""
    _check(lib().mlp_infer(_ptr(X, 4), X.shape[0], _ptr(blob, 4), team, _ptr(y, 4)))


def mlp_grad(X, Y, blob, grad, loss) -> None:
    _check(lib().mlp_grad(_ptr(X, 4), _ptr(Y, 4), X.shape[0], _ptr(blob, 4), _ptr(grad, 4), _ptr(loss, 4)))


def mlp_train(X, Y, blob, batch: int, steps: int, lr: float):
    import numpy as np
    lt = np.zeros(max(1, steps), np.float32)
    _check(lib().mlp_train(_ptr(X, 4), _ptr(Y, 4), X.shape[0], _ptr(blob, 4), batch, steps, lr,
                           lt.ctypes.data_as(C.POINTER(C.c_float))))
    return lt[:steps]
