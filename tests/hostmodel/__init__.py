"""ctypes driver for tests/hostmodel/hostmodel.hip: the GPU kernels' heap and
parDijkstra logic instantiated with a one-thread team on the CPU (tests only)."""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hostmodel.hip")
_CORE = [os.path.join(_HERE, "..", "..", "paper_1908_09378_amd", "csrc", f) for f in ("pbh_core.h", "pbh_team.h")]
INF = np.uint64(0xFFFFFFFFFFFFFFFF)
_lib = {}


def build(sanitize: bool = False) -> str:
    out = os.path.join(_HERE, "libhostmodel_asan.so" if sanitize else "libhostmodel.so")
    newest = max(os.path.getmtime(p) for p in [_SRC] + _CORE)
    if not os.path.exists(out) or os.path.getmtime(out) < newest:
        cmd = ["hipcc", "-O2", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        if sanitize:
            cmd += ["-Xarch_host", "-fsanitize=address,undefined"]
        tmp = out + f".tmp{os.getpid()}"
        subprocess.check_call(cmd + [_SRC, "-o", tmp], stderr=subprocess.DEVNULL)
        os.replace(tmp, out)
    return out


def _asan_runtime_loaded() -> bool:
    with open("/proc/self/maps") as f:
        return "libclang_rt.asan" in f.read()


def lib():
    sanitize = os.environ.get("PBH_HOSTMODEL_ASAN") == "1"
    if sanitize and not _asan_runtime_loaded():
        raise RuntimeError("PBH_HOSTMODEL_ASAN=1 needs the ASan runtime loaded before Python starts: "
                           "run tests/hostmodel/asan.sh (it sets LD_PRELOAD)")
    if sanitize not in _lib:
        L = C.CDLL(build(sanitize))
        u64p, u32p = C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)
        L.hm_create.restype = C.c_void_p
        L.hm_create.argtypes = [C.c_uint32, C.c_uint32, C.c_int]
        L.hm_destroy.argtypes = [C.c_void_p]
        L.hm_update.restype = C.c_int
        L.hm_update.argtypes = [C.c_void_p, u64p, u32p, C.c_uint64]
        L.hm_delete.restype = C.c_int
        L.hm_delete.argtypes = [C.c_void_p, u32p, C.c_uint64]
        L.hm_extract.restype = C.c_int
        L.hm_extract.argtypes = [C.c_void_p, C.c_uint64, u64p, u32p, u64p]
        L.hm_levels.argtypes = [C.c_void_p, u32p, C.POINTER(C.c_int), u32p, u32p, u64p, u32p, u64p, u64p]
        L.hm_level_items.argtypes = [C.c_void_p, C.c_int, u64p, u32p, u64p, u32p]
        L.hm_resolve_log.restype = C.c_uint64
        L.hm_resolve_log.argtypes = [C.c_void_p, C.POINTER(C.c_longlong), C.c_uint64]
        L.hm_sssp.restype = C.c_int
        L.hm_sssp.argtypes = [u64p, u32p, u32p, C.c_uint32, C.c_uint64, C.c_uint32, u64p, C.c_uint32,
                              C.c_int, C.c_uint64, C.c_int, u64p, C.c_int, C.c_uint32, C.c_uint32, u32p,
                              C.c_uint32, C.POINTER(C.c_float), C.c_int, C.c_uint64, C.c_uint32, C.c_int,
                              C.c_int, C.c_uint64]
        _lib[sanitize] = L
    return _lib[sanitize]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class HostHeap:
    def __init__(self, id_cap, d, sched=0):
        self.h = lib().hm_create(id_cap, d, sched)

    def __del__(self):
        if getattr(self, "h", None):
            lib().hm_destroy(self.h)
            self.h = None

    def bulk_update(self, keys, ids):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        rc = lib().hm_update(self.h, _p(keys, C.c_uint64), _p(ids, C.c_uint32), keys.shape[0])
        if rc:
            raise RuntimeError(f"hm_update rc={rc}")

    def delete(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        rc = lib().hm_delete(self.h, _p(ids, C.c_uint32), ids.shape[0])
        if rc:
            raise RuntimeError(f"hm_delete rc={rc}")

    def extract_min(self, k):
        ko = np.zeros(max(k, 1), np.uint64)
        io = np.zeros(max(k, 1), np.uint32)
        n = C.c_uint64(0)
        rc = lib().hm_extract(self.h, k, _p(ko, C.c_uint64), _p(io, C.c_uint32), C.byref(n))
        if rc:
            raise RuntimeError(f"hm_extract rc={rc}")
        return ko[: n.value], io[: n.value]

    def levels(self):
        q = C.c_uint32(0)
        ell = C.c_int(0)
        live = C.c_uint64(0)
        nB = np.zeros(16, np.uint32)
        nS = np.zeros(16, np.uint32)
        pk = np.zeros(16, np.uint64)
        pv = np.zeros(16, np.uint32)
        cnt = np.zeros(16, np.uint64)
        lib().hm_levels(self.h, C.byref(q), C.byref(ell), _p(nB, C.c_uint32), _p(nS, C.c_uint32),
                        _p(pk, C.c_uint64), _p(pv, C.c_uint32), _p(cnt, C.c_uint64), C.byref(live))
        q = q.value
        return dict(q=q, ell=ell.value, nB=nB[:q], nS=nS[:q], pk=pk[:q], pv=pv[:q], cnt=cnt[:q],
                    live=live.value)

    def resolve_log(self):
        """Records of every Resolve(i) since the last call, before and after
        it: dicts with lvl, after, ell, q, nB, nS (level i), nB1, nS1 (level
        i+1), cnt (Resolve(i) executions so far)."""
        cap = 1 << 16
        buf = np.zeros(9 * cap, np.int64)
        n = lib().hm_resolve_log(self.h, buf.ctypes.data_as(C.POINTER(C.c_longlong)), cap)
        assert n <= cap
        keys = ("lvl", "after", "ell", "q", "nB", "nS", "nB1", "nS1", "cnt")
        return [dict(zip(keys, buf[9 * j:9 * j + 9].tolist())) for j in range(n)]

    def items(self, i, nB, nS):
        bk = np.zeros(max(nB, 1), np.uint64)
        bv = np.zeros(max(nB, 1), np.uint32)
        sk = np.zeros(max(nS, 1), np.uint64)
        sv = np.zeros(max(nS, 1), np.uint32)
        lib().hm_level_items(self.h, i, _p(bk, C.c_uint64), _p(bv, C.c_uint32), _p(sk, C.c_uint64),
                             _p(sv, C.c_uint32))
        return bk[:nB], bv[:nB], sk[:nS], sv[:nS]


def sssp(g, src, d=0, sched=0, hcap=0, qlds=0, rule=0, kfix=0, kmax=0, kseq=None, model=None, check_live=False,
         stop_key=0, max_rounds=0, deep_lim=0, deep_mode=1, deep_seed=0):
    """The kernel's round loop on the CPU.  deep_lim > 0: levels >= max(deep_lim,
    2, qlds) are resolved by simulated deep-level workers (deep_mode 0 eager,
    1 lazy, 2 seeded random)."""
    off = np.ascontiguousarray(g.offsets, np.uint64)
    tg = np.ascontiguousarray(g.targets, np.uint32)
    wt = np.ascontiguousarray(g.weights, np.uint32)
    dist = np.zeros(g.n, np.uint64)
    st = np.zeros(32, np.uint64)
    ks = None if kseq is None else np.ascontiguousarray(kseq, np.uint32)
    mdl = None if model is None else np.ascontiguousarray(model, np.float32)
    rc = lib().hm_sssp(_p(off, C.c_uint64), _p(tg, C.c_uint32), _p(wt, C.c_uint32), g.n, g.m, src,
                       _p(dist, C.c_uint64), d, sched, hcap, qlds, _p(st, C.c_uint64), rule, kfix, kmax,
                       None if ks is None else _p(ks, C.c_uint32), 0 if ks is None else ks.shape[0],
                       None if mdl is None else _p(mdl, C.c_float), int(check_live), stop_key, max_rounds,
                       deep_lim, deep_mode, deep_seed)
    return rc, dist, dict(rounds=int(st[0]), relax=int(st[1]), updates=int(st[2]), elems=int(st[3]),
                          levels=int(st[4]), resolves=st[5:21].tolist(), extracted=int(st[21]),
                          first_bad=int(st[22].astype(np.int64)), violation=st[23:26].tolist(),
                          last_key=int(st[26]), stopped=bool(st[27]), worker_runs=int(st[28]),
                          deep_lim=int(st[29]))
