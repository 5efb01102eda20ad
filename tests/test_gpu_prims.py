"""GPU unit tests of the team primitives (scan, min/max, Merge+DeleteDuplicates,
three-way split, Select, (key, id) sort) for teams of 64, 256 and 1024
threads, against numpy, on sizes that span several tiles and ragged tails."""
import ctypes as C

import numpy as np
import pytest
import torch

import devprims
from gpu_util import DEV, dev32, dev64, host32, host64

pytestmark = pytest.mark.gpu
INF = np.uint64(0xFFFFFFFFFFFFFFFF)
TEAMS = [64, 256, 1024]
SIZES = [0, 1, 2, 7, 63, 64, 65, 300, 513, 4096 + 3]


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def run(nt, op, a=None, b=None, nc=0, cur=None, res=None):
    ak, av = (dev64(a[0]), dev32(a[1])) if a is not None else (None, None)
    bk, bv = (dev64(b[0]), dev32(b[1])) if b is not None else (None, None)
    na = 0 if a is None else len(a[1])
    nb = 0 if b is None else len(b[1])
    outs = [torch.zeros(max(nc, 1), dtype=torch.int64, device=DEV) for _ in range(3)]
    outv = [torch.zeros(max(nc, 1), dtype=torch.int32, device=DEV) for _ in range(3)]
    r = dev64(np.zeros(8, np.uint64) if res is None else res)
    curd = dev64(cur) if cur is not None else None
    rc = devprims.lib().dp_run(nt, op, _p(ak), _p(av), na, _p(bk), _p(bv), nb, _p(outs[0]), _p(outv[0]),
                               _p(outs[1]), _p(outv[1]), _p(outs[2]), _p(outv[2]), _p(curd), _p(r))
    assert rc == 0
    return ([host64(o) for o in outs], [host32(o) for o in outv], host64(r), ak, av, bk, bv)


def sorted_ids(rng, n, cap):
    return np.sort(rng.choice(cap, size=n, replace=False)).astype(np.uint32)


@pytest.mark.parametrize("nt", TEAMS)
@pytest.mark.parametrize("n", SIZES + [5000])
def test_scan(nt, n):
    rng = np.random.default_rng(n)
    v = rng.integers(0, 9, size=n).astype(np.uint32)
    (ck, cv, r, *_) = run(nt, 0, a=(np.zeros(n, np.uint64), v), nc=n)
    ex = np.concatenate([[0], np.cumsum(v)[:-1]]).astype(np.uint32) if n else np.zeros(0, np.uint32)
    assert np.array_equal(cv[0][:n], ex) and r[0] == v.sum()


@pytest.mark.parametrize("nt", TEAMS)
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1000, 5000])
def test_min_max(nt, n):
    rng = np.random.default_rng(n + nt)
    k = rng.integers(0, 50, size=n).astype(np.uint64) << np.uint64(30)
    v = rng.integers(0, 1 << 31, size=n).astype(np.uint32)
    (_, _, r, *_) = run(nt, 1, a=(k, v))
    i = np.lexsort((v, k))[0]
    assert (r[0], r[1]) == (k[i], v[i]) and r[2] == k.min() and r[3] == k.max()


@pytest.mark.parametrize("nt", TEAMS)
@pytest.mark.parametrize("na,nb", [(0, 0), (2, 0), (0, 3), (5, 7), (64, 64), (300, 17), (1000, 3000), (513, 4100)])
@pytest.mark.parametrize("mode", ["min", "live"])
def test_merge_dedup(nt, na, nb, mode):
    rng = np.random.default_rng(na * 7 + nb)
    cap = 3 * (na + nb) + 10
    ia, ib = sorted_ids(rng, na, cap), sorted_ids(rng, nb, cap)
    ka = rng.integers(0, 100, size=na).astype(np.uint64)
    kb = rng.integers(0, 100, size=nb).astype(np.uint64)
    cur = None
    if mode == "live":
        cur = rng.integers(0, 100, size=cap).astype(np.uint64)
        # make some elements live
        cur[ia[::2]] = ka[::2]
        cur[ib[::3]] = kb[::3]
    (ck, cv, r, *_) = run(nt, 2, a=(ka, ia), b=(kb, ib), nc=na + nb, cur=cur)
    m = int(r[0])
    # expected
    d = {}
    for k, i in zip(kb.tolist(), ib.tolist()):
        d.setdefault(i, []).append(("B", k))
    for k, i in zip(ka.tolist(), ia.tolist()):
        d.setdefault(i, []).insert(0, ("A", k))
    exp = []
    for i in sorted(d):
        c = d[i]
        if cur is None:
            exp.append((min(k for _, k in c), i))
        else:
            live = [k for _, k in c if k == cur[i]]
            if len(c) == 2:
                if c[0][1] == c[1][1]:
                    exp.append((c[0][1], i))
                elif live:
                    exp.append((live[0], i))
            else:
                src, k = c[0]
                if src == "A" or k == cur[i]:   # filterB drops dead B-only elements
                    exp.append((k, i))
    got = list(zip(ck[0][:m].tolist(), cv[0][:m].tolist()))
    assert got == exp


@pytest.mark.parametrize("nt", TEAMS)
@pytest.mark.parametrize("n", SIZES)
def test_partition3(nt, n):
    rng = np.random.default_rng(n + 3)
    ids = sorted_ids(rng, n, 4 * n + 5)
    keys = rng.integers(0, 20, size=n).astype(np.uint64)
    p1, p2 = (np.uint64(6), np.uint32(ids[n // 3] if n else 0)), (np.uint64(13), np.uint32(2 ** 31))
    res = np.array([p1[0], p1[1], p2[0], p2[1], 0, 0, 0, 0], np.uint64)
    (ck, cv, r, *_) = run(nt, 3, a=(keys, ids), nc=n, res=res)
    e = list(zip(keys.tolist(), ids.tolist()))
    c0 = [x for x in e if x <= (int(p1[0]), int(p1[1]))]
    c1 = [x for x in e if (int(p1[0]), int(p1[1])) < x <= (int(p2[0]), int(p2[1]))]
    c2 = [x for x in e if x > (int(p2[0]), int(p2[1]))]
    assert (r[4], r[5], r[6]) == (len(c0), len(c1), len(c2))
    for j, c in enumerate((c0, c1, c2)):
        assert list(zip(ck[j][:len(c)].tolist(), cv[j][:len(c)].tolist())) == c


@pytest.mark.parametrize("nt", TEAMS)
@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 500, 3000])
@pytest.mark.parametrize("kr", [1, 2, 3, 0.5, -2, -1])
@pytest.mark.parametrize("keys", ["wide", "ties"])
def test_select(nt, n, kr, keys):
    rng = np.random.default_rng(n * 11)
    ids = sorted_ids(rng, n, 5 * n + 3)
    k = (rng.integers(0, 1 << 40, size=n) if keys == "wide" else rng.integers(0, 3, size=n)).astype(np.uint64)
    r = kr if isinstance(kr, int) and kr > 0 else (max(1, int(n * kr)) if kr > 0 else n + 1 + kr)
    r = min(max(r, 1), n)
    b = (np.zeros(0, np.uint64), np.zeros(r, np.uint32))  # nb carries r
    (_, _, res, *_) = run(nt, 4, a=(k, ids), b=b)
    order = np.lexsort((ids, k))
    assert (res[0], res[1]) == (k[order[r - 1]], ids[order[r - 1]])


@pytest.mark.parametrize("nt", TEAMS)
@pytest.mark.parametrize("n", [0, 1, 5, 64, 65, 700, 5000])
def test_sort_kv(nt, n):
    rng = np.random.default_rng(n + 99)
    ids = rng.choice(1 << 20, size=n, replace=False).astype(np.uint32)
    k = rng.integers(0, 1 << 33, size=n).astype(np.uint64)
    k[::3] = 77
    ak, av = dev64(k), dev32(ids)
    bk, bv = torch.zeros(max(n, 1), dtype=torch.int64, device=DEV), torch.zeros(max(n, 1), dtype=torch.int32, device=DEV)
    r = dev64(np.array([20, 0, 0, 0, 0, 0, 0, 0], np.uint64))
    rc = devprims.lib().dp_run(nt, 5, _p(ak), _p(av), n, _p(bk), _p(bv), n, None, None, None, None, None, None,
                               None, _p(r))
    assert rc == 0
    in_tmp = host64(r)[1]
    gk, gv = (host64(bk), host32(bv)) if in_tmp else (host64(ak), host32(av))
    o = np.lexsort((ids, k))
    assert np.array_equal(gk[:n], k[o]) and np.array_equal(gv[:n], ids[o])
