"""Seeded synthetic inputs shared by the GPU path's tests/bench and by the oracle.

This module holds no arithmetic of the method itself (no heap, no shortest
paths).  It only turns a seed into arrays: CSR graphs and heap update batches.

Random numbers come from SplitMix64 used as a counter-based generator
(Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014): the i-th draw of a stream with seed s is
``mix(s + (i + 1) * 0x9E3779B97F4A7C15)`` with the published 64-bit finaliser
``mix``.  Being counter-based it vectorises in numpy and gives the same values
on every machine.

CSR layout used everywhere: ``offsets`` uint64[n+1], ``targets`` uint32[m],
``weights`` uint32[m]; the out-edges of vertex u are
``targets[offsets[u]:offsets[u+1]]``, sorted by target within each row.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def stream_seed(seed: int, tag: int) -> np.uint64:
    """Independent stream seed for (seed, tag) pairs."""
    with np.errstate(over="ignore"):
        s = _mix(np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ np.uint64(tag * 0xD1B54A32D192ED03 & 0xFFFFFFFFFFFFFFFF)],
                          dtype=np.uint64))
    return s[0]


def rand_u64(seed: np.uint64, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output number ``counters`` of the stream started at ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(np.uint64(seed) + (c + np.uint64(1)) * GAMMA)


def rand_unit(seed: np.uint64, counters: np.ndarray) -> np.ndarray:
    """Doubles uniform in [0, 1) with 53 random bits."""
    r = rand_u64(seed, counters) >> np.uint64(11)
    return r.astype(np.float64) * (1.0 / 9007199254740992.0)


def rand_int(seed: np.uint64, counters: np.ndarray, lo, hi) -> np.ndarray:
    """Integers uniform in [lo, hi] (inclusive; hi - lo < 2**53).

    floor(u * range) with u a 53-bit double: exact IEEE arithmetic, so the
    values are reproducible; the bias is below range / 2**53.
    """
    lo = np.asarray(lo, dtype=np.uint64)
    hi = np.asarray(hi, dtype=np.uint64)
    span = (hi - lo + np.uint64(1)).astype(np.float64)
    u = rand_unit(seed, counters)
    v = np.floor(u * span)
    v = np.minimum(v, span - 1.0)
    return lo + v.astype(np.uint64)


@dataclass
class Graph:
    """A directed graph in CSR form (rows sorted by target)."""
    name: str
    n: int
    offsets: np.ndarray  # uint64 [n+1]
    targets: np.ndarray  # uint32 [m]
    weights: np.ndarray  # uint32 [m]

    @property
    def m(self) -> int:
        return int(self.targets.shape[0])

    def max_degree(self) -> int:
        if self.n == 0:
            return 0
        return int(np.max(np.diff(self.offsets))) if self.n else 0


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray, name: str) -> Graph:
    """Build CSR with rows sorted by (target, weight) from an edge list."""
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    w = np.asarray(w, dtype=np.uint32)
    if n <= (1 << 31):
        key = src * np.uint64(n) + dst
        order = np.argsort(key, kind="stable")
        # equal (src, dst) pairs (multi-edges) are ordered by weight
        ks = key[order]
        dup = np.nonzero(ks[1:] == ks[:-1])[0]
        if dup.size:
            order = np.lexsort((w, dst, src))
    else:
        order = np.lexsort((w, dst, src))
    src, dst, w = src[order], dst[order], w[order]
    counts = np.bincount(src.astype(np.int64), minlength=n).astype(np.uint64)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=offsets[1:])
    return Graph(name, n, offsets, dst.astype(np.uint32), w)


def shuffle_rows(g: Graph, seed: int) -> Graph:
    """The same graph with the out-edges of every vertex in a random order
    (seeded): a CSR input whose rows are not sorted by target."""
    s = stream_seed(seed, 12)
    m = g.m
    row = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.offsets).astype(np.int64))
    r = rand_u64(s, np.arange(m, dtype=np.uint64))
    order = np.lexsort((r, row))  # by row, randomly within a row
    return Graph(g.name + "_shuffled", g.n, g.offsets.copy(), g.targets[order].copy(), g.weights[order].copy())


def _undirected(n, a, b, w, name):
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    return csr_from_edges(n, src, dst, ww, name)


def grid4(rows: int, cols: int, wlo: int = 1, whi: int = 100, seed: int = 1) -> Graph:
    """4-neighbour grid, vertex id = y*cols + x; each undirected neighbour pair
    gets one weight uniform in [wlo, whi], used in both directions."""
    ids = np.arange(rows * cols, dtype=np.uint64).reshape(rows, cols)
    a = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    b = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    s = stream_seed(seed, 1)
    w = rand_int(s, np.arange(a.shape[0], dtype=np.uint64), wlo, whi).astype(np.uint32)
    return _undirected(rows * cols, a, b, w, f"grid4_{rows}x{cols}")


def grid8_pairs(rows: int, cols: int):
    ids = np.arange(rows * cols, dtype=np.uint64).reshape(rows, cols)
    a = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel(), ids[:-1, :-1].ravel(), ids[:-1, 1:].ravel()])
    b = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel(), ids[1:, 1:].ravel(), ids[1:, :-1].ravel()])
    return a, b


def loguniform_weights(seed: np.uint64, count: int, wmax: int) -> np.ndarray:
    """w = min(wmax, floor(exp(u * ln(wmax + 1)))), u uniform in [0, 1): integer
    weights in [1, wmax] with a log-uniform distribution."""
    u = rand_unit(seed, np.arange(count, dtype=np.uint64))
    w = np.floor(np.exp(u * math.log(wmax + 1)))
    return np.clip(w, 1, wmax).astype(np.uint32)


def grid8(rows: int, cols: int, wmax: int = 10000, seed: int = 4, uniform=None) -> Graph:
    """8-neighbour grid (axis and diagonal neighbours), one weight per undirected
    pair.  Weights log-uniform integers in [1, wmax] unless ``uniform=(lo, hi)``."""
    a, b = grid8_pairs(rows, cols)
    s = stream_seed(seed, 2)
    if uniform is None:
        w = loguniform_weights(s, a.shape[0], wmax)
    else:
        w = rand_int(s, np.arange(a.shape[0], dtype=np.uint64), uniform[0], uniform[1]).astype(np.uint32)
    return _undirected(rows * cols, a, b, w, f"grid8_{rows}x{cols}")


def ring_lattice(n: int, k: int = 16, wlo: int = 1, whi: int = 1000, seed: int = 2) -> Graph:
    """Ring lattice: vertex i linked to i±j (mod n) for j = 1..k; one weight per
    undirected pair {i, i+j}, uniform in [wlo, whi], used in both directions.
    Built directly in CSR (rows sorted by target) without an edge-list sort."""
    assert n > 2 * k
    s = stream_seed(seed, 3)
    i = np.arange(n, dtype=np.uint64)
    # weight of pair (i, i+j mod n) is draw number i*k + (j-1)
    wpair = rand_int(s, np.arange(n * k, dtype=np.uint64), wlo, whi).astype(np.uint32).reshape(n, k)
    # neighbour offsets sorted: -k..-1, +1..+k; row of vertex i holds targets (i+delta) mod n
    deltas = np.concatenate([np.arange(-k, 0), np.arange(1, k + 1)]).astype(np.int64)
    tgt = (i.astype(np.int64)[:, None] + deltas[None, :]) % n
    # weight for delta<0: pair (i+delta, i) with j=-delta  -> wpair[(i+delta) mod n, -delta-1]
    wt = np.empty((n, 2 * k), dtype=np.uint32)
    for c, dl in enumerate(deltas):
        if dl < 0:
            wt[:, c] = wpair[(np.arange(n) + dl) % n, -dl - 1]
        else:
            wt[:, c] = wpair[:, dl - 1]
    # sort each row by target value (wrap-around rows near 0 and n-1 are not monotone)
    order = np.argsort(tgt, axis=1, kind="stable")
    tgt = np.take_along_axis(tgt, order, axis=1)
    wt = np.take_along_axis(wt, order, axis=1)
    offsets = (np.arange(n + 1, dtype=np.uint64) * np.uint64(2 * k))
    return Graph(f"ring_{n}_k{k}", n, offsets, tgt.astype(np.uint32).ravel(), wt.ravel())


def random_graph(n: int, m: int, wlo: int, whi: int, seed: int, self_loops=True) -> Graph:
    """Uniform random directed multigraph (test fixture: zero weights,
    multi-edges and self-loops allowed)."""
    s = stream_seed(seed, 5)
    c = np.arange(3 * m, dtype=np.uint64)
    src = rand_int(s, c[0::3], 0, n - 1) if m else np.zeros(0, np.uint64)
    dst = rand_int(s, c[1::3], 0, n - 1) if m else np.zeros(0, np.uint64)
    w = rand_int(s, c[2::3], wlo, whi).astype(np.uint32) if m else np.zeros(0, np.uint32)
    if not self_loops and m:
        keep = src != dst
        src, dst, w = src[keep], dst[keep], w[keep]
    return csr_from_edges(n, src, dst, w, f"rand_{n}_{m}")


def path_graph(n: int, seed: int = 7, wlo: int = 0, whi: int = 9) -> Graph:
    """Directed path 0 -> 1 -> ... -> n-1 with random weights."""
    s = stream_seed(seed, 6)
    w = rand_int(s, np.arange(max(n - 1, 0), dtype=np.uint64), wlo, whi).astype(np.uint32)
    src = np.arange(n - 1, dtype=np.uint64)
    return csr_from_edges(n, src, src + np.uint64(1), w, f"path_{n}")


def rgg(n: int, mean_degree: float = 24.0, seed: int = 9) -> Graph:
    """Random geometric graph: n points uniform in the unit square, an undirected
    edge between points closer than r = sqrt(mean_degree / (pi n)), both
    directions, weight round(1000 * length) + 1.  Neighbours are found by
    binning points into cells of side >= r and testing each pair of points in
    the same or adjacent cells once."""
    s = stream_seed(seed, 8)
    xy = rand_unit(s, np.arange(2 * n, dtype=np.uint64)).reshape(n, 2)
    r = math.sqrt(mean_degree / (math.pi * n))
    g = max(1, int(1.0 / r))
    cell = np.minimum((xy * g).astype(np.int64), g - 1)
    cid = cell[:, 0] * g + cell[:, 1]
    order = np.argsort(cid, kind="stable")
    cid_sorted = cid[order]
    starts = np.searchsorted(cid_sorted, np.arange(g * g + 1))
    cs = cell[order]
    srcs, dsts = [], []
    # half stencil: same cell (pairs i < j) and 4 of the 8 neighbour cells
    for dx, dy in ((0, 0), (0, 1), (1, -1), (1, 0), (1, 1)):
        nx = cs[:, 0] + dx
        ny = cs[:, 1] + dy
        ok = (nx >= 0) & (nx < g) & (ny >= 0) & (ny < g)
        pts = np.nonzero(ok)[0]
        nc = nx[pts] * g + ny[pts]
        lo = starts[nc]
        cnt = starts[nc + 1] - lo
        tot = int(cnt.sum())
        rep = np.repeat(pts, cnt)
        first = np.repeat(lo - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
        cand = first + np.arange(tot, dtype=np.int64)
        if dx == 0 and dy == 0:
            keep = rep < cand
            rep, cand = rep[keep], cand[keep]
        a, b = order[rep], order[cand]
        d2 = ((xy[a] - xy[b]) ** 2).sum(axis=1)
        keep = d2 < r * r
        srcs.append(a[keep])
        dsts.append(b[keep])
    a = np.concatenate(srcs)
    b = np.concatenate(dsts)
    d = np.sqrt(((xy[a] - xy[b]) ** 2).sum(axis=1))
    w = (np.rint(1000.0 * d) + 1).astype(np.uint32)
    return _undirected(n, a.astype(np.uint64), b.astype(np.uint64), w, f"rgg_{n}")


def paper_dag(n: int, m: int, seed: int = 11) -> Graph:
    """Random high-diameter DAG in the shape the paper evaluates on (Section 4.2).

    0-indexed here: chain edges (i, i+1) of weight 1 for i < n-1, then m-n+1
    extra forward edges (u, v), u < v, with weight 2*(v-u), which keeps the
    chain the unique shortest path, so dist(i) = i from source 0.  Extra edges
    are spread uniformly over the tails u in [0, n-2] subject to vertex u
    having at most n-1-u out-edges in total (a multigraph is avoided by
    drawing distinct heads per tail).  Tail counts that exceed a vertex's cap
    are clipped and the excess is handed to lower-index vertices, which have
    the most room."""
    extra = m - (n - 1)
    assert 0 <= extra <= (n - 1) * n // 2 - (n - 1)
    s = stream_seed(seed, 10)
    tails = rand_int(s, np.arange(extra, dtype=np.uint64), 0, n - 2).astype(np.int64)
    cnt = np.bincount(tails, minlength=n).astype(np.int64)
    cap = np.maximum(n - 1 - np.arange(n) - 1, 0)  # room besides the chain edge
    over = np.maximum(cnt - cap, 0)
    cnt = np.minimum(cnt, cap)
    left = int(over.sum())
    u = 0
    while left > 0:
        room = cap[u] - cnt[u]
        take = min(room, left)
        cnt[u] += take
        left -= take
        u += 1
    # CSR built row by row: vertex u's row is its chain edge (u, u+1) followed
    # by its extra heads in increasing order (all > u+1), so rows come out
    # sorted by target with no edge-list sort.
    deg = cnt.copy()
    deg[: n - 1] += 1
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(deg, out=offsets[1:])
    targets = np.empty(int(offsets[-1]), dtype=np.uint32)
    weights = np.empty(int(offsets[-1]), dtype=np.uint32)
    s2 = stream_seed(seed, 11)
    for uu in range(n - 1):
        o = int(offsets[uu])
        targets[o] = uu + 1
        weights[o] = 1
        k = int(cnt[uu])
        if k == 0:
            continue
        # k distinct heads among uu+2 .. n-1: the k smallest of one random draw per candidate
        cand = np.arange(uu + 2, n, dtype=np.int64)
        if k == cand.shape[0]:
            pick = cand
        else:
            r = rand_u64(s2, np.arange(uu * n, uu * n + cand.shape[0], dtype=np.uint64))
            pick = np.sort(cand[np.argpartition(r, k - 1)[:k]])
        targets[o + 1:o + 1 + k] = pick
        weights[o + 1:o + 1 + k] = 2 * (pick - uu)
    return Graph(f"dag_{n}_{m}", n, offsets, targets, weights)


# ---------------------------------------------------------------------------
# Heap workloads (keys uint64, ids uint32)
# ---------------------------------------------------------------------------

def heap_init_pairs(n_ids: int, key_bits: int = 40, seed: int = 3):
    """ids 0..n_ids-1 once each (shuffled order), keys uniform in [0, 2**key_bits)."""
    s = stream_seed(seed, 20)
    keys = rand_u64(s, np.arange(n_ids, dtype=np.uint64)) >> np.uint64(64 - key_bits)
    perm_keys = rand_u64(stream_seed(seed, 21), np.arange(n_ids, dtype=np.uint64))
    order = np.argsort(perm_keys, kind="stable")
    return keys[order].astype(np.uint64), order.astype(np.uint32)


def decrease_batch(live_ids: np.ndarray, live_keys_of, count: int, seed: int, rnd: int):
    """One batch of ``count`` decrease-keys: ids drawn with replacement from
    ``live_ids``; new key = old key - uniform[0, floor(old/2)].

    ``live_keys_of(ids)`` returns the current keys of the drawn ids."""
    s = stream_seed(seed, 1000 + rnd)
    c = np.arange(2 * count, dtype=np.uint64)
    pick = rand_int(s, c[0::2], 0, live_ids.shape[0] - 1).astype(np.int64)
    ids = live_ids[pick]
    old = live_keys_of(ids).astype(np.uint64)
    dec = rand_int(s, c[1::2], np.zeros(count, np.uint64), old >> np.uint64(1))
    return (old - dec).astype(np.uint64), ids.astype(np.uint32)


def random_script(n_ops: int, id_cap: int, max_batch: int, key_max: int, seed: int, deletes: bool = False):
    """A random script of heap operations for tests:
    list of ("update", keys, ids) / ("extract", k), and with ``deletes`` also
    ("delete", ids) (ids drawn from the whole id range, so some are absent)."""
    s = stream_seed(seed, 31 if deletes else 30)
    ctr = 0
    ops = []
    for _ in range(n_ops):
        r = rand_u64(s, np.array([ctr], dtype=np.uint64))[0]
        ctr += 1
        if deletes and r % np.uint64(4) == 1:
            cnt = int(rand_int(s, np.array([ctr], np.uint64), 0, max_batch)[0])
            ctr += 1
            c = np.arange(ctr, ctr + cnt, dtype=np.uint64)
            ctr += cnt
            ids = rand_int(s, c, 0, id_cap - 1).astype(np.uint32) if cnt else np.zeros(0, np.uint32)
            ops.append(("delete", ids))
        elif r % np.uint64(3) != 0:
            cnt = int(rand_int(s, np.array([ctr], np.uint64), 0, max_batch)[0])
            ctr += 1
            c = np.arange(ctr, ctr + 2 * cnt, dtype=np.uint64)
            ctr += 2 * cnt
            ids = rand_int(s, c[0::2], 0, id_cap - 1).astype(np.uint32) if cnt else np.zeros(0, np.uint32)
            keys = rand_int(s, c[1::2], 0, key_max).astype(np.uint64) if cnt else np.zeros(0, np.uint64)
            ops.append(("update", keys, ids))
        else:
            k = int(rand_int(s, np.array([ctr], np.uint64), 0, 2 * max_batch + 1)[0])
            ctr += 1
            ops.append(("extract", k))
    return ops


def _rgg_item(args):
    gi, n, seed, k = args
    g = rgg(n, 24.0, seed=seed * 1000 + gi)
    s2 = stream_seed(seed * 1000 + gi, 41)
    src = []
    c = 0
    while len(src) < min(k, n):
        v = int(rand_int(s2, np.array([c], np.uint64), 0, n - 1)[0])
        c += 1
        if v not in src:
            src.append(v)
    return g, src


def rgg_batch(n_graphs: int = 64, sources_per_graph: int = 4, lo_log2: int = 12, hi_log2: int = 18,
              seed: int = 50, workers: int = 8):
    """The multi-source workload: n_graphs random geometric graphs with
    n_g = floor(2^(lo + (hi-lo) u)), u uniform in [0, 1) (uneven sizes),
    mean degree 24, and `sources_per_graph` distinct sources each.
    Returns a list of (graph, [sources])."""
    s = stream_seed(seed, 40)
    u = rand_unit(s, np.arange(n_graphs, dtype=np.uint64))
    items = [(gi, int(np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u[gi]))), seed, sources_per_graph)
             for gi in range(n_graphs)]
    workers = max(1, min(workers, os.cpu_count() or 1))
    if workers == 1:
        return [_rgg_item(it) for it in items]
    import multiprocessing as mp
    # close + join rather than the context manager, whose exit terminates
    # (signals) the workers; inside a profiled process that signal is caught
    # by the profiler's handlers.
    pool = mp.get_context("fork").Pool(workers)
    try:
        out = pool.map(_rgg_item, items, chunksize=1)
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return out


def training_graphs(count: int = 200, lo_log2: int = 14, hi_log2: int = 18, seed: int = 70):
    """Graphs whose plain parDijkstra runs train the extraction-threshold model:
    ring lattices (w ~ U[1,1000]), 4-neighbour grids (w ~ U[1,100]) and
    8-neighbour grids (log-uniform w in [1, 10^4]) in turn, with n log-uniform
    in [2^lo, 2^hi] (grids use the nearest square)."""
    s = stream_seed(seed, 60)
    u = rand_unit(s, np.arange(count, dtype=np.uint64))
    out = []
    for i in range(count):
        n = int(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u[i]))
        fam = i % 3
        if fam == 0:
            out.append(ring_lattice(max(n, 64), 16, 1, 1000, seed=seed * 1000 + i))
        else:
            side = max(8, int(round(math.sqrt(n))))
            if fam == 1:
                out.append(grid4(side, side, 1, 100, seed=seed * 1000 + i))
            else:
                out.append(grid8(side, side, wmax=10000, seed=seed * 1000 + i))
    return out
