"""Pins of the oracle against things other than itself (CPU only).

* priority queue: brute force on tiny scripts, sort-equivalence with no
  updates, the hand-worked example in tests/golden, per-call invariants, and
  agreement of the numpy formulation with the sorted-multiset one;
* shortest paths: Bellman-Ford brute force, closed forms (unit grid, unit ring
  lattice, path prefix sums, the paper's DAG), the path-optimality invariants,
  settle order, and the relaxation count.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


# ----------------------------------------------------------------------------- PQ
class BrutePQ:
    """Dictionary of live ids; extractMin scans every live element."""

    def __init__(self):
        self.live = {}

    def update(self, k, i):
        if i not in self.live or k < self.live[i]:
            self.live[i] = k

    def delete(self, i):
        self.live.pop(i, None)

    def extract(self, k):
        out = []
        for _ in range(k):
            if not self.live:
                break
            best = None
            for i, kk in self.live.items():
                if best is None or (kk, i) < best:
                    best = (kk, i)
            del self.live[best[1]]
            out.append(best)
        return out


def _run_script(pq, ops):
    res = []
    for op in ops:
        if op[0] == "update":
            pq.bulk_update(op[1], op[2])
        elif op[0] == "delete":
            res.append(pq.delete(op[1]))
        else:
            k, v = pq.extract_min(op[1])
            res.append(list(zip(k.tolist(), v.tolist())))
    return res


@pytest.mark.parametrize("seed", range(25))
def test_pq_matches_brute_force(seed):
    cap = [1, 5, 17, 64][seed % 4]
    ops = W.random_script(40, cap, 9, [0, 3, 1000][seed % 3], seed)
    bp = BrutePQ()
    expect = []
    for op in ops:
        if op[0] == "update":
            for k, i in zip(op[1].tolist(), op[2].tolist()):
                bp.update(k, i)
        else:
            expect.append(bp.extract(op[1]))
    got = _run_script(oracle.PQ(cap), ops)
    assert got == [[tuple(x) for x in e] for e in expect]


@pytest.mark.parametrize("seed", range(10))
def test_pq_arrays_matches_multiset(seed):
    cap = [3, 40, 300][seed % 3]
    ops = W.random_script(60, cap, 30, [2, 10**6][seed % 2], 100 + seed)
    a = _run_script(oracle.PQ(cap), ops)
    b = _run_script(oracle.PQArrays(cap), ops)
    assert a == b


def _brute(ops):
    bp = BrutePQ()
    expect = []
    for op in ops:
        if op[0] == "update":
            for k, i in zip(op[1].tolist(), op[2].tolist()):
                bp.update(k, i)
        elif op[0] == "delete":
            before = len(bp.live)
            for i in op[1].tolist():
                bp.delete(i)
            expect.append(before - len(bp.live))
        else:
            expect.append([tuple(x) for x in bp.extract(op[1])])
    return expect


@pytest.mark.parametrize("seed", range(25))
def test_pq_delete_matches_brute_force(seed):
    """Scripts mixing bulk updates, deletes (of present and absent ids, with
    repeats) and batched extracts: every extract sequence and every count of
    removed elements equals the dictionary brute force."""
    cap = [1, 5, 17, 64][seed % 4]
    ops = W.random_script(50, cap, 9, [0, 3, 1000][seed % 3], seed, deletes=True)
    assert any(op[0] == "delete" for op in ops)
    got = _run_script(oracle.PQ(cap), ops)
    exp = _brute(ops)
    assert [g if isinstance(g, int) else [tuple(x) for x in g] for g in got] == exp


@pytest.mark.parametrize("seed", range(8))
def test_pq_arrays_delete_matches_multiset(seed):
    cap = [3, 40, 300][seed % 3]
    ops = W.random_script(60, cap, 30, [2, 10**6][seed % 2], 200 + seed, deletes=True)
    assert _run_script(oracle.PQ(cap), ops) == _run_script(oracle.PQArrays(cap), ops)


def test_pq_delete_then_drain_is_a_sort_of_the_rest():
    """Deleting a set of ids, then extracting everything, gives the sorted
    (key, id) list of the pairs that were not deleted (library sort)."""
    keys, ids = W.heap_init_pairs(3000, key_bits=10, seed=8)
    gone = ids[::3]
    for cls in (oracle.PQ, oracle.PQArrays):
        pq = cls(3000)
        pq.bulk_update(keys, ids)
        assert pq.delete(gone) == gone.shape[0]
        assert pq.delete(gone) == 0                                      # already absent
        k, v = pq.extract_min(5000)
        keep = np.ones(3000, bool)
        keep[gone] = False
        kk, vv = keys[keep[ids]], ids[keep[ids]]
        order = np.lexsort((vv, kk))
        assert np.array_equal(k, kk[order]) and np.array_equal(v, vv[order])


def test_pq_delete_worked_example():
    ex = json.load(open(os.path.join(GOLD, "pq_delete_worked_example.json")))
    for cls in (oracle.PQ, oracle.PQArrays):
        pq = cls(ex["id_capacity"])
        for st in ex["steps"]:
            if st["op"] == "update":
                p = np.array(st["pairs"], dtype=np.uint64).reshape(-1, 2)
                pq.bulk_update(p[:, 0], p[:, 1].astype(np.uint32))
            elif st["op"] == "delete":
                assert pq.delete(np.array(st["ids"], np.uint32)) == st["removed"]
            else:
                k, v = pq.extract_min(st["k"])
                assert [[int(a), int(b)] for a, b in zip(k, v)] == st["expect"]
            if "live_after" in st:
                cur = pq.cur() if cls is oracle.PQ else pq.cur
                live = {str(i): int(cur[i]) for i in np.nonzero(cur != INF)[0]}
                assert live == st["live_after"]


def test_pq_delete_rejects_bad_input():
    pq = oracle.PQ(4)
    pq.bulk_update([3], [1])
    with pytest.raises(ValueError):
        pq.delete([0, 4])
    assert pq.size() == 1                                                # nothing was applied


def test_pq_without_updates_is_a_sort():
    keys, ids = W.heap_init_pairs(5000, key_bits=12, seed=5)  # 12-bit keys: many ties
    pq = oracle.PQ(5000)
    pq.bulk_update(keys, ids)
    outk, outi = [], []
    for k in [1, 7, 100, 0, 3000, 5000]:
        a, b = pq.extract_min(k)
        outk.append(a)
        outi.append(b)
    outk, outi = np.concatenate(outk), np.concatenate(outi)
    order = np.lexsort((ids, keys))  # library sort by (key, id)
    assert np.array_equal(outk, keys[order]) and np.array_equal(outi, ids[order])
    assert pq.size() == 0


def test_pq_worked_example():
    ex = json.load(open(os.path.join(GOLD, "pq_worked_example.json")))
    for cls in (oracle.PQ, oracle.PQArrays):
        pq = cls(ex["id_capacity"])
        for st in ex["steps"]:
            if st["op"] == "update":
                p = np.array(st["pairs"], dtype=np.uint64).reshape(-1, 2)
                pq.bulk_update(p[:, 0], p[:, 1].astype(np.uint32))
                if "live_after" in st:
                    cur = pq.cur() if cls is oracle.PQ else pq.cur
                    live = {str(i): int(cur[i]) for i in np.nonzero(cur != INF)[0]}
                    assert live == {k: v for k, v in st["live_after"].items()}
            else:
                k, v = pq.extract_min(st["k"])
                assert [[int(a), int(b)] for a, b in zip(k, v)] == st["expect"]


@pytest.mark.parametrize("seed", range(8))
def test_pq_call_invariants(seed):
    cap = 200
    ops = W.random_script(80, cap, 40, 500, 300 + seed)
    pq = oracle.PQ(cap)
    size = 0
    for op in ops:
        if op[0] == "update":
            before = pq.cur()
            pq.bulk_update(op[1], op[2])
            newly = len({int(i) for k, i in zip(op[1], op[2]) if before[int(i)] == INF})
            size += newly
        else:
            cur = pq.cur()
            k, v = pq.extract_min(op[1])
            assert len(set(v.tolist())) == len(v)                       # no id twice
            pairs = list(zip(k.tolist(), v.tolist()))
            assert pairs == sorted(pairs)                                # ascending
            assert all(cur[i] == kk for kk, i in pairs)                 # each = current key
            assert len(v) == min(op[1], size)
            size -= len(v)
        assert pq.size() == size


def test_pq_rejects_bad_input():
    pq = oracle.PQ(4)
    with pytest.raises(ValueError):
        pq.bulk_update([1], [4])
    with pytest.raises(ValueError):
        pq.bulk_update([int(INF)], [0])
    assert pq.size() == 0


# --------------------------------------------------------------------------- SSSP
def _reach(g, src):
    seen = np.zeros(g.n, bool)
    seen[src] = True
    stack = [src]
    while stack:
        u = stack.pop()
        for v in g.targets[g.offsets[u]:g.offsets[u + 1]]:
            if not seen[v]:
                seen[v] = True
                stack.append(int(v))
    return seen


def check_sssp_invariants(g, src, dist):
    """dist[src]=0; dist[v] <= dist[u]+w on every edge out of a reached u;
    equality on some in-edge of every reached v != src; INF <=> unreachable."""
    assert dist[src] == 0
    deg = np.diff(g.offsets).astype(np.int64)
    u = np.repeat(np.arange(g.n), deg)
    v = g.targets.astype(np.int64)
    du = dist[u]
    ok = du != INF
    cand = du[ok] + g.weights[ok].astype(np.uint64)
    assert np.all(dist[v[ok]] <= cand)
    tight = np.zeros(g.n, bool)
    tight[v[ok][dist[v[ok]] == cand]] = True
    reached = dist != INF
    need = reached.copy()
    need[src] = False
    assert np.all(tight[need])
    assert np.array_equal(reached, _reach(g, src))


@pytest.mark.parametrize("seed", range(200))
def test_dijkstra_matches_bellman_ford(seed):
    n = 1 + seed % 37
    m = (seed * 7) % (4 * n + 3)
    wl, wh = [(0, 0), (0, 3), (1, 10), (0, 1000)][seed % 4]
    g = W.random_graph(n, m, wl, wh, seed)
    src = seed % n
    d1 = oracle.dijkstra(g, src)
    d2 = oracle.bellman_ford(g, src)
    assert np.array_equal(d1, d2)
    check_sssp_invariants(g, src, d1)


def test_sssp_worked_example():
    ex = json.load(open(os.path.join(GOLD, "sssp_worked_example.json")))
    e = np.array(ex["edges"], dtype=np.uint64)
    g = W.csr_from_edges(ex["n"], e[:, 0], e[:, 1], e[:, 2].astype(np.uint32), "ex")
    d, order, _ = oracle.dijkstra(g, ex["source_vertex"], want_order=True)
    assert d.tolist() == ex["dist"]
    assert order.tolist() == ex["settle_order"]


def test_closed_form_unit_grid():
    R, Cc = 23, 31
    g = W.grid4(R, Cc, 1, 1)
    d = oracle.dijkstra(g, 0)
    y, x = np.divmod(np.arange(R * Cc), Cc)
    assert np.array_equal(d, (x + y).astype(np.uint64))


def test_closed_form_unit_ring():
    n, k = 1000, 16
    g = W.ring_lattice(n, k, 1, 1)
    d = oracle.dijkstra(g, 0)
    i = np.arange(n)
    hops = np.minimum(i, n - i)
    assert np.array_equal(d, ((hops + k - 1) // k).astype(np.uint64))


def test_closed_form_path():
    g = W.path_graph(300, seed=3, wlo=0, whi=50)
    d = oracle.dijkstra(g, 0)
    expect = np.concatenate([[0], np.cumsum(g.weights.astype(np.uint64))])
    assert np.array_equal(d, expect)
    d5 = oracle.dijkstra(g, 5)
    assert np.all(d5[:5] == INF) and np.array_equal(d5[5:], expect[5:] - expect[5])


def test_closed_form_paper_dag():
    n = 400
    g = W.paper_dag(n, 20000, seed=1)
    assert g.m == 20000
    d = oracle.dijkstra(g, 0)
    assert np.array_equal(d, np.arange(n, dtype=np.uint64))
    # every non-chain edge u->v has weight 2(v-u): DAG, forward only
    u = np.repeat(np.arange(n), np.diff(g.offsets).astype(np.int64))
    v = g.targets.astype(np.int64)
    assert np.all(v > u)
    assert np.all(g.weights == np.where(v == u + 1, 1, 2 * (v - u)))


@pytest.mark.parametrize("make", [
    lambda: W.grid4(20, 30, 1, 100, seed=3),
    lambda: W.ring_lattice(700, 16, 1, 1000, seed=4),
    lambda: W.grid8(17, 19, wmax=10000, seed=5),
    lambda: W.rgg(1500, seed=6),
])
def test_settle_order_and_counts(make):
    g = make()
    d, order, nrelax = oracle.dijkstra(g, 0, want_order=True)
    reached = np.nonzero(d != INF)[0]
    expect = reached[np.lexsort((reached, d[reached]))]     # ascending (dist, id)
    assert np.array_equal(order, expect)
    deg = np.diff(g.offsets).astype(np.int64)
    assert nrelax == int(deg[reached].sum())
    check_sssp_invariants(g, 0, d)


def test_generators_sizes():
    assert W.grid4(64, 64).m == 16128
    assert W.ring_lattice(1 << 12).m == 2 * 16 * (1 << 12)
    assert W.grid8(64, 64).m == 2 * (2 * 64 * 63 + 2 * 63 * 63)
    g = W.ring_lattice(1 << 10, 16, 1, 1000, seed=2)
    assert g.weights.min() >= 1 and g.weights.max() <= 1000
    # weight symmetry: w(u,v) == w(v,u)
    u = np.repeat(np.arange(g.n), np.diff(g.offsets).astype(np.int64))
    fwd = dict(zip(zip(u.tolist(), g.targets.tolist()), g.weights.tolist()))
    assert all(fwd[(b, a)] == w for (a, b), w in fwd.items())


def test_oracle_rejects_bad_graph():
    g = W.grid4(3, 3)
    bad = W.Graph("bad", g.n, g.offsets.copy(), g.targets.copy(), g.weights)
    bad.targets[0] = 99
    with pytest.raises(ValueError):
        oracle.dijkstra(bad, 0)
    with pytest.raises(ValueError):
        oracle.dijkstra(g, 9)
