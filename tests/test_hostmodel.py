"""CPU tests of the GPU kernels' heap and parDijkstra logic.

tests/hostmodel builds the same team-templated code as the kernels with a
one-thread team.  These tests run adversarial operation scripts and graphs
through it and compare with the oracle, and check the structural invariants of
the parallel bucket heap after every operation:

* every bucket and signal buffer is sorted by id with unique ids (Section 2.1);
* B_i <= p_i < every element of levels > i, and p_0 <= p_1 <= ... (Section 2.1,
  the heap property between levels);
* sizes never exceed the allocated buffers; after an operation S_0 is empty
  (Resolve(0) postcondition, Algorithm 1);
* B_0 holds only live elements (its keys equal the current keys);
* the element count never exceeds what was inserted.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from hostmodel import INF, HostHeap, sssp as hm_sssp


def check_structure(h: HostHeap, cur: np.ndarray, d: int):
    L = h.levels()
    q, ell = L["q"], L["ell"]
    deeper_min = None  # smallest (key, id) at levels > i, scanning bottom-up
    levels = []
    for i in range(q):
        bk, bv, sk, sv = h.items(i, int(L["nB"][i]), int(L["nS"][i]))
        levels.append((bk, bv, sk, sv))
        assert int(L["nB"][i]) <= 4 * d * 4 ** i and int(L["nS"][i]) <= 2 * d * 4 ** i
        for ids in (bv, sv):
            assert np.all(np.diff(ids.astype(np.int64)) > 0), "not sorted by id / duplicate id"
    assert L["nS"][0] == 0
    nonempty = [i for i in range(q) if L["nB"][i] + L["nS"][i] > 0]
    assert ell == (max(nonempty) if nonempty else -1)
    # pivots: B_i <= p_i < everything deeper; p non-decreasing
    pks = [(int(L["pk"][i]), int(L["pv"][i])) for i in range(q)]
    for i in range(q):
        bk, bv, sk, sv = levels[i]
        p = pks[i]
        for k, v in zip(bk.tolist(), bv.tolist()):
            assert (k, v) <= p
        for j in range(i + 1, q):
            for arrk, arrv in ((levels[j][0], levels[j][1]), (levels[j][2], levels[j][3])):
                for k, v in zip(arrk.tolist(), arrv.tolist()):
                    assert (k, v) > p
        if i < ell:
            # S_{i+1} elements are > p_i (checked above); p_i <= p_{i+1}
            assert pks[i] <= pks[i + 1]
    # B_0 only live elements
    bk, bv = levels[0][0], levels[0][1]
    assert np.array_equal(cur[bv], bk)
    return L


@pytest.mark.parametrize("seed", range(40))
def test_random_scripts_vs_oracle(seed):
    d = [1, 2, 3, 4, 7, 16][seed % 6]
    cap = [5, 40, 300, 1000][seed % 4]
    sched = seed % 2
    maxb = [d, 3 * d, 60][seed % 3]
    ops = W.random_script(60, cap, maxb, [3, 50, 10 ** 9][seed % 3], 500 + seed)
    h = HostHeap(cap, d, sched)
    o = oracle.PQ(cap)
    for op in ops:
        if op[0] == "update":
            h.bulk_update(op[1], op[2])
            o.bulk_update(op[1], op[2])
        else:
            k1, v1 = h.extract_min(op[1])
            k2, v2 = o.extract_min(op[1])
            assert np.array_equal(k1, k2) and np.array_equal(v1, v2)
        L = check_structure(h, o.cur(), d)
        assert L["live"] == o.size()


@pytest.mark.parametrize("seed", range(30))
def test_random_scripts_with_deletes_vs_oracle(seed):
    """Delete (Section 1.2) mixed with bulk updates and batched extracts:
    extract sequences and sizes equal the oracle's after every operation, and
    the level structure keeps its invariants (B_0 holds only live elements,
    so a deleted id is never extracted)."""
    d = [1, 2, 3, 4, 7, 16][seed % 6]
    cap = [5, 40, 300, 1000][seed % 4]
    maxb = [d, 3 * d, 60][seed % 3]
    ops = W.random_script(70, cap, maxb, [3, 50, 10 ** 9][seed % 3], 700 + seed, deletes=True)
    h = HostHeap(cap, d, seed % 2)
    o = oracle.PQ(cap)
    for op in ops:
        if op[0] == "update":
            h.bulk_update(op[1], op[2])
            o.bulk_update(op[1], op[2])
        elif op[0] == "delete":
            h.delete(op[1])
            o.delete(op[1])
        else:
            k1, v1 = h.extract_min(op[1])
            k2, v2 = o.extract_min(op[1])
            assert np.array_equal(k1, k2) and np.array_equal(v1, v2)
        L = check_structure(h, o.cur(), d)
        assert L["live"] == o.size()


def test_delete_everything_then_reinsert():
    """Deleting every id leaves dead copies in the deeper levels; the heap
    reports size 0, extracts nothing, and ids inserted again afterwards
    (some with their old keys) come out exactly once."""
    n, d = 3000, 8
    keys, ids = W.heap_init_pairs(n, key_bits=12, seed=4)
    h = HostHeap(n, d)
    o = oracle.PQ(n)
    h.bulk_update(keys, ids)
    o.bulk_update(keys, ids)
    h.delete(ids[::2])
    o.delete(ids[::2])
    h.delete(np.arange(n, dtype=np.uint32))
    o.delete(np.arange(n, dtype=np.uint32))
    assert h.levels()["live"] == 0
    assert h.extract_min(10)[0].shape[0] == 0
    back = ids[: n // 3]
    h.bulk_update(keys[: n // 3], back)
    o.bulk_update(keys[: n // 3], back)
    a = h.extract_min(n)
    b = o.extract_min(n)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert h.levels()["ell"] == -1 or h.levels()["live"] == 0


@pytest.mark.parametrize("seed", range(6))
def test_decrease_key_workload_small(seed):
    """The standalone-heap workload shape at small scale: initial load in
    pieces of d, then rounds of decrease-keys on live ids and batched
    extracts."""
    n_ids, d, rounds, upd, ext = 4096, 64, 12, 256, 64
    keys, ids = W.heap_init_pairs(n_ids, key_bits=20 if seed % 2 else 40, seed=seed)
    h = HostHeap(n_ids, d, seed % 2)
    o = oracle.PQArrays(n_ids)
    for c in range(0, n_ids, d):
        h.bulk_update(keys[c:c + d], ids[c:c + d])
        o.bulk_update(keys[c:c + d], ids[c:c + d])
    for r in range(rounds):
        live = np.nonzero(o.cur != INF)[0].astype(np.uint32)
        if live.size == 0:
            break
        bk, bi = W.decrease_batch(live, lambda x: o.cur[x], upd, seed, r)
        h.bulk_update(bk, bi)
        o.bulk_update(bk, bi)
        k1, v1 = h.extract_min(ext)
        k2, v2 = o.extract_min(ext)
        assert np.array_equal(k1, k2) and np.array_equal(v1, v2)
    check_structure(h, o.cur, d)


def test_drain_and_refill():
    h = HostHeap(2000, 4)
    o = oracle.PQ(2000)
    keys, ids = W.heap_init_pairs(2000, key_bits=10, seed=9)
    h.bulk_update(keys, ids)
    o.bulk_update(keys, ids)
    for k in (1, 2000, 5):
        a = h.extract_min(k)
        b = o.extract_min(k)
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    # re-insert extracted ids with larger keys than before (absent -> insert)
    h.bulk_update(keys + np.uint64(7), ids)
    o.bulk_update(keys + np.uint64(7), ids)
    a = h.extract_min(3000)
    b = o.extract_min(3000)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert h.levels()["ell"] == -1


def _graphs():
    yield W.grid4(13, 17, 1, 100, seed=2)
    yield W.ring_lattice(600, 16, 1, 1000, seed=3)
    yield W.grid8(11, 12, wmax=10000, seed=4)
    yield W.grid4(9, 9, 1, 1, seed=5)
    yield W.rgg(700, seed=6)
    yield W.paper_dag(150, 3000, seed=7)
    # many dead copies pile up in B_1 and B_2: refilling B_0 takes repeated
    # Resolve(0) calls, each dropping a window of dead elements
    yield W.grid8(96, 96, wmax=10000, seed=9)
    for s in range(12):
        yield W.random_graph(1 + 7 * s, 5 * s * s, [0, 0, 1][s % 3], [0, 5, 50][s % 3], 40 + s)


NGRAPHS = 19


@pytest.mark.parametrize("gi", range(NGRAPHS))
@pytest.mark.parametrize("variant", [(0, 0, 0), (1, 0, 2), (0, 1, 1), (0, 3, 0)])
def test_sssp_logic_vs_oracle(gi, variant):
    """Distances, rounds and relaxations equal the oracle's; after every
    operation the smallest live element is in B_0 and each reached vertex is
    extracted or live in the heap exactly once."""
    sched, dmul, qlds = variant
    g = list(_graphs())[gi]
    src = (gi * 7) % g.n
    ref, order, nrelax = oracle.dijkstra(g, src, want_order=True)
    d = 0 if dmul == 0 else max(1, g.max_degree()) * dmul
    rc, dist, st = hm_sssp(g, src, d=d, sched=sched, qlds=qlds, check_live=True)
    assert rc == 0
    assert st["first_bad"] == -1, st["violation"]
    assert np.array_equal(dist, ref)
    assert st["rounds"] == order.shape[0]          # plain rule: one round per settled vertex
    assert st["relax"] == nrelax


def test_sssp_small_capacity_reports_capacity():
    g = W.ring_lattice(2000, 16, 1, 1000, seed=1)
    rc, dist, st = hm_sssp(g, 0, hcap=8)
    # with a tiny heap arena the kernel either succeeds or reports the
    # capacity error; it never writes outside the arena
    assert rc in (0, -2)
    if rc == 0:
        assert np.array_equal(dist, oracle.dijkstra(g, 0))


# ---------------------------------------------------------------- speculative rounds
@pytest.mark.parametrize("gi", range(NGRAPHS))
@pytest.mark.parametrize("kcase", ["fixed4", "fixed64", "random", "adversarial"])
def test_speculative_rounds_exact_for_any_k(gi, kcase):
    """Rounds that extract k > 1 minima re-insert improved vertices, so the
    distances equal the oracle's for every k-sequence."""
    g = list(_graphs())[gi]
    src = (gi * 5) % g.n
    ref, order, _ = oracle.dijkstra(g, src, want_order=True)
    rng = np.random.default_rng(gi)
    if kcase == "fixed4":
        rc, dist, st = hm_sssp(g, src, rule=1, kfix=4)
    elif kcase == "fixed64":
        rc, dist, st = hm_sssp(g, src, rule=1, kfix=64, kmax=64)
    elif kcase == "random":
        rc, dist, st = hm_sssp(g, src, rule=3, kseq=rng.integers(1, 40, size=97), kmax=256)
    else:  # alternate huge pulls with single ones
        rc, dist, st = hm_sssp(g, src, rule=3, kseq=[256, 1, 1, 256, 3], kmax=256, check_live=True)
        assert st["first_bad"] == -1, st["violation"]
    assert rc == 0
    assert np.array_equal(dist, ref)
    assert st["extracted"] >= order.shape[0]       # every reached vertex is extracted at least once
    if kcase == "fixed4":
        assert st["rounds"] <= order.shape[0]


def test_rule_fixed_one_equals_plain_counts():
    g = W.grid4(20, 20, 1, 100, seed=3)
    rc0, d0, s0 = hm_sssp(g, 0)
    rc1, d1, s1 = hm_sssp(g, 0, rule=1, kfix=1)
    assert rc0 == rc1 == 0 and np.array_equal(d0, d1)
    assert s0["rounds"] == s1["rounds"] == s1["extracted"] and s0["relax"] == s1["relax"]


@pytest.mark.parametrize("rule", [0, 2])
def test_trial_limits_settle_everything_below_the_frontier(rule):
    """max_rounds stops after that many rounds and reports the smallest key
    left; stop_key = that key then settles every vertex at or below it, for
    any k rule (the autotuner's equal-work trials)."""
    g = W.grid8(60, 60, wmax=10000, seed=12)
    ref = oracle.dijkstra(g, 0)
    rc, dist, st = hm_sssp(g, 0, max_rounds=500)
    assert rc == 0 and st["stopped"] and st["rounds"] == 500
    D = st["last_key"]
    assert D == int(np.sort(ref)[500])              # plain rounds settle vertices in (dist, id) order
    kw = dict(rule=1, kfix=12) if rule else {}
    rc, dist, st = hm_sssp(g, 0, stop_key=D, **kw)
    assert rc == 0 and st["stopped"] and st["last_key"] > D
    settled = ref <= D
    assert np.array_equal(dist[settled], ref[settled])
    rc, dist, st = hm_sssp(g, 0, stop_key=1 << 62)
    assert rc == 0 and not st["stopped"] and st["last_key"] == 2 ** 64 - 1
    assert np.array_equal(dist, ref)


# ------------------------------------------------- Algorithm 1 and Theorem 1
def _pure_script(n_ops, d, cap, seed):
    """Operations in the setting of Theorem 1: each inserts at most d new
    distinct ids (no key of a present id changes, so no copy of an id is ever
    left behind) or extracts at most d minima."""
    rng = np.random.default_rng(seed)
    fresh = iter(rng.permutation(cap).astype(np.uint32).tolist())
    ops, live = [], 0
    for _ in range(n_ops):
        if live >= d and rng.random() < 0.35:
            k = int(rng.integers(1, d + 1))
            ops.append(("extract", k))
            live -= min(k, live)
            continue
        cnt = int(rng.integers(1, d + 1))
        ids = np.array([next(fresh) for _ in range(cnt)], np.uint32)
        ops.append(("update", rng.integers(0, 1 << 20, size=cnt).astype(np.uint64), ids))
        live += cnt
    return ops


def _apply(h, o, op):
    if op[0] == "update":
        h.bulk_update(op[1], op[2])
        o.bulk_update(op[1], op[2])
    elif op[0] == "delete":
        h.delete(op[1])
        o.delete(op[1])
    else:
        a = h.extract_min(op[1])
        b = o.extract_min(op[1])
        assert all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("seed", range(8))
def test_theorem1_schedule_and_algorithm1_conditions(seed):
    """Schedule 0 on operations of at most d elements (Theorem 1's setting):

    * every operation is followed by Resolve(0), then Resolve(i) runs exactly
      when the count of Resolve(i-1) reaches a multiple of four (and level i
      holds elements) -- no other Resolve runs;
    * before every Resolve(i) Algorithm 1's preconditions hold: |S_i| <= d 4^i,
      |B_i| >= d 4^i if i < l, |S_i+1| <= d 4^(i+1) - d 4^i, and
      |B_i+1| >= d 4^(i+1) + d 4^i if i+1 < l (l = deepest non-empty level);
    * after it the postconditions hold: S_i empty, and |B_i| = 2d 4^i if i < l;
    * the k-th Resolve(i) comes after the 4k-th Resolve(i-1)."""
    d = [1, 2, 4, 8][seed % 4]
    cap = 4000
    h = HostHeap(cap, d, 0)
    o = oracle.PQ(cap)
    counts = {}
    for op in _pure_script(400, d, cap, 100 + seed):
        _apply(h, o, op)
        log = h.resolve_log()
        assert log and log[0]["lvl"] == 0 and log[0]["after"] == 0, "the operation's first Resolve is Resolve(0)"
        expect_next = 0
        for j in range(0, len(log), 2):
            b, a = log[j], log[j + 1]
            i = b["lvl"]
            assert a["lvl"] == i and b["after"] == 0 and a["after"] == 1
            assert i == expect_next, f"Resolve({i}) out of Theorem 1's order"
            ell, nom = b["ell"], d * 4 ** i
            # preconditions
            assert b["nS"] <= nom
            if i < ell:
                assert b["nB"] >= nom
            assert b["nS1"] <= 4 * nom - nom
            if i + 1 < ell:
                assert b["nB1"] >= 4 * nom + nom
            # postconditions
            assert a["nS"] == 0
            if i < a["ell"]:
                assert a["nB"] == 2 * nom
            counts[i] = a["cnt"]
            if i >= 1:
                assert counts[i] * 4 <= counts[i - 1]
            # Theorem 1: the next Resolve is of level i+1 iff Resolve(i)'s count
            # is now a multiple of four and level i+1 holds elements
            expect_next = i + 1 if (a["cnt"] % 4 == 0 and i + 1 <= a["ell"] and i + 1 < a["q"]) else None
        assert expect_next is None, "a Resolve that Theorem 1's rule asks for did not run"
        check_structure(h, o.cur(), d)


@pytest.mark.parametrize("seed", range(8))
def test_algorithm1_postconditions_with_duplicates_and_deletes(seed):
    """Outside Theorem 1's setting (decrease-keys that leave stale copies,
    deletes, extracts of up to 4d, both schedules) the schedule adds Resolves
    (room-making, refills of an empty B_0) and copies are dropped when they
    meet, so |B_i| can end below 2d 4^i; what still holds after every
    Resolve(i): S_i is empty and |B_i| <= 2d 4^i (EMPTY runs whenever B_i is
    above it, which a FILL of level i-1 can cause by keeping the elements of
    S_i at or below p_i)."""
    d = [1, 3, 8][seed % 3]
    cap = [50, 600][seed % 2]
    h = HostHeap(cap, d, seed % 2)
    o = oracle.PQ(cap)
    above = 0
    for op in W.random_script(80, cap, 3 * d, [20, 10 ** 6][seed % 2], 1300 + seed, deletes=True):
        if op[0] == "extract":
            op = ("extract", min(op[1], 4 * d))
        _apply(h, o, op)
        for r in h.resolve_log():
            if r["after"]:
                assert r["nS"] == 0 and r["nB"] <= 2 * d * 4 ** r["lvl"]
            else:
                above += r["nB"] > 2 * d * 4 ** r["lvl"]
        check_structure(h, o.cur(), d)
    print(f"Resolves entered with B_i above its nominal size: {above}")


# ------------------------------------------------------------ deep-level service
# Levels >= max(deep_lim, 2, qlds) resolved by their own workers (Section
# 2.2.1, Theorem 1), with the workers simulated on the CPU: lazy (a worker
# runs only when a team waits for it), eager (as soon as it is asked) and
# seeded random interleavings of whole Resolves.


def _deep_graphs():
    yield W.grid8(40, 40, wmax=10000, seed=4)
    yield W.random_graph(3000, 30000, 0, 9, seed=4)
    yield W.rgg(1500, seed=6)
    yield W.paper_dag(200, 6000, seed=7)
    yield W.shuffle_rows(W.grid8(30, 30, wmax=10000, seed=9), 1)
    yield W.grid8(96, 96, wmax=10000, seed=9)   # dead copies: refills of B_0 from the worker levels


@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("rule", ["plain", "plain_d4x", "fixed8", "random_k"])
def test_deep_workers_exact_and_ordered(gi, mode, rule):
    """With deep-level workers the distances equal the oracle's for every
    interleaving, after every operation the level order of Section 2.2 holds
    over the round loop's and the workers' levels together (B_i <= p_i < every
    deeper element) and the smallest live element is in B_0; the plain rule
    keeps one round per settled vertex and one relaxation per out-edge."""
    g = list(_deep_graphs())[gi]
    src = (gi * 11) % g.n
    ref, order, nrelax = oracle.dijkstra(g, src, want_order=True)
    kw = dict(check_live=True, deep_lim=2, deep_mode=mode, deep_seed=gi * 3 + mode)
    if rule == "plain_d4x":
        kw["d"] = 4 * max(1, g.max_degree())
    elif rule == "fixed8":
        kw.update(rule=1, kfix=8)
    elif rule == "random_k":
        kw.update(rule=3, kseq=np.random.default_rng(gi).integers(1, 64, size=61), kmax=256)
    rc, dist, st = hm_sssp(g, src, **kw)
    assert rc == 0
    assert st["first_bad"] == -1, st["violation"]
    assert np.array_equal(dist, ref)
    if rule.startswith("plain"):
        assert st["rounds"] == order.shape[0] and st["relax"] == nrelax
    else:
        assert st["extracted"] >= order.shape[0]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_deep_workers_take_the_deep_levels(mode):
    """The workers run the Resolves of their levels (all but the few the
    round loop runs itself while refilling an empty B_0 with every worker
    idle), and Theorem 1's pacing holds between the levels (Resolve(i+1) is
    asked for after every fourth Resolve(i), so cnt(i+1) <= cnt(i) / 4 +
    extra room-making ones, which stay rare here)."""
    g = W.grid8(64, 64, wmax=10000, seed=4)
    ref = oracle.dijkstra(g, 0)
    rc, dist, st = hm_sssp(g, 0, d=8, deep_lim=2, deep_mode=mode, deep_seed=5, check_live=True)
    assert rc == 0 and np.array_equal(dist, ref) and st["first_bad"] == -1
    res = st["resolves"][:st["levels"]]
    assert st["deep_lim"] == 2 and 0.9 * sum(res[2:]) <= st["worker_runs"] <= sum(res[2:])
    for i in range(1, len(res) - 1):
        assert res[i + 1] <= res[i] // 4 + 2, res


def test_deep_workers_off_past_the_deepest_level_and_lds_levels():
    """deep_lim at or past the deepest level means no workers; the first
    worker level is never above the LDS levels."""
    g = W.grid4(20, 20, 1, 100, seed=3)
    rc, dist, st = hm_sssp(g, 0, deep_lim=15)
    assert rc == 0 and st["deep_lim"] == 0 and st["worker_runs"] == 0
    rc, dist, st = hm_sssp(g, 0, d=4, qlds=3, deep_lim=2)
    assert rc == 0 and np.array_equal(dist, oracle.dijkstra(g, 0))
    assert st["deep_lim"] in (0, 3)
