"""GPU parity of parDijkstra (sssp through the C ABI) with the oracle:
distances bit-exact, element by element, and the plain-rule round and
relaxation counts (one round per settled vertex, every out-edge of a settled
vertex scanned once)."""
import numpy as np
import pytest

import oracle
import paper_1908_09378_amd as pkg
import workloads as W
from gpu_util import run_sssp

pytestmark = pytest.mark.gpu
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def _check(g, src, **kw):
    print(f"[sssp] {g.name} n={g.n} m={g.m} src={src} {kw}", flush=True)
    ref, order, nrelax = oracle.dijkstra(g, src, want_order=True)
    got, st = run_sssp(pkg, g, src, **kw)
    assert np.array_equal(got, ref), f"{int((got != ref).sum())} distances differ"
    if st is not None:
        assert st["rounds"] == order.shape[0]
        assert st["relaxations"] == nrelax
    return st


def test_grid_64x64_weights_1_100():
    _check(W.grid4(64, 64, 1, 100, seed=1), 0)


@pytest.mark.parametrize("team", [64, 256, 1024])
@pytest.mark.parametrize("schedule", [0, 1])
def test_grid_teams_and_schedules(team, schedule):
    _check(W.grid4(64, 64, 1, 100, seed=1), 0, team=team, schedule=schedule)


@pytest.mark.parametrize("lds", [0, 1, 2, 0xFFFFFFFF])
def test_ring_lds_levels(lds):
    _check(W.ring_lattice(1 << 12, 16, 1, 1000, seed=2), 5, lds_levels=lds)


def test_small_heap_capacity_retries_exactly():
    _check(W.ring_lattice(1 << 12, 16, 1, 1000, seed=2), 0, heap_capacity=64)


@pytest.mark.parametrize("seed", range(12))
def test_random_multigraphs_zero_weights_selfloops(seed):
    n = [1, 2, 17, 300, 1000, 5000][seed % 6]
    m = [0, 3, 50, 4000, 20000, 60000][seed % 6]
    wl, wh = [(0, 0), (0, 3), (1, 1000)][seed % 3]
    g = W.random_graph(n, m, wl, wh, 70 + seed)
    _check(g, seed % n, team=[64, 256, 1024][seed % 3])


def test_unreachable_and_isolated():
    g = W.path_graph(200, seed=3)
    _check(g, 100)   # vertices 0..99 unreachable


def test_grid8_loguniform():
    _check(W.grid8(128, 128, wmax=10000, seed=4), 0)


@pytest.mark.parametrize("kw", [dict(), dict(team=256), dict(lds_levels=0), dict(schedule=1),
                                dict(k_rule=1, k_fixed=16), dict(k_rule=1, k_fixed=1)])
def test_grid8_dead_copies_refill(kw):
    """Many dead copies collect in B_1 and B_2 on this graph, so refilling an
    empty B_0 takes repeated Resolve(0) calls."""
    g = W.grid8(96, 96, wmax=10000, seed=9)
    if "k_rule" not in kw:
        _check(g, 0, **kw)
        return
    print(f"[sssp] {g.name} {kw}", flush=True)
    got, _ = run_sssp(pkg, g, 0, **kw)
    assert np.array_equal(got, oracle.dijkstra(g, 0))


def test_unit_weights_many_ties():
    _check(W.grid4(100, 100, 1, 1, seed=5), 0)
    _check(W.ring_lattice(1 << 13, 16, 1, 1, seed=5), 0)


def test_rgg():
    _check(W.rgg(1 << 14, seed=6), 3)


def test_paper_dag_high_degree():
    n = 3000
    g = W.paper_dag(n, 400000, seed=7)
    st = _check(g, 0)


def test_ring_lattice_full_size():
    """The full-size ring lattice: n = 2^20, 16 neighbours per side,
    weights uniform in [1, 1000], source 0 -- every distance compared."""
    g = W.ring_lattice(1 << 20, 16, 1, 1000, seed=2)
    st = _check(g, 0, team=64)
    print(f"[sssp] ring 2^20: {st['kernel_ms']:.1f} ms, rounds {st['rounds']}", flush=True)


@pytest.mark.parametrize("gname", ["grid64", "ring2e16"])
def test_plain_settle_order_is_the_oracles(gname):
    """The plain rule extracts one vertex per round, always the heap's
    minimum (key, id): the whole extraction sequence equals the oracle's
    settle order, which is the reached vertices in (dist, id) order."""
    import torch
    g = W.grid4(64, 64, 1, 100, seed=1) if gname == "grid64" else W.ring_lattice(1 << 16, 16, 1, 1000, seed=2)
    ref, order, _ = oracle.dijkstra(g, 0, want_order=True)
    assert np.array_equal(order, np.lexsort((np.arange(g.n)[ref != INF], ref[ref != INF])))
    from gpu_util import DEV, dev32
    for kw in (dict(), dict(team=256), dict(lds_levels=0xFFFFFFFF, schedule=1)):
        rec = torch.full((g.n + 8,), -1, dtype=torch.int32, device=DEV)
        print(f"[sssp] settle order {gname} {kw}", flush=True)
        got, st = run_sssp(pkg, g, 0, settle_order=rec, **kw)
        seq = rec.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref)
        assert np.array_equal(seq[:order.shape[0]], order)
        assert np.all(seq[order.shape[0]:] == np.uint32(0xFFFFFFFF))


def test_speculative_extraction_record_covers_every_vertex():
    import torch
    from gpu_util import DEV
    g = W.grid8(64, 64, wmax=10000, seed=9)
    ref = oracle.dijkstra(g, 0)
    rec = torch.full((8 * g.n,), -1, dtype=torch.int32, device=DEV)
    print("[sssp] speculative extraction record", flush=True)
    got, st = run_sssp(pkg, g, 0, k_rule=1, k_fixed=16, k_max=16, settle_order=rec)
    seq = rec.cpu().numpy().view(np.uint32)[: st["extracted"]]
    assert np.array_equal(got, ref)
    assert st["extracted"] <= 8 * g.n
    assert np.array_equal(np.unique(seq), np.nonzero(ref != INF)[0].astype(np.uint32))


@pytest.mark.parametrize("kw", [dict(), dict(team=256), dict(k_rule=1, k_fixed=16),
                                dict(k_rule=3, k_max=256)])
def test_rows_not_sorted_by_target(kw):
    """CSR rows in random order (the ABI allows any order): the plain round's
    intake sorts the relaxation output by id, the speculative rounds' intake
    sorts their list; distances, rounds and relaxations stay the oracle's."""
    from gpu_util import dev32
    for g in (W.shuffle_rows(W.grid8(96, 96, wmax=10000, seed=9), 1),
              W.shuffle_rows(W.ring_lattice(1 << 13, 16, 1, 1000, seed=2), 2),
              W.shuffle_rows(W.random_graph(3000, 40000, 0, 9, seed=4), 3)):
        assert not all(np.all(np.diff(g.targets[g.offsets[u]:g.offsets[u + 1]].astype(np.int64)) >= 0)
                       for u in range(min(g.n, 50)))
        kk = dict(kw)
        if kk.get("k_rule") == 3:
            kk["k_seq"] = dev32(np.array([1, 17, 2, 250, 5, 1, 64], np.uint32))
        print(f"[sssp] shuffled rows {g.name} {kw}", flush=True)
        if "k_rule" in kk:
            got, st = run_sssp(pkg, g, 0, **kk)
            assert np.array_equal(got, oracle.dijkstra(g, 0))
        else:
            _check(g, 0, **kk)


def test_invalid_inputs():
    import torch
    from gpu_util import DEV, dev32, dev64
    g = W.grid4(4, 4)
    off, tg, wt = dev64(g.offsets), dev32(g.targets), dev32(g.weights)
    dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
    with pytest.raises(pkg.PBHError) as e:
        pkg.sssp(off, tg, wt, g.n, g.m, g.n, dist)
    assert e.value.code == pkg.PBH_EINVAL
    bad = g.targets.copy()
    bad[3] = 999
    with pytest.raises(pkg.PBHError) as e:
        pkg.sssp(off, dev32(bad), wt, g.n, g.m, 0, dist)
    assert e.value.code == pkg.PBH_EINVAL
    badoff = g.offsets.copy()
    badoff[2], badoff[3] = badoff[3], badoff[2]
    with pytest.raises(pkg.PBHError):
        pkg.sssp(dev64(badoff), tg, wt, g.n, g.m, 0, dist)


def _batch_check(graphs_sources, **kw):
    import torch
    from gpu_util import DEV, graph_to_dev, host64
    qs, refs, keep = [], [], []
    for g, srcs in graphs_sources:
        off, tg, wt = graph_to_dev(g)
        keep.append((off, tg, wt))
        for s in srcs:
            dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
            qs.append((off, tg, wt, g.n, g.m, s, dist))
            refs.append(oracle.dijkstra(g, s, want_order=True))
    print(f"[batch] {len(qs)} queries {kw}", flush=True)
    st = pkg.sssp_batch(qs, **kw)
    for q, (ref, order, nrelax) in zip(qs, refs):
        got = host64(q[6])
        assert np.array_equal(got, ref), f"{int((got != ref).sum())} distances differ"
    assert st["rounds"] == sum(r[1].shape[0] for r in refs)
    assert st["relaxations"] == sum(r[2] for r in refs)
    return st


def test_batch_mixed_graphs():
    gs = [(W.rgg(4096 + 1000 * i, seed=20 + i), [0, 7, 100 + i, 4095]) for i in range(6)]
    gs.append((W.grid4(64, 64, 1, 100, seed=1), [0, 4095]))
    gs.append((W.random_graph(300, 3000, 0, 5, seed=3), [0, 1, 2]))
    gs.append((W.path_graph(50, seed=2), [0, 49]))
    _batch_check(gs)


@pytest.mark.parametrize("kw", [dict(team=256), dict(lds_levels=0xFFFFFFFF), dict(schedule=1),
                                dict(heap_capacity=64)])
def test_batch_options(kw):
    gs = [(W.rgg(3000 + 500 * i, seed=40 + i), [0, 11]) for i in range(4)]
    gs.append((W.ring_lattice(2048, 16, 1, 1000, seed=5), [0, 1000]))
    _batch_check(gs, **kw)


def test_batch_many_queries_more_than_resident():
    g = W.grid4(16, 16, 1, 100, seed=9)
    _batch_check([(g, list(range(0, 256, 1)))] * 1 + [(W.rgg(2048, seed=8), list(range(0, 2048, 2)))])


@pytest.mark.parametrize("gname", ["grid", "ring", "rgg", "multi"])
@pytest.mark.parametrize("rule", ["fixed3", "fixed64", "seq"])
def test_speculative_rounds_exact(gname, rule):
    import torch
    from gpu_util import dev32
    g = {"grid": lambda: W.grid4(64, 64, 1, 100, seed=1), "ring": lambda: W.ring_lattice(1 << 13, 16, 1, 1000, seed=2),
         "rgg": lambda: W.rgg(1 << 13, seed=3), "multi": lambda: W.random_graph(2000, 20000, 0, 9, seed=4)}[gname]()
    kw = {"fixed3": dict(k_rule=1, k_fixed=3), "fixed64": dict(k_rule=1, k_fixed=64, k_max=64),
          "seq": dict(k_rule=3, k_seq=dev32(np.array([1, 17, 2, 250, 5, 1, 64], np.uint32)), k_max=256)}[rule]
    print(f"[spec] {g.name} {rule}", flush=True)
    ref, order, _ = oracle.dijkstra(g, 0, want_order=True)
    got, st = run_sssp(pkg, g, 0, **kw)
    assert np.array_equal(got, ref)
    assert st["extracted"] >= order.shape[0]


def test_batch_speculative_exact():
    import torch
    from gpu_util import DEV, graph_to_dev, host64
    gs = [(W.rgg(3000 + 700 * i, seed=60 + i), [0, 5]) for i in range(5)]
    qs, refs, keep = [], [], []
    for g, srcs in gs:
        off, tg, wt = graph_to_dev(g)
        keep.append((off, tg, wt))
        for s in srcs:
            qs.append((off, tg, wt, g.n, g.m, s, torch.empty(g.n, dtype=torch.int64, device=DEV)))
            refs.append(oracle.dijkstra(g, s))
    pkg.sssp_batch(qs, k_rule=1, k_fixed=8)
    for q, ref in zip(qs, refs):
        assert np.array_equal(host64(q[6]), ref)


def test_trial_limits_on_gpu():
    """max_rounds / stop_key: the autotuner's equal-work trials."""
    g = W.grid8(80, 80, wmax=10000, seed=12)
    ref = oracle.dijkstra(g, 0)
    print("[sssp] trial limits", flush=True)
    got, st = run_sssp(pkg, g, 0, max_rounds=700)
    assert st["rounds"] == 700 and st["last_key"] == int(np.sort(ref)[700])
    D = st["last_key"]
    for kw in (dict(), dict(k_rule=1, k_fixed=9), dict(k_rule=1, k_fixed=40, d=64)):
        got, st = run_sssp(pkg, g, 0, stop_key=D, **kw)
        settled = ref <= D
        assert np.array_equal(got[settled], ref[settled]) and st["last_key"] > D


@pytest.mark.parametrize("rule", [0, 1])
def test_autotune_then_exact(rule):
    from gpu_util import graph_to_dev, DEV, host64
    import torch
    g = W.ring_lattice(1 << 14, 16, 1, 1000, seed=5)
    off, tg, wt = graph_to_dev(g)
    dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
    kw = dict(k_rule=1, k_fixed=8) if rule else {}
    print(f"[sssp] autotune rule={rule}", flush=True)
    t = pkg.sssp_autotune(off, tg, wt, g.n, g.m, 0, dist, **kw)
    assert t["d"] % g.max_degree() == 0 and t["d"] >= g.max_degree()
    if rule:
        assert t["k_max"] in (1, 64, 256)
    kw.update(t)
    pkg.sssp_ex(off, tg, wt, g.n, g.m, 0, dist, **kw)
    assert np.array_equal(host64(dist), oracle.dijkstra(g, 0))


def test_batch_autotune_then_exact():
    import torch
    from gpu_util import DEV, graph_to_dev, host64
    gs = [(W.rgg(1500 + 900 * i, seed=80 + i), [0, 3]) for i in range(4)]
    qs, refs, keep = [], [], []
    for g, srcs in gs:
        off, tg, wt = graph_to_dev(g)
        keep.append((off, tg, wt))
        for s in srcs:
            qs.append((off, tg, wt, g.n, g.m, s, torch.empty(g.n, dtype=torch.int64, device=DEV)))
            refs.append(oracle.dijkstra(g, s))
    print("[sssp] batch autotune", flush=True)
    t = pkg.sssp_batch_autotune(qs, k_rule=1, k_fixed=6)
    assert t["d"] == 0 and t["d_scale"] >= 1
    pkg.sssp_batch(qs, k_rule=1, k_fixed=6, **t)
    for q, r in zip(qs, refs):
        assert np.array_equal(host64(q[6]), r)


def test_out_of_memory_reports_enomem_and_the_next_call_works():
    """A heap arena far beyond the GPU's memory: sssp_ex returns PBH_ENOMEM
    (nothing runs); the library keeps no half-made arena, so the next call,
    which needs a small one, allocates it and is exact."""
    g = W.grid4(32, 32, 1, 100, seed=3)
    ref = oracle.dijkstra(g, 0)
    print("[sssp] out of memory", flush=True)
    with pytest.raises(pkg.PBHError) as e:
        run_sssp(pkg, g, 0, d=4, heap_capacity=1 << 40)
    assert e.value.code == pkg.PBH_ENOMEM
    got, st = run_sssp(pkg, g, 0, d=4, heap_capacity=1 << 14)
    assert np.array_equal(got, ref)
    got, st = run_sssp(pkg, g, 0)
    assert np.array_equal(got, ref)
