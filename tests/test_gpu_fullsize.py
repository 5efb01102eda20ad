"""GPU parity at the full sizes of the benchmark's configurations, in the
settings the benchmark times them with:

* the standalone heap: all 256 rounds of 2^20 decrease-keys + extract_min(2^16)
  on 2^24 ids, every extracted (key, id) compared with the oracle, down to the
  drained heap;
* the 8-neighbour grid 2048x2048 (w log-uniform in [1, 10^4]): the learned
  threshold at the autotuned settings (d = 1024, 256 threads, k_max 256; with
  and without deep-level workers) and at d = 8, every distance compared, and
  the first 2^18 rounds of plain parDijkstra (settle order and settled
  distances);
* the 256-query batch over 64 random geometric graphs: learned (autotuned) and
  plain, every query's distances compared;
* the heap engines' level states after every operation equal the CPU model's,
  whose Resolve schedule is pinned to Theorem 1 (tests/test_hostmodel.py)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1908_09378_amd as pkg
import workloads as W
from gpu_util import DEV, dev32, dev64, graph_to_dev, host32, host64, run_sssp

pytestmark = pytest.mark.gpu
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.mark.timeout(900)
def test_heap_all_256_rounds_full_size():
    n_ids, d, ext, rounds = 1 << 24, 1 << 20, 1 << 16, 256
    keys, ids = W.heap_init_pairs(n_ids, seed=3)
    h = pkg.Heap(n_ids, d)
    o = oracle.PQArrays(n_ids)
    for c in range(0, n_ids, d):
        h.bulk_update(dev64(keys[c:c + d]), dev32(ids[c:c + d]))
    o.bulk_update(keys, ids)
    ko = torch.empty(ext, dtype=torch.int64, device=DEV)
    io = torch.empty(ext, dtype=torch.int32, device=DEV)
    for r in range(rounds):
        if r % 32 == 0:
            print(f"[full] heap round {r}", flush=True)
        live = np.nonzero(o.cur != INF)[0].astype(np.uint32)
        bk, bi = W.decrease_batch(live, lambda x: o.cur[x], d, 3, r)
        h.bulk_update(dev64(bk), dev32(bi))
        o.bulk_update(bk, bi)
        n = h.extract_min(ext, ko, io)
        ek, ei = o.extract_min(ext)
        assert n == ek.shape[0] == ext
        assert np.array_equal(host64(ko[:n]), ek) and np.array_equal(host32(io[:n]), ei), f"round {r}"
        assert h.size() == o.size()
    assert h.size() == 0                       # 256 x 2^16 = 2^24: the heap drains at the last round
    assert h.extract_min(ext, ko, io) == 0


@pytest.fixture(scope="module")
def grid8_full():
    g = W.grid8(2048, 2048, wmax=10000, seed=4)
    return g, oracle.dijkstra(g, 0), graph_to_dev(g)


def _run_dev(gd, g, **kw):
    off, tg, wt = gd
    dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
    st = pkg.sssp_ex(off, tg, wt, g.n, g.m, 0, dist, **kw)
    return host64(dist), st


GRID8_TUNED = dict(d=1024, team=256, k_max=256)


@pytest.mark.parametrize("kw", [GRID8_TUNED, dict(d=8)], ids=["tuned", "d8"])
def test_grid8_2048_learned(grid8_full, kw):
    from paper_1908_09378_amd import learn
    g, ref, gd = grid8_full
    blob = torch.from_numpy(learn.load_model()).to(DEV)
    print(f"[full] grid8 2048^2 learned {kw}", flush=True)
    got, st = _run_dev(gd, g, k_rule=2, k_model=blob, **kw)
    print(f"[full]   {st['kernel_ms']:.0f} ms, {st['rounds']} rounds, {st['extracted']} extracted", flush=True)
    assert np.array_equal(got, ref), f"{int((got != ref).sum())} distances differ"
    assert st["extracted"] >= g.n


def test_grid8_2048_learned_deep_workers(grid8_full):
    """The learned threshold at the tuned settings with deep-level workers
    (levels >= 2 resolved by workgroups of their own)."""
    from paper_1908_09378_amd import learn
    g, ref, gd = grid8_full
    blob = torch.from_numpy(learn.load_model()).to(DEV)
    print("[full] grid8 2048^2 learned, deep-level workers", flush=True)
    got, st = _run_dev(gd, g, k_rule=2, k_model=blob, deep_level=2, **GRID8_TUNED)
    print(f"[full]   {st['kernel_ms']:.0f} ms, {st['rounds']} rounds, resolves {st['resolves'][:st['levels']]}",
          flush=True)
    assert np.array_equal(got, ref), f"{int((got != ref).sum())} distances differ"


def test_grid8_2048_plain_first_rounds(grid8_full):
    """Plain parDijkstra on the full grid at the bench's settings (d = 2048,
    256 threads, deep-level workers): its whole run takes many minutes, so
    the test stops after 2^18 rounds and checks what they settled: the extraction
    sequence is the oracle's settle order and those vertices have their final
    distances."""
    g, ref, gd = grid8_full
    _, order, _ = oracle.dijkstra(g, 0, want_order=True)
    R = 1 << 18
    rec = torch.full((R + 8,), -1, dtype=torch.int32, device=DEV)
    print("[full] grid8 2048^2 plain, first 2^18 rounds", flush=True)
    got, st = _run_dev(gd, g, d=2048, team=256, deep_level=2, max_rounds=R, settle_order=rec)
    print(f"[full]   {st['kernel_ms']:.0f} ms, {st['rounds']} rounds", flush=True)
    assert st["rounds"] == R
    seq = host32(rec)[:R]
    assert np.array_equal(seq, order[:R])
    assert np.array_equal(got[seq], ref[seq])


def test_rgg_batch_256_queries_full_size():
    from paper_1908_09378_amd import learn
    batch = W.rgg_batch(64, 4)
    qs, refs, keep = [], [], []
    for g, srcs in batch:
        off, tg, wt = graph_to_dev(g)
        keep.append((off, tg, wt))
        for s in srcs:
            qs.append((off, tg, wt, g.n, g.m, s, torch.empty(g.n, dtype=torch.int64, device=DEV)))
            refs.append(oracle.dijkstra(g, s))
    assert len(qs) == 256
    blob = torch.from_numpy(learn.load_model()).to(DEV)
    print("[full] batch autotune", flush=True)
    t = pkg.sssp_batch_autotune(qs, k_rule=2, k_model=blob)
    for kw in (dict(k_rule=2, k_model=blob, d_scale=t["d_scale"], k_max=t["k_max"], team=t["team"]), dict()):
        for q in qs:
            q[6].fill_(0)
        print(f"[full] batch {'learned ' + str(t) if kw else 'plain'}", flush=True)
        st = pkg.sssp_batch(qs, **kw)
        bad = [i for i, (q, r) in enumerate(zip(qs, refs)) if not np.array_equal(host64(q[6]), r)]
        assert not bad, f"queries {bad[:8]} differ"
        if not kw:
            assert st["rounds"] == sum(int(np.count_nonzero(r != INF)) for r in refs)


@pytest.mark.parametrize("engine", [pkg.ENGINE_TEAM, pkg.ENGINE_WIDE])
@pytest.mark.parametrize("d", [1, 4, 8])
def test_engine_states_follow_the_theorem1_schedule(engine, d):
    """Operations of at most d elements (Theorem 1's setting): after every
    operation each engine's level sizes, pivots and Resolve counts equal the
    CPU model's, whose every Resolve is checked against Theorem 1 and
    Algorithm 1 in tests/test_hostmodel.py."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from hostmodel import HostHeap
    from test_hostmodel import _pure_script
    cap = 3000
    h = pkg.Heap(cap, d, engine, 0)
    m = HostHeap(cap, d, 0)
    ko = torch.empty(d, dtype=torch.int64, device=DEV)
    io = torch.empty(d, dtype=torch.int32, device=DEV)
    print(f"[full] engine {engine} states d={d}", flush=True)
    for j, op in enumerate(_pure_script(300, d, cap, 40 + d)):
        if op[0] == "update":
            h.bulk_update(dev64(op[1]), dev32(op[2]))
            m.bulk_update(op[1], op[2])
        else:
            n = h.extract_min(op[1], ko, io)
            mk, mv = m.extract_min(op[1])
            assert np.array_equal(host64(ko[:n]), mk) and np.array_equal(host32(io[:n]), mv)
        G, M = h.debug_levels(), m.levels()
        q = min(G["q"], M["q"])
        assert G["ell"] == M["ell"], j
        for f, gf in (("nB", "nB"), ("nS", "nS"), ("pk", "pk"), ("pv", "pv"), ("cnt", "resolves")):
            assert np.array_equal(np.asarray(G[gf][:q], np.uint64), np.asarray(M[f][:q], np.uint64)), (j, f)
    h.close()


def test_paper_dag_m4e7_closed_form():
    """The paper's DAG at n = 30,000 and m = 4e7 (Section 4.2): parDijkstra's
    distances equal the closed form dist(i) = i, one round per vertex."""
    g = W.paper_dag(30000, 40_000_000, seed=11)
    print("[full] paper DAG m=4e7", flush=True)
    got, st = run_sssp(pkg, g, 0, team=1024)
    assert np.array_equal(got, np.arange(g.n, dtype=np.uint64))
    assert st["rounds"] == g.n and st["relaxations"] == g.m
