"""GPU parity of the deep-level workers (sssp_opts.deep_level; Section 2.2.1,
Theorem 1, Section 4.1's block per level): levels from the first worker level
down each have a workgroup of their own, launched cooperatively with the round
loop.  Distances bit-exact against the oracle for every rule; the plain rule
keeps the oracle's settle order, one round per settled vertex and one
relaxation per out-edge; the worker levels' Resolves are done by the workers;
a level overflow found by a worker is retried with more levels; the
no-allocation entry point runs them from its fixed scratch."""
import numpy as np
import pytest
import torch

import oracle
import paper_1908_09378_amd as pkg
import workloads as W
from gpu_util import DEV, dev32, graph_to_dev, host64, run_sssp

pytestmark = pytest.mark.gpu
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def _graphs():
    return {
        "grid8_96": W.grid8(96, 96, wmax=10000, seed=9),        # dead copies: refills from the worker levels
        "grid4_64": W.grid4(64, 64, 1, 100, seed=1),
        "rgg_2e14": W.rgg(1 << 14, seed=6),
        "random_multi": W.random_graph(5000, 60000, 0, 9, seed=4),
        "dag": W.paper_dag(400, 40000, seed=7),
        "shuffled_grid8": W.shuffle_rows(W.grid8(80, 80, wmax=10000, seed=3), 1),
    }


GRAPHS = _graphs()


@pytest.mark.parametrize("gname", sorted(GRAPHS))
@pytest.mark.parametrize("kw", [dict(), dict(d_scale=8), dict(team=256, d_scale=32), dict(k_rule=1, k_fixed=8),
                                dict(k_rule=3, k_max=256)],
                         ids=["plain", "plain_d8x", "plain_t256_d32x", "fixed8", "seq"])
@pytest.mark.parametrize("deep", [2, 3])
def test_deep_workers_exact(gname, kw, deep):
    g = GRAPHS[gname]
    src = 3 % g.n
    ref, order, nrelax = oracle.dijkstra(g, src, want_order=True)
    kk = dict(kw)
    if kk.get("k_rule") == 3:
        kk["k_seq"] = dev32(np.array([1, 33, 2, 250, 5, 1, 64], np.uint32))
    print(f"[deep] {gname} {kw} deep_level={deep}", flush=True)
    got, st = run_sssp(pkg, g, src, deep_level=deep, **kk)
    assert np.array_equal(got, ref), f"{int((got != ref).sum())} distances differ"
    if "k_rule" not in kw:
        assert st["rounds"] == order.shape[0] and st["relaxations"] == nrelax
    else:
        assert st["extracted"] >= order.shape[0]


@pytest.mark.parametrize("gname", ["grid8_96", "rgg_2e14"])
def test_deep_workers_plain_settle_order(gname):
    """With workers the plain rule still extracts the heap's minimum every
    round: the whole extraction sequence is the oracle's settle order."""
    g = GRAPHS[gname]
    ref, order, _ = oracle.dijkstra(g, 0, want_order=True)
    for kw in (dict(deep_level=2), dict(deep_level=2, d_scale=16, team=256)):
        rec = torch.full((g.n + 8,), -1, dtype=torch.int32, device=DEV)
        print(f"[deep] settle order {gname} {kw}", flush=True)
        got, st = run_sssp(pkg, g, 0, settle_order=rec, **kw)
        seq = rec.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref)
        assert np.array_equal(seq[:order.shape[0]], order)


def test_deep_workers_run_the_deep_levels_and_profile():
    """The worker levels' Resolves happen (their counts are positive), and
    with time accounting each worker level reports its busy time."""
    from paper_1908_09378_amd import learn
    g = W.grid8(256, 256, wmax=10000, seed=4)
    ref = oracle.dijkstra(g, 0)
    blob = torch.from_numpy(learn.load_model()).to(DEV)
    for kw in (dict(d=8), dict(k_rule=2, k_model=blob, d=256, team=256, k_max=256)):
        print(f"[deep] worker levels {kw}", flush=True)
        got0, s0 = run_sssp(pkg, g, 0, **kw)
        got, st = run_sssp(pkg, g, 0, deep_level=2, profile=1, **kw)
        assert np.array_equal(got, ref) and np.array_equal(got0, ref)
        assert st["levels"] > 3 and st["resolves"][2] > 0
        assert all(st["level_us"][i] > 0 for i in range(2, st["levels"]) if st["resolves"][i] > 0)
        assert st["phase_us"]["wait"] >= 0
        print(f"[deep]   {s0['kernel_ms']:.1f} ms without workers, {st['kernel_ms']:.1f} ms with "
              f"(profiled); resolves {st['resolves'][:st['levels']]}", flush=True)


def test_deep_workers_capacity_retry():
    """A tiny heap capacity: the deepest worker finds its level overflowing,
    the run is repeated with more levels (and so more workers) until it fits."""
    g = W.grid8(64, 64, wmax=10000, seed=2)
    ref = oracle.dijkstra(g, 0)
    print("[deep] capacity retry", flush=True)
    got, st = run_sssp(pkg, g, 0, deep_level=2, heap_capacity=64, d=8)
    assert np.array_equal(got, ref)
    assert st["levels"] >= 3


def test_deep_workers_need_schedule_0():
    g = W.grid4(8, 8)
    with pytest.raises(pkg.PBHError) as e:
        run_sssp(pkg, g, 0, deep_level=2, schedule=1)
    assert e.value.code == pkg.PBH_EINVAL


def test_deep_workers_noalloc_twice_second_smaller():
    """sssp_noalloc with workers (their control block in the fixed scratch)
    equals sssp_ex with them, twice in a row, the second query smaller."""
    for g, src in ((W.grid8(64, 64, wmax=10000, seed=5), 0), (W.grid4(30, 31, 1, 100, seed=2), 7)):
        off, tg, wt = graph_to_dev(g)
        d1 = torch.empty(g.n, dtype=torch.int64, device=DEV)
        d2 = torch.full((g.n,), 5, dtype=torch.int64, device=DEV)
        print(f"[deep] noalloc n={g.n}", flush=True)
        s1 = pkg.sssp_ex(off, tg, wt, g.n, g.m, src, d1, deep_level=2, d=8)
        s2 = pkg.sssp_noalloc(off, tg, wt, g.n, g.m, src, d2, deep_level=2, d=8)
        ref = oracle.dijkstra(g, src)
        assert np.array_equal(host64(d1), ref) and np.array_equal(host64(d2), ref)
        for k in ("rounds", "relaxations", "levels"):
            assert s1[k] == s2[k]
