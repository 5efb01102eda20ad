"""GPU parity of the parallel bucket heap (pbh_* through the C ABI) with the
sorted-multiset oracle: every extracted (key, id) sequence bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_1908_09378_amd as pkg
import workloads as W
from gpu_util import DEV, dev32, dev64, host32, host64

pytestmark = pytest.mark.gpu
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def _script(cap, d, ops, engine=pkg.ENGINE_AUTO, schedule=0):
    h = pkg.Heap(cap, d, engine, schedule)
    o = oracle.PQ(cap)
    kmax = max([op[1] for op in ops if op[0] == "extract"] + [1])
    ko = torch.empty(kmax, dtype=torch.int64, device=DEV)
    io = torch.empty(kmax, dtype=torch.int32, device=DEV)
    for op in ops:
        if op[0] == "update":
            h.bulk_update(dev64(op[1]), dev32(op[2]))
            o.bulk_update(op[1], op[2])
        elif op[0] == "delete":
            h.delete(dev32(op[1]))
            o.delete(op[1])
        else:
            n = h.extract_min(op[1], ko, io)
            ek, ei = o.extract_min(op[1])
            assert n == ek.shape[0]
            assert np.array_equal(host64(ko[:n]), ek) and np.array_equal(host32(io[:n]), ei)
        assert h.size() == o.size()
    return h


@pytest.mark.parametrize("seed", range(10))
def test_random_scripts(seed):
    d = [1, 3, 8, 32, 100][seed % 5]
    cap = [7, 100, 2000][seed % 3]
    print(f"[heap] script seed={seed} d={d} cap={cap}", flush=True)
    _script(cap, d, W.random_script(50, cap, [d, 4 * d][seed % 2], [5, 10 ** 12][seed % 2], 900 + seed))


@pytest.mark.parametrize("engine", [pkg.ENGINE_TEAM, pkg.ENGINE_WIDE])
@pytest.mark.parametrize("seed", range(8))
def test_random_scripts_with_deletes(engine, seed):
    """pbh_delete (Section 1.2) mixed with bulk updates and batched extracts,
    on both engines: every extract sequence and size equals the oracle's."""
    d = [1, 3, 8, 32][seed % 4]
    cap = [7, 100, 2000][seed % 3]
    print(f"[heap] delete script engine={engine} seed={seed} d={d} cap={cap}", flush=True)
    _script(cap, d, W.random_script(60, cap, [d, 4 * d][seed % 2], [5, 10 ** 12][seed % 2], 950 + seed,
                                    deletes=True), engine=engine, schedule=seed % 2)


@pytest.mark.parametrize("seed", range(2))
def test_wide_engine_deletes_multi_tile(seed):
    """Deletes of thousands of ids at once on the device-wide engine, with
    batches spanning many 2048-element tiles."""
    cap, d = 60000, 4096
    print(f"[heap] wide multi-tile deletes seed={seed}", flush=True)
    h = _script(cap, d, W.random_script(30, cap, 3 * d, [1 << 40, 3000][seed], 60 + seed, deletes=True),
                engine=pkg.ENGINE_WIDE, schedule=seed)
    _check_levels(h, d)


def test_delete_worked_example():
    import json, os
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pq_delete_worked_example.json")))
    for engine in (pkg.ENGINE_TEAM, pkg.ENGINE_WIDE):
        h = pkg.Heap(ex["id_capacity"], 2, engine)
        ko = torch.empty(8, dtype=torch.int64, device=DEV)
        io = torch.empty(8, dtype=torch.int32, device=DEV)
        for st in ex["steps"]:
            if st["op"] == "update":
                p = np.array(st["pairs"], dtype=np.uint64).reshape(-1, 2)
                h.bulk_update(dev64(p[:, 0]), dev32(p[:, 1].astype(np.uint32)))
            elif st["op"] == "delete":
                before = h.size()
                h.delete(dev32(np.array(st["ids"], np.uint32)))
                assert before - h.size() == st["removed"]
            else:
                n = h.extract_min(st["k"], ko, io)
                got = [[int(a), int(b)] for a, b in zip(host64(ko[:n]), host32(io[:n]))]
                assert got == st["expect"]
        h.close()


def test_invalid_delete_changes_nothing():
    for engine in (pkg.ENGINE_TEAM, pkg.ENGINE_WIDE):
        h = pkg.Heap(10, 2, engine)
        h.bulk_update(dev64(np.array([5, 6], np.uint64)), dev32(np.array([3, 4], np.uint32)))
        with pytest.raises(pkg.PBHError) as e:
            h.delete(dev32(np.array([3, 10], np.uint32)))
        assert e.value.code == pkg.PBH_EINVAL
        assert h.size() == 2
        ko = torch.empty(5, dtype=torch.int64, device=DEV)
        io = torch.empty(5, dtype=torch.int32, device=DEV)
        assert h.extract_min(5, ko, io) == 2
        h.close()


def test_worked_example():
    import json, os
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pq_worked_example.json")))
    ops = []
    for st in ex["steps"]:
        if st["op"] == "update":
            p = np.array(st["pairs"], dtype=np.uint64).reshape(-1, 2)
            ops.append(("update", p[:, 0].copy(), p[:, 1].astype(np.uint32)))
        else:
            ops.append(("extract", st["k"]))
    _script(ex["id_capacity"], 2, ops)


@pytest.mark.parametrize("seed", range(10))
def test_random_scripts_wide_engine(seed):
    """The device-wide engine on the same scripts (tiny d: single-tile steps)."""
    d = [1, 3, 8, 32, 100][seed % 5]
    cap = [7, 100, 2000][seed % 3]
    print(f"[heap] wide script seed={seed} d={d} cap={cap}", flush=True)
    _script(cap, d, W.random_script(50, cap, [d, 4 * d][seed % 2], [5, 10 ** 12][seed % 2], 900 + seed),
            engine=pkg.ENGINE_WIDE, schedule=seed % 2)


def _check_levels(h, d):
    L = h.debug_levels()
    assert L["nS"][0] == 0
    for i in range(L["q"]):
        assert L["nB"][i] <= 4 * d * 4 ** i and L["nS"][i] <= 2 * d * 4 ** i
    ps = [(int(L["pk"][i]), int(L["pv"][i])) for i in range(max(L["ell"], 0))]
    assert ps == sorted(ps)


@pytest.mark.parametrize("seed", range(4))
def test_wide_engine_multi_tile(seed):
    """Sizes that span many 2048-element tiles: merges across tile edges,
    radix Select passes over more than 4096 candidates, and several merge
    passes when sorting the extracted minima."""
    cap, d = 60000, [4096, 5000][seed % 2]
    keymax = [1 << 40, 3000, 1 << 63][seed % 3]
    print(f"[heap] wide multi-tile seed={seed} d={d} keymax={keymax}", flush=True)
    h = _script(cap, d, W.random_script(24, cap, 3 * d, keymax, 40 + seed), engine=pkg.ENGINE_WIDE,
                schedule=seed % 2)
    _check_levels(h, d)


@pytest.mark.parametrize("seed", range(3))
def test_wide_engine_duplicate_heavy(seed):
    """Batches of 3d pairs over fewer ids than that (every id several times
    in a batch), few distinct keys (ties decided by id), and extractions in
    between that leave stale copies in deeper levels: the merges' duplicate
    deletion across tile edges, with and without a live copy."""
    cap, d = [3000, 5000, 9000][seed], 2048
    print(f"[heap] wide duplicate-heavy seed={seed} cap={cap}", flush=True)
    h = _script(cap, d, W.random_script(30, cap, 3 * d, [100, 7, 1 << 20][seed], 70 + seed), engine=pkg.ENGINE_WIDE,
                schedule=seed % 2)
    _check_levels(h, d)


def test_merge_profiling_switch():
    """pbh_set_profiling: merge writing passes are timed only while it is
    on, and the results are the same either way."""
    cap, d = 60000, 4096
    ops = W.random_script(12, cap, 3 * d, 1 << 40, 123)
    h = pkg.Heap(cap, d, pkg.ENGINE_WIDE)
    o = oracle.PQ(cap)
    kmax = max([op[1] for op in ops if op[0] == "extract"] + [1])
    ko = torch.empty(kmax, dtype=torch.int64, device=DEV)
    io = torch.empty(kmax, dtype=torch.int32, device=DEV)
    seen = []
    for j, op in enumerate(ops):
        h.set_profiling(j % 2 == 1)
        before = h.merge_profile()
        if op[0] == "update":
            h.bulk_update(dev64(op[1]), dev32(op[2]))
            o.bulk_update(op[1], op[2])
        else:
            n = h.extract_min(op[1], ko, io)
            ek, ei = o.extract_min(op[1])
            assert np.array_equal(host64(ko[:n]), ek) and np.array_equal(host32(io[:n]), ei)
        after = h.merge_profile()
        grew = after["launches"] - before["launches"]
        if j % 2 == 0:
            assert grew == 0 and after["ms"] == before["ms"] and after["bytes"] == before["bytes"]
        else:
            seen.append(grew)
            assert (grew == 0) == (after["ms"] == before["ms"])
            if grew:
                assert after["bytes"] > before["bytes"]
    assert sum(seen) > 0
    assert h.size() == o.size()


def test_invariants_after_ops():
    h = _script(500, 4, W.random_script(40, 500, 30, 1000, 77))
    L = h.debug_levels()
    assert L["nS"][0] == 0
    for i in range(L["q"]):
        assert L["nB"][i] <= 4 * 4 * 4 ** i and L["nS"][i] <= 2 * 4 * 4 ** i


def _decrease_key_workload(n_ids, d, rounds, ext, engine, seed=3):
    keys, ids = W.heap_init_pairs(n_ids, seed=seed)
    h = pkg.Heap(n_ids, d, engine)
    o = oracle.PQArrays(n_ids)
    for c in range(0, n_ids, d):
        h.bulk_update(dev64(keys[c:c + d]), dev32(ids[c:c + d]))
    o.bulk_update(keys, ids)
    ko = torch.empty(ext, dtype=torch.int64, device=DEV)
    io = torch.empty(ext, dtype=torch.int32, device=DEV)
    for r in range(rounds):
        live = np.nonzero(o.cur != INF)[0].astype(np.uint32)
        bk, bi = W.decrease_batch(live, lambda x: o.cur[x], d, seed, r)
        h.bulk_update(dev64(bk), dev32(bi))
        o.bulk_update(bk, bi)
        n = h.extract_min(ext, ko, io)
        ek, ei = o.extract_min(ext)
        assert n == ext
        assert np.array_equal(host64(ko[:n]), ek) and np.array_equal(host32(io[:n]), ei)
    assert h.size() == o.size()
    _check_levels(h, d)
    return h


@pytest.mark.parametrize("engine", [pkg.ENGINE_TEAM, pkg.ENGINE_WIDE])
def test_decrease_key_workload_reduced(engine):
    """The standalone-heap workload at reduced scale: 2^18 ids loaded in pieces
    of d = 2^14, then rounds of 2^14 decrease-keys on live ids (new = old -
    uniform[0, old/2]) and extracts of 2^10."""
    print(f"[heap] reduced workload engine={engine}", flush=True)
    _decrease_key_workload(1 << 18, 1 << 14, 16, 1 << 10, engine)


def test_decrease_key_workload_full_size():
    """The standalone-heap workload at its full sizes (2^24 ids with keys in
    [0, 2^40), d = 2^20, rounds of 2^20 decrease-keys and extracts of 2^16),
    8 rounds, every extracted pair checked against the oracle."""
    print("[heap] full-size workload, 8 rounds", flush=True)
    _decrease_key_workload(1 << 24, 1 << 20, 8, 1 << 16, pkg.ENGINE_AUTO, seed=5)


def test_invalid_updates_change_nothing():
    h = pkg.Heap(10, 2)
    h.bulk_update(dev64(np.array([5], np.uint64)), dev32(np.array([3], np.uint32)))
    with pytest.raises(pkg.PBHError) as e:
        h.bulk_update(dev64(np.array([1, 2], np.uint64)), dev32(np.array([1, 10], np.uint32)))
    assert e.value.code == pkg.PBH_EINVAL
    with pytest.raises(pkg.PBHError):
        h.bulk_update(dev64(np.array([INF], np.uint64)), dev32(np.array([1], np.uint32)))
    ko = torch.empty(5, dtype=torch.int64, device=DEV)
    io = torch.empty(5, dtype=torch.int32, device=DEV)
    assert h.extract_min(5, ko, io) == 1
    assert host64(ko[:1])[0] == 5 and host32(io[:1])[0] == 3
    assert h.extract_min(5, ko, io) == 0
