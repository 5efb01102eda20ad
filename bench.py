"""Benchmark: parDijkstra on the parallel bucket heap, 1 MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ring|grid64|grid8|dag|multi|heap|copy]
                    [--method plain|learned|both]

One step = one complete sssp() over the resident graph (every round of the
hot path: the extraction threshold, extract-min, relaxation, bulk update,
Resolve schedule).  The
default workload is the large high-diameter ring lattice: n = 2^20 vertices,
each linked to its 16 nearest neighbours on each side (m = 33,554,432 directed
edges), integer weights uniform in [1, 1000], source 0.

Prints one JSON line: GTEPS = m / seconds per step, the roofline of the
round-loop kernel (algorithmic bytes per launch / its HIP-event duration vs
8 TB/s) and the CPU oracle (single-thread binary-heap Dijkstra) timed on a
bounded sample of the same workload.  With --method both (the default) the
value is the learned-threshold rule's and the line also carries plain
parDijkstra on the same graph ("plain") and the speedup; both runs' distances
are checked against the oracle.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSSP GTEPS (m/time) on 1 MI355X: learned-threshold & batched vs plain parDijkstra"
HBM_PEAK_GBS = 8000.0


def make_graph(name):
    import workloads as W
    if name == "ring":
        return W.ring_lattice(1 << 20, 16, 1, 1000, seed=2), "ring lattice n=2^20, 16 neighbours per side, w~U[1,1000], source 0"
    if name == "grid64":
        return W.grid4(64, 64, 1, 100, seed=1), "4-neighbour grid 64x64, w~U[1,100], source 0"
    if name == "grid8":
        return W.grid8(2048, 2048, wmax=10000, seed=4), "8-neighbour grid 2048x2048, w log-uniform [1,1e4], source 0"
    if name == "dag":
        return (W.paper_dag(30000, 40_000_000, seed=11),
                "the paper's high-diameter DAG: n=30000, chain of weight 1 plus random forward edges of weight "
                "2(v-u), m=4e7, source 0")
    raise SystemExit(f"unknown workload {name}")


def run_multi(args):
    """The batched workload: 256 queries (64 random geometric graphs with
    uneven n in 2^12..2^18, mean degree 24, 4 sources each) in one launch."""
    import numpy as np
    import torch

    import oracle
    import paper_1908_09378_amd as pkg
    import workloads as W

    batch = W.rgg_batch(64, 4)
    dev = torch.device("cuda:0")
    qs, keep = [], []
    for g, srcs in batch:
        off = torch.from_numpy(g.offsets.view(np.int64)).to(dev)
        tg = torch.from_numpy(g.targets.view(np.int32)).to(dev)
        wt = torch.from_numpy(g.weights.view(np.int32)).to(dev)
        keep.append((off, tg, wt))
        for s in srcs:
            qs.append((off, tg, wt, g.n, g.m, s, torch.empty(g.n, dtype=torch.int64, device=dev)))
    sum_m = sum(q[4] for q in qs)
    refs = [oracle.dijkstra(g, s) for g, srcs in batch for s in srcs]

    def timed(**kw):
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            pkg.sssp_batch(qs, **kw)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            stats.append(pkg.sssp_batch(qs, **kw))
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        exact = all(np.array_equal(q[6].cpu().numpy().view(np.uint64), r) for q, r in zip(qs, refs))
        st = stats[-1]
        kern_ms = sum(x["kernel_ms"] for x in stats) / len(stats)
        abytes = algorithmic_bytes(st)
        achieved = abytes / (kern_ms * 1e-3) / 1e9
        print(f"[bench] batch {kw.get('k_rule', 0)}: {sec * 1e3:.1f} ms/step exact={exact}", file=sys.stderr,
              flush=True)
        return {"value": sum_m / sec / 1e9, "ms_per_step": sec * 1e3, "rounds": st["rounds"],
                "relaxations": st["relaxations"], "extracted": st["extracted"], "team": st["team"],
                "exact": exact,
                "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sssp_multi",
                             "kernel_ms": kern_ms, "algorithmic_bytes": abytes}}

    from paper_1908_09378_amd import learn
    blob = torch.from_numpy(learn.load_model()).to(dev)
    t0 = time.perf_counter()
    tuned = pkg.sssp_batch_autotune(qs, k_rule=2, k_model=blob)
    tuned["tune_s"] = time.perf_counter() - t0
    print(f"[bench] batch autotune: {tuned}", file=sys.stderr, flush=True)
    lr = timed(k_rule=2, k_model=blob, d_scale=tuned["d_scale"], k_max=tuned["k_max"], team=tuned["team"],
               k_scale=tuned["k_scale"])
    pr = timed()
    line = {
        "metric": METRIC, "value": lr["value"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": lr["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "256 queries: 64 random geometric graphs (n = floor(2^(12+6u)), mean degree 24, "
                               "w = round(1000 len)+1), 4 sources each, one launch",
                   "method": "batched parDijkstra with the learned threshold, one parBucketHeap per query; "
                             "d (as a multiple of each query's max out-degree) and k_max autotuned",
                   "autotune": tuned,
                   "queries": len(qs), "sum_n": sum(g.n for g, _ in batch), "sum_m_over_queries": sum_m,
                   "team": lr["team"]},
        "roofline": lr["roofline"], "rounds": lr["rounds"], "relaxations": lr["relaxations"],
        "extracted": lr["extracted"], "exact": lr["exact"] and pr["exact"],
        "plain": pr, "speedup_vs_plain": lr["value"] / pr["value"],
    }
    if not args.no_cpu:
        t0 = time.perf_counter()
        runs = 0
        for g, srcs in batch:
            for s in srcs:
                oracle.dijkstra(g, s)
                runs += 1
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": sum_m / el / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
                                "sample": f"all {runs} queries, single-thread binary-heap Dijkstra ({el:.1f} s), "
                                          f"host {os.cpu_count()} cpus"}
    print(json.dumps(line), flush=True)


def run_heap(args):
    """The standalone heap: 2^24 ids with keys uniform in [0, 2^40) loaded in
    16 pieces of d = 2^20 (untimed), then rounds of bulk_update with 2^20
    decrease-keys (ids drawn with replacement from the live set, new key = old
    - uniform[0, old/2]) and extract_min of 2^16.  Each call is synchronous
    and timed on its own; the batches come from a host copy of the current
    keys kept in lockstep.  Every extraction is checked exactly: ascending,
    keys equal to the current keys, and the largest extracted pair below every
    remaining one."""
    import numpy as np
    import torch

    import oracle
    import paper_1908_09378_amd as pkg
    import workloads as W

    INF = np.uint64(0xFFFFFFFFFFFFFFFF)
    n_ids, d, ext = 1 << 24, 1 << 20, 1 << 16
    rounds = args.heap_rounds
    dev = torch.device("cuda:0")

    def to_dev(k, i):
        return (torch.from_numpy(k.view(np.int64)).to(dev), torch.from_numpy(i.view(np.int32)).to(dev))

    keys, ids = W.heap_init_pairs(n_ids, seed=3)
    h = pkg.Heap(n_ids, d)
    for c in range(0, n_ids, d):
        h.bulk_update(*to_dev(keys[c:c + d], ids[c:c + d]))
    torch.cuda.synchronize()
    cur = np.full(n_ids, INF, dtype=np.uint64)
    cur[ids] = keys
    ko = torch.empty(ext, dtype=torch.int64, device=dev)
    io = torch.empty(ext, dtype=torch.int32, device=dev)
    t_upd = t_ext = 0.0
    elems_upd = 0
    ok = True
    kept = []

    def one_round(r):
        """bulk_update + extract_min of round r, checked; returns (update s, extract s, elements)."""
        nonlocal ok
        live = np.flatnonzero(cur != INF).astype(np.uint32)
        bk, bi = W.decrease_batch(live, lambda x: cur[x], d, 3, r)
        if len(kept) < 4:
            kept.append((bk, bi))
        dk, di = to_dev(bk, bi)
        torch.cuda.synchronize()
        e0 = h.traffic()
        t0 = time.perf_counter()
        h.bulk_update(dk, di)
        tu = time.perf_counter() - t0
        el = h.traffic() - e0
        np.minimum.at(cur, bi, bk)
        t0 = time.perf_counter()
        n = h.extract_min(ext, ko, io)
        te = time.perf_counter() - t0
        hk = ko[:n].cpu().numpy().view(np.uint64)
        hi = io[:n].cpu().numpy().view(np.uint32)
        good = n == ext and bool(np.all(cur[hi] == hk)) and np.unique(hi).shape[0] == n
        good = good and bool(np.all((hk[1:] > hk[:-1]) | ((hk[1:] == hk[:-1]) & (hi[1:] > hi[:-1]))))
        cur[hi] = INF
        mk = cur.min()
        if good and mk != INF:
            good = mk > hk[-1] or (mk == hk[-1] and int(np.flatnonzero(cur == mk).min()) > int(hi[-1]))
        ok &= bool(good)
        return tu, te, el

    # Every 32nd round (the last one, for short runs) is profiled instead of
    # timed: HIP events around each merge writing pass give the kernel's own
    # duration for the roofline; the timed rounds run without instrumentation.
    profiled = {r for r in range(rounds) if r % 32 == 31} if rounds >= 32 else {rounds - 1}
    if rounds < 2:
        profiled = set()
    timed = 0
    m_launch = m_bytes_tot = 0
    m_ms_tot = 0.0
    for r in range(rounds):
        if r in profiled:
            h.set_profiling(True)
            mp0 = h.merge_profile()
            one_round(r)
            mp1 = h.merge_profile()
            h.set_profiling(False)
            m_launch += mp1["launches"] - mp0["launches"]
            m_bytes_tot += mp1["bytes"] - mp0["bytes"]
            m_ms_tot += mp1["ms"] - mp0["ms"]
            continue
        tu, te, el = one_round(r)
        t_upd += tu
        t_ext += te
        elems_upd += el
        timed += 1
        if timed % 32 == 1:
            print(f"[bench] heap round {r}: update {t_upd / timed * 1e3:.2f} ms, extract "
                  f"{t_ext / timed * 1e3:.2f} ms, exact={ok}", file=sys.stderr, flush=True)
    ok &= h.size() == int(np.count_nonzero(cur != INF))
    m_bytes = m_bytes_tot / max(1, m_launch)
    m_ms = m_ms_tot / max(1, m_launch)
    n_rounds = rounds
    rounds = max(1, timed)
    upd_s = t_upd / rounds
    # algorithmic bytes of one bulk_update: the level operations' elements
    # (12 B each) plus the intake: read the pairs (12 B), the atomicMin on the
    # current key (8 B) and a changed-id mark of one bit per id, scanned twice
    abytes = 12.0 * elems_upd / rounds + 20.0 * d + n_ids / 4
    achieved = abytes / upd_s / 1e9
    line = {"metric": "parBucketHeap bulk_update keys/s on 1 MI355X", "value": d / upd_s, "unit": "keys/s",
            "n_gpus": 1, "steps": rounds, "warmup": 0, "ms_per_step": (t_upd + t_ext) / rounds * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "standalone heap: 2^24 ids, keys U[0,2^40), d=2^20; rounds of 2^20 "
                                   "decrease-keys (new = old - U[0, old/2]) + extract_min(2^16)",
                       "rounds": n_rounds, "timed_rounds": rounds, "engine": "device-wide"},
            "update_ms": upd_s * 1e3, "extract_ms": t_ext / rounds * 1e3,
            "extract_keys_per_s": ext / (t_ext / rounds),
            "roofline": {"bound": "hbm", "achieved": m_bytes / (m_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": m_bytes / (m_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_merge<true> (merge + DeleteDuplicates, writing pass)",
                         "kernel_ms": m_ms, "algorithmic_bytes": m_bytes, "launches": m_launch,
                         "measured": f"HIP events around each launch in {len(profiled)} profiled rounds"},
            "op_level": {"achieved": achieved, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "what": "bulk_update as a whole (all kernels and host steps)", "algorithmic_bytes": abytes},
            "exact": ok}
    if not args.no_cpu:
        o = oracle.PQ(n_ids)
        o.bulk_update(keys, ids)
        t0 = time.perf_counter()
        done = 0
        for bk, bi in kept:
            o.bulk_update(bk, bi)
            o.extract_min(ext)
            done += bk.shape[0]
            if time.perf_counter() - t0 > args.cpu_budget:
                break
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": done / el, "unit": "keys/s", "cores": 1, "kind": "oracle",
                                "sample": f"{len(kept)} rounds (bulk_update 2^20 + extract_min 2^16) on the "
                                          f"std::set oracle after the same 2^24 load ({el:.1f} s)"}
    print(json.dumps(line), flush=True)


def run_copy(args):
    """Calibration for the HBM counters: a plain device-to-device copy of
    2 GiB (torch's copy kernel), repeated `steps` times.  FETCH_SIZE and
    WRITE_SIZE of this kernel, divided by 2 GiB, give the factor by which the
    counters over- or under-count HBM bytes."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.int64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"metric": "device copy GB/s", "value": 2 * 8 * n / sec / 1e9, "unit": "GB/s",
                      "bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n, "steps": args.steps}),
          flush=True)


def algorithmic_bytes(st):
    """Bytes the method must move per launch: per extracted vertex its two CSR
    offsets (16 B); per scanned edge its target and weight (8 B) and the 8-byte
    atomicMin on dist; per heap element read or written by the level operations
    (Merge, DeleteDuplicates, Select, splits) 12 B (u64 key + u32 id)."""
    return 16 * st["extracted"] + 16 * st["relaxations"] + 12 * st["heap_elems"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ring")
    ap.add_argument("--method", default="both", choices=["plain", "learned", "both"],
                    help="plain parDijkstra (the timed value), the learned threshold, or both on the same graph")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--heap-rounds", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the bench runs on one GPU only; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)

    if args.workload == "multi":
        return run_multi(args)
    if args.workload == "heap":
        return run_heap(args)
    if args.workload == "copy":
        return run_copy(args)

    import numpy as np
    import torch

    import paper_1908_09378_amd as pkg

    g, desc = make_graph(args.workload)
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.offsets.view(np.int64)).to(dev)
    tg = torch.from_numpy(g.targets.view(np.int32)).to(dev)
    wt = torch.from_numpy(g.weights.view(np.int32)).to(dev)
    dist = torch.empty(g.n, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    import oracle
    if args.workload == "dag":
        ref = np.arange(g.n, dtype=np.uint64)  # the chain of weight-1 edges is the shortest path (closed form)
    else:
        ref = oracle.dijkstra(g, 0)

    def timed(steps, warmup, **kw):
        stats = []
        for _ in range(warmup):
            pkg.sssp_ex(off, tg, wt, g.n, g.m, 0, dist, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            stats.append(pkg.sssp_ex(off, tg, wt, g.n, g.m, 0, dist, **kw))
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        exact = bool(np.array_equal(dist.cpu().numpy().view(np.uint64), ref))
        print(f"[bench] {kw.get('k_rule', 0) and 'learned' or 'plain'}: {sec * 1e3:.1f} ms/step, "
              f"{stats[-1]['rounds']} rounds, exact={exact}", file=sys.stderr, flush=True)
        return sec, stats, exact

    def record(sec, stats, exact, method):
        st = stats[-1]
        kern_ms = sum(x["kernel_ms"] for x in stats) / len(stats)
        abytes = algorithmic_bytes(st)
        achieved = abytes / (kern_ms * 1e-3) / 1e9
        return {"value": g.m / sec / 1e9, "ms_per_step": sec * 1e3, "method": method, "rounds": st["rounds"],
                "relaxations": st["relaxations"], "extracted": st["extracted"], "updates": st["updates"],
                "d": st["d"], "team": st["team"], "levels": st["levels"], "lds_levels": st["lds_levels"],
                "us_per_round": kern_ms * 1e3 / max(1, st["rounds"]), "exact": exact,
                "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sssp",
                             "kernel_ms": kern_ms, "algorithmic_bytes": abytes}}

    def tune(**kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = pkg.sssp_autotune(off, tg, wt, g.n, g.m, 0, dist, **kw)
        torch.cuda.synchronize()
        t["tune_s"] = time.perf_counter() - t0
        print(f"[bench] autotune {kw.get('k_rule', 0)}: {t}", file=sys.stderr, flush=True)
        return t

    runs = {}
    if args.method in ("both", "learned"):
        from paper_1908_09378_amd import learn
        blob = torch.from_numpy(learn.load_model()).to(dev)
        t = tune(k_rule=2, k_model=blob)
        r = record(*timed(args.steps, args.warmup, k_rule=2, k_model=blob, d=t["d"], k_max=t["k_max"],
                          team=t["team"], k_scale=t["k_scale"]),
                   "learned threshold: an 8-64-64-1 GELU MLP (bf16 weights, models/k_mlp.bin) picks how many "
                   "minima each round extracts, improved vertices are re-inserted; d, team and k_max autotuned")
        r["autotune"] = t
        runs["learned"] = r
    if args.method in ("both", "plain"):
        runs["plain"] = record(*timed(args.steps, args.warmup), "plain parDijkstra (k = 1, d = max out-degree)")
    if args.method == "both":
        t = tune()
        r = record(*timed(args.steps, args.warmup, d=t["d"], team=t["team"]),
                   "plain parDijkstra (k = 1), d and team autotuned")
        r["autotune"] = t
        runs["plain_tuned"] = r
    main_run = runs["learned" if "learned" in runs else "plain"]
    line = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "method": main_run["method"], "n": g.n, "m": g.m, "d": main_run["d"],
                   "team": main_run["team"], "levels": main_run["levels"], "lds_levels": main_run["lds_levels"],
                   "parallelism": "1 workgroup per query"},
        "roofline": main_run["roofline"],
        "rounds": main_run["rounds"],
        "relaxations": main_run["relaxations"],
        "extracted": main_run["extracted"],
        "us_per_round": main_run["us_per_round"],
        "exact": all(r["exact"] for r in runs.values()),
    }
    if "autotune" in main_run:
        line["config"]["autotune"] = main_run["autotune"]
    if "learned" in runs and "plain" in runs:
        line["plain"] = {k: v for k, v in runs["plain"].items() if k != "method"}
        line["speedup_vs_plain"] = runs["learned"]["value"] / runs["plain"]["value"]
    if "plain_tuned" in runs:
        line["plain_tuned"] = runs["plain_tuned"]
        line["speedup_vs_plain_tuned"] = runs["learned"]["value"] / runs["plain_tuned"]["value"]
    if not args.no_cpu:
        per_run, runs = oracle.time_dijkstra(g, 0, args.cpu_budget)
        line["cpu_baseline"] = {"value": g.m / per_run / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
                                "sample": f"{runs} full run(s) of single-thread binary-heap Dijkstra on the "
                                          f"same graph ({per_run:.2f} s each), host {os.cpu_count()} cpus"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
