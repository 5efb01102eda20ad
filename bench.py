"""Benchmark: parDijkstra on the parallel bucket heap, 1 MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload all|ring|grid64|grid8|batch|heap|dag|copy] [--no-cpu]
                    [--dag-m M] [--dag-seeds S] [--dag-trials T] [--nearfar-factors F ...]

One step of the headline = one complete sssp() over the resident ring
lattice (n = 2^20 vertices, each linked to its 16 nearest neighbours on each
side, m = 33,554,432 directed edges, integer weights uniform in [1, 1000],
source 0) with the learned extraction threshold: every round of the hot path
(features and MLP, extract-min, relaxation, re-insertion, bulk update, the
Resolve schedule).  Plain parDijkstra on the same graph (d = the maximum
out-degree, and d autotuned) is timed beside it.

The default (--workload all) prints ONE JSON line: the headline (GTEPS =
m / seconds per step, K timed steps after W warm-up steps, the roofline of
the round-loop kernel and the single-thread CPU oracle on the same graph) and,
under "workloads", one record per other configuration, each with its own
steps, exactness check against the oracle, roofline and CPU baseline:

  grid64   4-neighbour grid 64x64, w ~ U[1,100]: plain and learned;
  grid8    8-neighbour grid 2048x2048, w log-uniform in [1, 10^4]: learned
           threshold vs plain parDijkstra;
  batch    256 queries over 64 random geometric graphs in one launch
           (learned and plain), with a sample of the same queries run one by
           one, and the oracle on 1 and on all host threads;
  heap     the standalone heap: 2^24 ids, 256 rounds of bulk_update(2^20
           decrease-keys) + extract_min(2^16), every extraction checked;
  dag      the paper's high-diameter DAG (n = 30,000, m = 4e7 by default):
           plain parDijkstra and Near-Far against the closed-form distances.

Near-Far (Delta-stepping, the paper's comparison family) runs beside
parDijkstra on the ring, the large grid and the DAG.

--workload X runs one of them alone and prints its record as the line.
Inputs are synthetic and seeded (workloads/), resident in HBM before timing.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSSP GTEPS (m/time) on 1 MI355X: learned-threshold & batched vs plain parDijkstra"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1908_09378_amd", "csrc")
KERNEL_SOURCES = ["pbh_core.h", "pbh_team.h", "pbh_launch.h", "round_loop.h", "kernels.hip", "kernels_full.hip",
                  "wide.h", "wide.hip", "learn.hip", "nearfar.hip"]

RING_DESC = "ring lattice n=2^20, 16 neighbours per side, w~U[1,1000], source 0"
GRID64_DESC = "4-neighbour grid 64x64, w~U[1,100], source 0"
GRID8_DESC = "8-neighbour grid 2048x2048, w log-uniform [1,1e4], source 0"
LEARNED_DESC = ("learned threshold: an 8-64-64-1 GELU MLP (bf16 weights, models/k_mlp.bin) picks how many "
                "minima each round extracts, improved vertices are re-inserted")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------- helpers
# The sources each measured kernel is built from: a change to any of them
# voids that kernel's recorded counters.
_CORE = ["pbh_team.h", "pbh_core.h"]
KERNEL_FAMILIES = {
    "k_sssp": _CORE + ["pbh_launch.h", "round_loop.h", "kernels.hip"],
    "k_sssp_full": _CORE + ["pbh_launch.h", "round_loop.h", "kernels_full.hip"],
    "k_sssp_multi": _CORE + ["pbh_launch.h", "round_loop.h", "kernels_full.hip"],
    "k_nearfar": ["pbh_team.h", "nearfar.hip"],
    "heap": _CORE + ["wide.h", "wide.hip"],
}


def kernel_source_sha(kernel=None, workload=None):
    """Hash of the sources `kernel` is built from (all kernel sources when
    no kernel is named; every engine kernel of the standalone heap shares the
    "heap" family)."""
    fam = "heap" if workload == "heap" else kernel
    files = KERNEL_FAMILIES.get(fam, KERNEL_SOURCES)
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the calibrated
    rocprofv3 counters recorded in profiles/traffic.md -- or None when none
    were taken, or when the kernel's sources changed since (the row's source
    hash differs from the current one)."""
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path):
        return None
    sha = kernel_source_sha(kernel, workload)
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == kernel and cells[1] == workload and cells[2] == sha:
            try:
                return float(cells[3]) + float(cells[4])
            except ValueError:
                return None
    return None


def roofline(kernel, workload, abytes, kern_ms, extra=None):
    achieved = abytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else 0.0
    r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(kernel, workload), "kernel": kernel,
         "kernel_ms": kern_ms, "algorithmic_bytes": abytes}
    if extra:
        r.update(extra)
    return r


def sssp_bytes(st):
    """Bytes the method must move per launch: per extracted vertex its two CSR
    offsets (16 B); per scanned edge its target and weight (8 B) and the 8-byte
    atomicMin on dist; per heap element read or written by the level operations
    (Merge, DeleteDuplicates, Select, splits) 12 B (u64 key + u32 id)."""
    return 16 * st["extracted"] + 16 * st["relaxations"] + 12 * st["heap_elems"]


def to_dev(g):
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    return (torch.from_numpy(g.offsets.view(np.int64)).to(dev), torch.from_numpy(g.targets.view(np.int32)).to(dev),
            torch.from_numpy(g.weights.view(np.int32)).to(dev))


def load_blob():
    import torch
    from paper_1908_09378_amd import learn
    return torch.from_numpy(learn.load_model()).to(torch.device("cuda:0"))


class Query:
    """One resident graph + source + distance buffer, and the oracle's answer."""

    def __init__(self, g, src, ref):
        import torch
        self.g, self.src, self.ref = g, src, ref
        self.off, self.tg, self.wt = to_dev(g)
        self.dist = torch.empty(g.n, dtype=torch.int64, device=torch.device("cuda:0"))
        torch.cuda.synchronize()

    def run(self, **kw):
        import paper_1908_09378_amd as pkg
        return pkg.sssp_ex(self.off, self.tg, self.wt, self.g.n, self.g.m, self.src, self.dist, **kw)

    def exact(self):
        import numpy as np
        return bool(np.array_equal(self.dist.cpu().numpy().view(np.uint64), self.ref))

    def timed(self, steps, warmup, label, **kw):
        """warmup untimed runs, then `steps` timed runs (synchronised on both
        sides); distances checked after the last one."""
        import torch
        for _ in range(warmup):
            self.run(**kw)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            stats.append(self.run(**kw))
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        ex = self.exact()
        log(f"{label}: {sec * 1e3:.1f} ms/step over {steps}, {stats[-1]['rounds']} rounds, exact={ex}")
        return sec, stats, ex

    def record(self, sec, stats, exact, method, workload, steps, warmup, kernel="k_sssp"):
        st = stats[-1]
        kern_ms = sum(x["kernel_ms"] for x in stats) / len(stats)
        kms = sorted(x["kernel_ms"] for x in stats)
        return {"value": self.g.m / sec / 1e9, "unit": "GTEPS", "steps": steps, "warmup": warmup,
                "ms_per_step": sec * 1e3, "kernel_ms_mean": kern_ms, "kernel_ms_median": kms[len(kms) // 2],
                "method": method, "rounds": st["rounds"],
                "relaxations": st["relaxations"], "extracted": st["extracted"], "updates": st["updates"],
                "d": st["d"], "team": st["team"], "levels": st["levels"], "lds_levels": st["lds_levels"],
                "us_per_round": kern_ms * 1e3 / max(1, st["rounds"]), "exact": exact,
                "roofline": roofline(kernel, workload, sssp_bytes(st), kern_ms)}

    def nearfar(self, steps, factors=(1.0,)):
        """The Near-Far (Delta-stepping) baseline on the same graph: delta =
        f x Davidson et al.'s choice for each f, one untimed and `steps` timed
        runs each; the fastest delta is the record, the others are listed."""
        import numpy as np
        import torch
        import paper_1908_09378_amd as pkg
        base = pkg.sssp_nearfar(self.off, self.tg, self.wt, self.g.n, self.g.m, self.src, self.dist)["delta"]
        tried = []
        for f in factors:
            delta = max(1, int(base * f))
            pkg.sssp_nearfar(self.off, self.tg, self.wt, self.g.n, self.g.m, self.src, self.dist, delta)
            torch.cuda.synchronize()
            stats = []
            t0 = time.perf_counter()
            for _ in range(steps):
                stats.append(pkg.sssp_nearfar(self.off, self.tg, self.wt, self.g.n, self.g.m, self.src, self.dist,
                                              delta))
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / steps
            ex = self.exact()
            st = stats[-1]
            tried.append({"delta": delta, "value": self.g.m / sec / 1e9, "ms_per_step": sec * 1e3, "exact": ex,
                          "relaxations": st["relaxations"], "phases": st["phases"], "splits": st["splits"],
                          "kernel_ms": sum(x["kernel_ms"] for x in stats) / len(stats)})
            log(f"nearfar delta={delta}: {sec * 1e3:.1f} ms, {st['phases']} phases, exact={ex}")
        best = min(tried, key=lambda r: r["ms_per_step"])
        abytes = 16 * best["relaxations"]  # per scanned edge: target + weight + the dist atomic
        return {"unit": "GTEPS", "value": best["value"], "ms_per_step": best["ms_per_step"], "steps": steps,
                "delta": best["delta"], "exact": all(r["exact"] for r in tried),
                "method": "Near-Far (Delta-stepping), one cooperative launch over every CU; the fastest of "
                          "delta = f x (mean weight x 64 / mean degree), f in " + str(list(factors)),
                "roofline": roofline("k_nearfar", "nearfar", abytes, best["kernel_ms"]),
                "tried": tried}

    def tune(self, **kw):
        import torch
        import paper_1908_09378_amd as pkg
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = pkg.sssp_autotune(self.off, self.tg, self.wt, self.g.n, self.g.m, self.src, self.dist, **kw)
        torch.cuda.synchronize()
        t["tune_s"] = time.perf_counter() - t0
        log(f"autotune rule {kw.get('k_rule', 0)}: {t}")
        return t


def cpu_sssp(g, src, budget):
    import oracle
    per_run, runs = oracle.time_dijkstra(g, src, budget)
    return {"value": g.m / per_run / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{runs} full run(s) of single-thread binary-heap Dijkstra on the same graph "
                      f"({per_run:.2f} s each), host {os.cpu_count()} cpus"}


# ----------------------------------------------------------------- workloads
def run_ring(args):
    """The headline: learned threshold on the ring lattice, with plain
    parDijkstra (d = maximum out-degree, and d autotuned) beside it."""
    import oracle
    import workloads as W
    g = W.ring_lattice(1 << 20, 16, 1, 1000, seed=2)
    q = Query(g, 0, oracle.dijkstra(g, 0))
    blob = load_blob()
    t = q.tune(k_rule=2, k_model=blob)
    kw = dict(k_rule=2, k_model=blob, d=t["d"], k_max=t["k_max"], team=t["team"], k_scale=t["k_scale"],
              k_every=t["k_every"])
    lr = q.record(*q.timed(args.steps, args.warmup, "ring learned", **kw),
                  LEARNED_DESC + "; d, team and k_max autotuned", "ring", args.steps, args.warmup)
    lr["autotune"] = t
    if args.learned_only:  # profiling runs: the learned launches are the last k_sssp dispatches
        rec = dict(lr)
        rec["config"] = {"workload": RING_DESC, "method": lr["method"], "n": g.n, "m": g.m}
        return rec
    pl = q.record(*q.timed(args.base_steps, 0, "ring plain"), "plain parDijkstra (k = 1, d = max out-degree)",
                  "ring_plain", args.base_steps, 0)
    pt = q.record(*q.timed(args.base_steps, 0, "ring plain tuned", **RING_PLAIN_TUNED),
                  "plain parDijkstra (k = 1), d = 512, team 64 (one of sssp_autotune's choices for the plain "
                  "rule on this graph, d = 64 to 512 within 0.5%)", "ring_plain", args.base_steps, 0)
    rec = dict(lr)
    rec["plain"] = pl
    rec["plain_tuned"] = pt
    rec["speedup_vs_plain"] = lr["value"] / pl["value"]
    rec["speedup_vs_plain_tuned"] = lr["value"] / pt["value"]
    rec["nearfar"] = q.nearfar(args.base_steps, args.nearfar_factors)
    rec["exact"] = lr["exact"] and pl["exact"] and pt["exact"] and rec["nearfar"]["exact"]
    rec["config"] = {"workload": RING_DESC, "method": lr["method"], "n": g.n, "m": g.m, "d": lr["d"],
                     "team": lr["team"], "levels": lr["levels"], "lds_levels": lr["lds_levels"],
                     "parallelism": "1 workgroup per query"}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_sssp(g, 0, args.cpu_budget)
    return rec


def run_grid64(args):
    """The small 64x64 grid: plain parDijkstra (every round of the method,
    4,096 of them) and the learned threshold; at least 10 timed runs after at
    least one warm-up run (the paper's protocol), mean and median reported."""
    import oracle
    import workloads as W
    g = W.grid4(64, 64, 1, 100, seed=1)
    q = Query(g, 0, oracle.dijkstra(g, 0))
    steps, warm = max(10, args.steps), max(1, args.warmup)
    pl = q.record(*q.timed(steps, warm, "grid64 plain"), "plain parDijkstra (k = 1, d = max out-degree)",
                  "grid64", steps, warm)
    blob = load_blob()
    lr = q.record(*q.timed(steps, warm, "grid64 learned", k_rule=2, k_model=blob, d=32),
                  LEARNED_DESC + "; d = 32", "grid64_learned", steps, warm)
    rec = {"metric": "SSSP GTEPS (m/time), plain parDijkstra", **pl,
           "config": {"workload": GRID64_DESC, "n": g.n, "m": g.m}, "learned": lr,
           "exact": pl["exact"] and lr["exact"]}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_sssp(g, 0, min(args.cpu_budget, 5.0))
    return rec


# Settings sssp_autotune chose for the 2048x2048 grid with the deep-level
# workers (its trials take about 70 s there, so the bench does not repeat
# them): d = 32 x the maximum out-degree, 256 threads, at most 256 minima per
# round, the model every fourth round.  The plain rule runs
# at d = 2048 with 256 threads, the fastest per round of the settings the
# autotuner tries, measured over the first 200,000 rounds.  Both with the
# deep-level workers (levels >= 2 resolved by workgroups of their own).
GRID8_LEARNED = dict(d=256, team=256, k_max=256, k_every=4, deep_level=2)
GRID8_PLAIN = dict(d=2048, team=256, deep_level=2)
# sssp_autotune's choice for the plain rule on the ring lattice: 64 threads
# and d = 64, 256 or 512 from run to run, all within 0.5% of each other
# (6.72 s at d = 512, 6.74 s at d = 64).
RING_PLAIN_TUNED = dict(d=512, team=64)


def run_grid8(args):
    import oracle
    import workloads as W
    g = W.grid8(2048, 2048, wmax=10000, seed=4)
    q = Query(g, 0, oracle.dijkstra(g, 0))
    blob = load_blob()
    lr = q.record(*q.timed(args.base_steps, 1, "grid8 learned", k_rule=2, k_model=blob, **GRID8_LEARNED),
                  LEARNED_DESC + "; d = 256, team 256, k_max 256, model every 4th round (autotuned settings for "
                  "this graph), deep-level workers from level 2", "grid8", args.base_steps, 1,
                  kernel="k_sssp_full")
    # Plain parDijkstra settles one vertex per round, 4,194,304 rounds here
    # (many minutes); the bench times its first 2^18 rounds and reports their
    # rate.  The heap grows during a run, so later rounds cost more and the
    # estimate of the whole run (per-round time x n) is a lower bound.
    pre = 1 << 18
    sec, sts, _ = q.timed(1, 0, "grid8 plain (first 2^18 rounds)", max_rounds=pre, **GRID8_PLAIN)
    st = sts[-1]
    kern_s = st["kernel_ms"] * 1e-3
    pl = {"method": "plain parDijkstra (k = 1), d = 2048, team 256, deep-level workers from level 2; the first "
                    "2^18 of its 4,194,304 rounds (one per vertex)",
          "rounds": st["rounds"], "relaxations": st["relaxations"], "ms": sec * 1e3,
          "us_per_round": kern_s * 1e6 / st["rounds"], "edges_per_s": st["relaxations"] / kern_s,
          "estimated_full_s": kern_s / st["rounds"] * g.n,
          "roofline": roofline("k_sssp_full", "grid8_plain", sssp_bytes(st), st["kernel_ms"])}
    nfr = q.nearfar(args.base_steps, args.nearfar_factors)
    rec = {"metric": "SSSP GTEPS (m/time), learned threshold", **lr,
           "config": {"workload": GRID8_DESC, "n": g.n, "m": g.m}, "plain": pl,
           "speedup_vs_plain_estimate": pl["estimated_full_s"] / (lr["ms_per_step"] * 1e-3), "nearfar": nfr,
           "reinsertions": lr["extracted"] - g.n, "exact": lr["exact"] and nfr["exact"]}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_sssp(g, 0, args.cpu_budget)
    return rec


def run_batch(args):
    """256 queries (64 random geometric graphs with uneven n in 2^12..2^18,
    mean degree 24, 4 sources each) in one persistent launch."""
    import numpy as np
    import torch

    import oracle
    import paper_1908_09378_amd as pkg
    import workloads as W

    batch = W.rgg_batch(64, 4)
    dev = torch.device("cuda:0")
    qs, keep, graphs = [], [], []
    for g, srcs in batch:
        off, tg, wt = to_dev(g)
        keep.append((off, tg, wt))
        for s in srcs:
            qs.append((off, tg, wt, g.n, g.m, s, torch.empty(g.n, dtype=torch.int64, device=dev)))
            graphs.append((g, s))
    sum_m = sum(q[4] for q in qs)
    refs = [oracle.dijkstra(g, s) for g, s in graphs]

    def exact():
        return all(np.array_equal(q[6].cpu().numpy().view(np.uint64), r) for q, r in zip(qs, refs))

    def timed(steps, warmup, label, **kw):
        torch.cuda.synchronize()
        for _ in range(warmup):
            pkg.sssp_batch(qs, **kw)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            stats.append(pkg.sssp_batch(qs, **kw))
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        ex = exact()
        log(f"{label}: {sec * 1e3:.1f} ms/step over {steps}, exact={ex}")
        st = stats[-1]
        kern_ms = sum(x["kernel_ms"] for x in stats) / len(stats)
        return {"value": sum_m / sec / 1e9, "unit": "GTEPS", "steps": steps, "warmup": warmup,
                "ms_per_step": sec * 1e3, "rounds": st["rounds"], "relaxations": st["relaxations"],
                "extracted": st["extracted"], "team": st["team"], "exact": ex,
                "roofline": roofline("k_sssp_multi", "batch", sssp_bytes(st), kern_ms)}

    blob = load_blob()
    t0 = time.perf_counter()
    tuned = pkg.sssp_batch_autotune(qs, k_rule=2, k_model=blob)
    tuned["tune_s"] = time.perf_counter() - t0
    log(f"batch autotune: {tuned}")
    kw = dict(k_rule=2, k_model=blob, d_scale=tuned["d_scale"], k_max=tuned["k_max"], team=tuned["team"],
              k_scale=tuned["k_scale"])
    lr = timed(args.steps, args.warmup, "batch learned", **kw)
    pr = timed(args.base_steps, 0, "batch plain")
    # the same settings, the first queries of the batch's order one launch each:
    # what batching itself gains over running queries one after another
    ns = 16
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in qs[:ns]:
        pkg.sssp_ex(q[0], q[1], q[2], q[3], q[4], q[5], q[6], k_rule=2, k_model=blob, d_scale=tuned["d_scale"],
                    k_max=tuned["k_max"], team=tuned["team"], k_scale=tuned["k_scale"])
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    seq_ok = all(np.array_equal(q[6].cpu().numpy().view(np.uint64), r) for q, r in zip(qs[:ns], refs[:ns]))
    sub = qs[:ns]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pkg.sssp_batch(sub, **kw)
    torch.cuda.synchronize()
    sub_s = time.perf_counter() - t0
    sub_m = sum(q[4] for q in sub)
    rec = {"metric": "batched SSSP GTEPS (sum of m over queries / time)", **lr,
           "config": {"workload": "256 queries: 64 random geometric graphs (n = floor(2^(12+6u)), mean degree 24, "
                                  "w = round(1000 len)+1), 4 sources each, one launch",
                      "method": "batched parDijkstra with the learned threshold, one parBucketHeap per query; "
                                "d (as a multiple of each query's max out-degree), team and k_max autotuned",
                      "autotune": tuned, "queries": len(qs), "sum_n": sum(g.n for g, _ in batch),
                      "sum_m_over_queries": sum_m},
           "plain": pr, "speedup_vs_plain": lr["value"] / pr["value"],
           "one_by_one": {"queries": ns, "sequential_s": seq_s, "batched_s": sub_s,
                          "sequential_gteps": sub_m / seq_s / 1e9, "batched_gteps": sub_m / sub_s / 1e9,
                          "speedup_of_batching": seq_s / sub_s, "exact": seq_ok,
                          "what": "the first 16 queries (largest first), learned rule with the tuned settings: "
                                  "one sssp_ex call each vs one sssp_batch launch"},
           "exact": lr["exact"] and pr["exact"] and seq_ok}
    if not args.no_cpu:
        from concurrent.futures import ThreadPoolExecutor
        t0 = time.perf_counter()
        for g, s in graphs:
            oracle.dijkstra(g, s)
        el1 = time.perf_counter() - t0
        nthreads = os.cpu_count() or 1
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=nthreads) as ex:  # the oracle call releases the GIL
            list(ex.map(lambda gs: oracle.dijkstra(gs[0], gs[1]), graphs))
        eln = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": sum_m / el1 / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
                               "sample": f"all {len(graphs)} queries, single-thread binary-heap Dijkstra "
                                         f"({el1:.1f} s), host {nthreads} cpus"}
        rec["cpu_baseline_all_cores"] = {"value": sum_m / eln / 1e9, "unit": "GTEPS", "cores": nthreads,
                                         "kind": "oracle",
                                         "sample": f"all {len(graphs)} queries, one query per thread on "
                                                   f"{nthreads} threads ({eln:.2f} s)"}
    return rec


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

    def dev_pairs(k, i):
        return (torch.from_numpy(k.view(np.int64)).to(dev), torch.from_numpy(i.view(np.int32)).to(dev))

    keys, ids = W.heap_init_pairs(n_ids, seed=3)
    h = pkg.Heap(n_ids, d)
    for c in range(0, n_ids, d):
        h.bulk_update(*dev_pairs(keys[c:c + d], ids[c:c + d]))
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
        dk, di = dev_pairs(bk, bi)
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
        good = n == min(ext, int(np.count_nonzero(cur != INF))) and bool(np.all(cur[hi] == hk))
        good = good and np.unique(hi).shape[0] == n
        good = good and bool(np.all((hk[1:] > hk[:-1]) | ((hk[1:] == hk[:-1]) & (hi[1:] > hi[:-1]))))
        cur[hi] = INF
        if good and n:
            left = np.flatnonzero(cur != INF)
            if left.size:
                mk = cur[left].min()
                good = mk > hk[-1] or (mk == hk[-1] and int(left[cur[left] == mk].min()) > int(hi[-1]))
        ok &= bool(good)
        return tu, te, el

    # Every 32nd round (the last one, for short runs) is profiled instead of
    # timed: HIP events around every kernel of the engine give each kernel's
    # own duration; the timed rounds run without instrumentation.
    profiled = {r for r in range(rounds) if r % 32 == 31} if rounds >= 32 else {rounds - 1}
    if rounds < 2:
        profiled = set()
    timed = 0
    prof0 = h.kernel_profile()
    for r in range(rounds):
        if r in profiled:
            h.set_profiling(True)
            one_round(r)
            h.set_profiling(False)
            continue
        tu, te, el = one_round(r)
        t_upd += tu
        t_ext += te
        elems_upd += el
        timed += 1
        if timed % 32 == 1:
            log(f"heap round {r}: update {t_upd / timed * 1e3:.2f} ms, extract {t_ext / timed * 1e3:.2f} ms, "
                f"exact={ok}")
    prof = {k: {f: v[f] - prof0[k][f] for f in v} for k, v in h.kernel_profile().items()}
    ok &= h.size() == int(np.count_nonzero(cur != INF))
    n_rounds = rounds
    rounds = max(1, timed)
    upd_s = t_upd / rounds
    # algorithmic bytes of one bulk_update: the level operations' elements
    # (12 B each) plus the intake: read the pairs (12 B), the atomicMin on the
    # current key (8 B) and a changed-id mark of one byte per id, written for
    # changed ids and scanned once
    abytes = 12.0 * elems_upd / rounds + 20.0 * d + n_ids
    achieved = abytes / upd_s / 1e9
    # the roofline names the engine kernel with the most event-timed time
    kern = max(prof, key=lambda k: prof[k]["ms"]) if prof else None
    tot_ms = sum(v["ms"] for v in prof.values()) or 1.0
    if kern:
        kp = prof[kern]
        rl = roofline(kern, "heap", kp["bytes"] / max(1, kp["launches"]), kp["ms"] / max(1, kp["launches"]),
                      {"launches": kp["launches"], "share_of_kernel_time": kp["ms"] / tot_ms,
                       "measured": f"HIP events around each launch in {len(profiled)} profiled rounds"})
    else:
        rl = None
    line = {"metric": "parBucketHeap bulk_update keys/s on 1 MI355X", "value": d / upd_s, "unit": "keys/s",
            "steps": rounds, "warmup": 0, "ms_per_step": (t_upd + t_ext) / rounds * 1e3,
            "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "standalone heap: 2^24 ids, keys U[0,2^40), d=2^20; rounds of 2^20 "
                                   "decrease-keys (new = old - U[0, old/2]) + extract_min(2^16)",
                       "rounds": n_rounds, "timed_rounds": rounds, "engine": "device-wide"},
            "update_ms": upd_s * 1e3, "extract_ms": t_ext / rounds * 1e3,
            "extract_keys_per_s": ext / (t_ext / rounds),
            "roofline": rl,
            "kernels": {k: {"launches": v["launches"], "ms": v["ms"],
                            "GB/s": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else 0.0}
                        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])},
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
    return line


def run_dag(args):
    """The paper's high-diameter DAG (Section 4.2): n = 30,000, a weight-1
    chain plus random forward edges of weight 2(v-u); distances checked
    against the closed form dist(i) = i after every run.  --dag-m sets m,
    --dag-seeds the number of random DAGs (the paper: 5) and --dag-trials the
    timed runs on each (the paper: 10; one untimed run first).  Plain
    parDijkstra and the Near-Far baseline run on every DAG; the means over all
    DAGs and trials are the record."""
    import numpy as np
    import workloads as W
    per = []
    for si in range(args.dag_seeds):
        t0 = time.perf_counter()
        g = W.paper_dag(30000, args.dag_m, seed=11 + si)
        log(f"dag seed {11 + si}: m={g.m} built in {time.perf_counter() - t0:.1f} s")
        q = Query(g, 0, np.arange(g.n, dtype=np.uint64))
        pl = q.record(*q.timed(args.dag_trials, 1, "dag plain", team=1024),
                      "plain parDijkstra (k = 1, d = max out-degree, 1024 threads)", "dag", args.dag_trials, 1)
        nfr = q.nearfar(args.dag_trials, factors=(1.0,))
        per.append({"seed": 11 + si, "plain": pl, "nearfar": nfr})
        if si == 0 and not args.no_cpu:
            cpu = cpu_sssp(g, 0, args.cpu_budget)
        del q, g
    mean = lambda xs: sum(xs) / len(xs)
    pl_ms = mean([p["plain"]["ms_per_step"] for p in per])
    nf_ms = mean([p["nearfar"]["ms_per_step"] for p in per])
    rec = {"metric": "SSSP GTEPS (m/time), plain parDijkstra", "unit": "GTEPS", "value": args.dag_m / pl_ms * 1e-6,
           "ms_per_step": pl_ms, "steps": args.dag_trials, "warmup": 1,
           "us_per_round": mean([p["plain"]["us_per_round"] for p in per]),
           "roofline": per[0]["plain"]["roofline"],
           "nearfar": {"value": args.dag_m / nf_ms * 1e-6, "ms_per_step": nf_ms,
                       "speedup_of_pardijkstra": nf_ms / pl_ms},
           "exact": all(p["plain"]["exact"] and p["nearfar"]["exact"] for p in per),
           "config": {"workload": f"the paper's DAGs: n=30000, m={args.dag_m}, chain of weight 1 plus random forward "
                                  f"edges of weight 2(v-u), source 0; {args.dag_seeds} seeds x {args.dag_trials} "
                                  f"timed trials", "n": 30000, "m": args.dag_m},
           "per_dag": per}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu
    return rec


def run_train(args):
    """Training of the extraction-threshold model, timed stage by stage with
    the settings that produced the committed model (paper_1908_09378_amd/learn.py):
    200 seeded training graphs (ring / 4-neighbour / 8-neighbour grids, n in
    2^14..2^18), plain runs with traces every 16th round in one batched
    launch, labels, then 4000 Adam steps of batch 1024 on the GPU."""
    import torch
    import workloads as W
    from paper_1908_09378_amd import learn
    t0 = time.perf_counter()
    graphs = W.training_graphs(args.train_graphs)
    gen_s = time.perf_counter() - t0
    log(f"train: {len(graphs)} graphs generated in {gen_s:.1f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, Y, st = learn.collect(graphs, 16)
    torch.cuda.synchronize()
    trace_s = time.perf_counter() - t0
    log(f"train: {X.shape[0]} traced rounds in {trace_s:.1f} s")
    t0 = time.perf_counter()
    blob, losses = learn.train(X, Y, 4000, 1024, 1e-3)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    log(f"train: 4000 steps in {fit_s:.1f} s")
    return {"metric": "extraction-threshold model training time", "value": trace_s + fit_s, "unit": "s",
            "higher_is_better": False, "graphs": len(graphs), "sum_n": sum(g.n for g in graphs),
            "traced_rounds": int(X.shape[0]), "graph_generation_s": gen_s, "trace_and_label_s": trace_s,
            "fit_s": fit_s, "steps": 4000, "batch": 1024,
            "loss_first_10": float(losses[:10].mean()), "loss_last_50": float(losses[-50:].mean()),
            "label_variance": float(Y.var().item()),
            "what": "value = trace collection + labels + training on the GPU (graph generation on the host "
                    "reported apart)"}


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
    return {"metric": "device copy GB/s", "value": 2 * 8 * n / sec / 1e9, "unit": "GB/s",
            "bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n, "steps": args.steps}


RUNNERS = {"ring": run_ring, "grid64": run_grid64, "grid8": run_grid8, "batch": run_batch, "heap": run_heap,
           "dag": run_dag, "copy": run_copy, "train": run_train}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="all", choices=["all"] + sorted(RUNNERS))
    ap.add_argument("--base-steps", type=int, default=2,
                    help="timed runs of the long baselines (plain parDijkstra, the large learned grid)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--heap-rounds", type=int, default=256)
    ap.add_argument("--dag-m", type=int, default=40_000_000)
    ap.add_argument("--dag-seeds", type=int, default=1)
    ap.add_argument("--dag-trials", type=int, default=2)
    ap.add_argument("--train-graphs", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--learned-only", action="store_true",
                    help="ring: only the autotuned learned runs (for profiling; not a bench line)")
    ap.add_argument("--nearfar-factors", type=float, nargs="+", default=[1.0],
                    help="Near-Far deltas tried, as multiples of Davidson et al.'s choice")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the bench runs on one GPU only; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    t_start = time.perf_counter()
    if args.workload != "all":
        rec = RUNNERS[args.workload](args)
        rec.setdefault("metric", METRIC)
        rec["n_gpus"] = 1
        print(json.dumps(rec), flush=True)
        return
    head = run_ring(args)
    subs = {}
    for name in ("grid64", "grid8", "batch", "heap", "dag", "train"):
        t0 = time.perf_counter()
        subs[name] = RUNNERS[name](args)
        subs[name]["wall_s"] = time.perf_counter() - t0
        log(f"{name} done in {subs[name]['wall_s']:.1f} s")
    line = {
        "metric": METRIC, "value": head["value"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic", "config": head["config"],
        "roofline": head["roofline"], "cpu_baseline": head.get("cpu_baseline"),
        "rounds": head["rounds"], "relaxations": head["relaxations"], "extracted": head["extracted"],
        "us_per_round": head["us_per_round"],
        "exact": head["exact"] and all(s.get("exact", True) for s in subs.values()),
        "autotune": head["autotune"], "plain": head["plain"], "plain_tuned": head["plain_tuned"],
        "speedup_vs_plain": head["speedup_vs_plain"], "speedup_vs_plain_tuned": head["speedup_vs_plain_tuned"],
        "workloads": subs, "wall_s": time.perf_counter() - t_start,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
