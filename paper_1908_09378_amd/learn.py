"""Training and use of the extraction-threshold model (an addition to the
paper's method): an MLP (8 features -> 64 -> 64 -> 1, GELU, bfloat16 weights,
FP32 accumulation) that picks how many minima each parDijkstra round pulls.

Pipeline (all device work in the library's kernels):
  1. plain parDijkstra runs over training graphs in one batched launch, with
     traces: every `every`-th round records 8 features and the TK (32)
     smallest (key, id) of B_0 in key order (d_scales can repeat the runs
     with larger bulk sizes d);
  2. labels: log2 of the longest traced prefix whose keys are already final
     distances (the pull size that wastes no relaxation);
  3. feature normalisation and Adam training on the GPU;
  4. the weights (a PBH_MLP_BLOB float32 vector) are saved to a small file
     and passed to sssp_ex / sssp_batch as k_model with k_rule = 2.

    python -m paper_1908_09378_amd.learn --out paper_1908_09378_amd/models/k_mlp.bin
"""
from __future__ import annotations

import argparse
import math
import os
import struct
import time

import numpy as np

from . import MLP_BLOB, MLP_PARAMS, mlp_feature_stats, mlp_trace_labels, mlp_train, sssp_batch

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "models", "k_mlp.bin")
MAGIC = b"PBHKMLP1"
NF, H = 8, 64
TK = 32  # trace record length (PBH_TRACE_K)


def save_model(blob: np.ndarray, path: str) -> None:
    blob = np.ascontiguousarray(blob, np.float32)
    assert blob.shape == (MLP_BLOB,)
    with open(path, "wb") as f:
        f.write(MAGIC + struct.pack("<II", MLP_BLOB, 0))
        f.write(blob.tobytes())


def load_model(path: str = DEFAULT_MODEL) -> np.ndarray:
    with open(path, "rb") as f:
        head = f.read(16)
        if head[:8] != MAGIC:
            raise ValueError(f"{path}: not a model file")
        (n, _) = struct.unpack("<II", head[8:])
        if n != MLP_BLOB:
            raise ValueError(f"{path}: {n} values, expected {MLP_BLOB}")
        return np.frombuffer(f.read(4 * n), dtype=np.float32).copy()


def init_blob(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights from the seeded counter generator, zero biases,
    unit normalisation (replaced by the data's statistics) and output scale 1."""
    import workloads as W
    b = np.zeros(MLP_BLOB, np.float32)
    s = W.stream_seed(seed, 90)
    ctr = 0

    def glorot(fan_in, fan_out):
        nonlocal ctr
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        u = W.rand_unit(s, np.arange(ctr, ctr + fan_in * fan_out, dtype=np.uint64))
        ctr += fan_in * fan_out
        return ((2 * u - 1) * lim).astype(np.float32)

    o = 0
    b[o:o + NF * H] = glorot(NF, H); o += NF * H + H
    b[o:o + H * H] = glorot(H, H); o += H * H + H
    b[o:o + H] = glorot(H, 1); o += H + 1
    b[MLP_PARAMS + NF:MLP_PARAMS + 2 * NF] = 1.0
    b[-1] = 1.0
    return b


def collect(graphs, every: int = 16, cap: int = 1 << 21, source: int = 0, d_scales=(1,)):
    """Plain runs with traces over `graphs` (one query each, one launch per
    d_scale).  Returns device tensors X [n, 8] and Y [n] (labels) and the
    last run's stats."""
    import torch
    dev = torch.device("cuda:0")
    qs, keep, dists = [], [], []
    for g in graphs:
        off = torch.from_numpy(g.offsets.view(np.int64)).to(dev)
        tg = torch.from_numpy(g.targets.view(np.int32)).to(dev)
        wt = torch.from_numpy(g.weights.view(np.int32)).to(dev)
        dist = torch.empty(g.n, dtype=torch.int64, device=dev)
        keep.append((off, tg, wt))
        dists.append(dist)
        qs.append((off, tg, wt, g.n, g.m, source, dist))
    tf = torch.zeros(cap * NF, dtype=torch.float32, device=dev)
    tk = torch.zeros(cap * TK, dtype=torch.int64, device=dev)
    tv = torch.zeros(cap * TK, dtype=torch.int32, device=dev)
    tq = torch.zeros(cap, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    for ds in d_scales:
        st = sssp_batch(qs, trace=(tf, tk, tv, cnt, tq, every), d_scale=ds)
    n = min(int(cnt.item()), cap)
    labels = torch.empty(n, dtype=torch.float32, device=dev)
    mlp_trace_labels(tk, tv, tq, n, dists, labels)
    X = tf[: n * NF].view(n, NF).clone()
    return X, labels, st


def train(X, Y, steps: int = 3000, batch: int = 1024, lr: float = 1e-3, seed: int = 0):
    """Shuffle (seeded), normalise, train; returns the blob (device tensor)."""
    import torch
    g = torch.Generator().manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=g).to(X.device)
    Xs, Ys = X[perm].contiguous(), Y[perm].contiguous()
    blob = torch.from_numpy(init_blob(seed)).to(X.device)
    mlp_feature_stats(Xs, blob)
    losses = mlp_train(Xs, Ys, blob, batch, steps, lr)
    return blob, losses


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--graphs", type=int, default=200)
    ap.add_argument("--every", type=int, default=16)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=1e-3)
    args = ap.parse_args()
    import torch
    import workloads as W
    t0 = time.time()
    graphs = W.training_graphs(args.graphs)
    print(f"[learn] {len(graphs)} graphs, sum n = {sum(g.n for g in graphs)} ({time.time() - t0:.1f} s)", flush=True)
    t0 = time.time()
    X, Y, st = collect(graphs, args.every)
    torch.cuda.synchronize()
    print(f"[learn] {X.shape[0]} traced rounds in {time.time() - t0:.1f} s; label mean 2^{Y.mean().item():.2f}",
          flush=True)
    t0 = time.time()
    blob, losses = train(X, Y, args.steps, 1024, args.lr)
    torch.cuda.synchronize()
    print(f"[learn] trained {args.steps} steps in {time.time() - t0:.1f} s; loss {losses[:10].mean():.4f} -> "
          f"{losses[-50:].mean():.4f} (label variance {Y.var().item():.4f})", flush=True)
    save_model(blob.cpu().numpy(), args.out)
    print(f"[learn] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
