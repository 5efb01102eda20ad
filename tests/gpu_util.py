"""Helpers for GPU tests: numpy <-> torch device arrays (uint64 data travels as
int64, uint32 as int32, bit for bit)."""
import numpy as np
import torch

DEV = torch.device("cuda:0")


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(DEV)


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


def host64(t):
    return t.cpu().numpy().view(np.uint64)


def host32(t):
    return t.cpu().numpy().view(np.uint32)


def graph_to_dev(g):
    return dev64(g.offsets), dev32(g.targets), dev32(g.weights)


def run_sssp(pkg, g, src, **kw):
    off, tg, wt = graph_to_dev(g)
    dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
    if kw:
        st = pkg.sssp_ex(off, tg, wt, g.n, g.m, src, dist, **kw)
    else:
        pkg.sssp(off, tg, wt, g.n, g.m, src, dist)
        st = None
    return host64(dist), st
