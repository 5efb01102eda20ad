"""sssp_noalloc (the entry point that allocates no device memory) against
sssp_ex, through the C ABI: two calls in a row, the second on a smaller graph,
with the plain rule and with a rule that pulls ahead (which uses the scratch's
update lists); distances bit-exact and equal run statistics; a query whose
heap does not fit in the fixed scratch is refused before anything runs."""
import numpy as np
import pytest
import torch

import oracle
import paper_1908_09378_amd as pkg
import workloads as W
from gpu_util import DEV, graph_to_dev, host64

pytestmark = pytest.mark.gpu

STATS = ("rounds", "relaxations", "updates", "extracted", "heap_elems", "levels", "d", "team", "lds_levels")


def _pair(g, src, **kw):
    off, tg, wt = graph_to_dev(g)
    d_ex = torch.empty(g.n, dtype=torch.int64, device=DEV)
    d_na = torch.full((g.n,), 7, dtype=torch.int64, device=DEV)
    print(f"[noalloc] {g.name} n={g.n} m={g.m} {kw}", flush=True)
    s_ex = pkg.sssp_ex(off, tg, wt, g.n, g.m, src, d_ex, **kw)
    s_na = pkg.sssp_noalloc(off, tg, wt, g.n, g.m, src, d_na, **kw)
    ref = oracle.dijkstra(g, src)
    assert np.array_equal(host64(d_ex), ref)
    assert np.array_equal(host64(d_na), host64(d_ex))
    for k in STATS:
        assert s_na[k] == s_ex[k], k
    assert s_na["kernel_ms"] == 0.0


@pytest.mark.parametrize("kw", [dict(), dict(k_rule=1, k_fixed=8), dict(team=256, schedule=1)])
def test_noalloc_matches_sssp_ex_twice_second_smaller(kw):
    _pair(W.grid4(64, 64, 1, 100, seed=1), 0, **kw)
    _pair(W.grid4(20, 23, 1, 100, seed=2), 5, **kw)


def test_noalloc_refuses_a_query_larger_than_its_scratch():
    g = W.ring_lattice(1 << 16, 16, 1, 1000, seed=2)
    off, tg, wt = graph_to_dev(g)
    dist = torch.full((g.n,), 7, dtype=torch.int64, device=DEV)
    print("[noalloc] oversized query", flush=True)
    with pytest.raises(pkg.PBHError) as e:
        pkg.sssp_noalloc(off, tg, wt, g.n, g.m, 0, dist)
    assert e.value.code == pkg.PBH_EINVAL and "scratch" in str(e.value)
    assert bool((dist == 7).all())
    # the scratch still serves a query that fits afterwards
    _pair(W.grid4(16, 16, 1, 100, seed=3), 0)
