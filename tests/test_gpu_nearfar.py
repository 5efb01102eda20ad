"""GPU parity of the Near-Far (Delta-stepping) baseline with the oracle:
distances bit-exact on every graph family, for deltas from 1 to far above the
largest distance (where it degenerates into frontier Bellman-Ford), with zero
weights, self-loops, multi-edges, unreachable vertices and vertices of high
degree (scanned by the whole grid)."""
import numpy as np
import pytest

import oracle
import paper_1908_09378_amd as pkg
import workloads as W
from gpu_util import DEV, graph_to_dev, host64

pytestmark = pytest.mark.gpu
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def _nf(g, src, delta=0):
    import torch
    off, tg, wt = graph_to_dev(g)
    dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
    print(f"[nearfar] {g.name} n={g.n} m={g.m} src={src} delta={delta}", flush=True)
    st = pkg.sssp_nearfar(off, tg, wt, g.n, g.m, src, dist, delta)
    ref = oracle.dijkstra(g, src)
    got = host64(dist)
    assert np.array_equal(got, ref), f"{int((got != ref).sum())} distances differ"
    reached_edges = int(np.diff(g.offsets)[ref != INF].sum())
    assert st["relaxations"] >= reached_edges
    return st


@pytest.mark.parametrize("delta", [0, 1, 37, 1 << 40])
def test_grid_and_ring(delta):
    _nf(W.grid4(64, 64, 1, 100, seed=1), 0, delta)
    _nf(W.ring_lattice(1 << 12, 16, 1, 1000, seed=2), 5, delta)


@pytest.mark.parametrize("seed", range(8))
def test_random_multigraphs_zero_weights_selfloops(seed):
    n = [1, 2, 17, 300, 1000, 5000][seed % 6]
    m = [0, 3, 50, 4000, 20000, 60000][seed % 6]
    wl, wh = [(0, 0), (0, 3), (1, 1000)][seed % 3]
    _nf(W.random_graph(n, m, wl, wh, 70 + seed), seed % n, [0, 1, 5][seed % 3])


def test_unreachable_and_rgg_and_grid8():
    _nf(W.path_graph(200, seed=3), 100)
    _nf(W.rgg(1 << 14, seed=6), 3)
    _nf(W.grid8(128, 128, wmax=10000, seed=4), 0)


def test_paper_dag_high_degree_vertices():
    """Degrees up to n: vertices above the heavy threshold are scanned by
    every workgroup; distances equal the closed form dist(i) = i."""
    g = W.paper_dag(3000, 4_000_000, seed=7)
    assert g.max_degree() > 1024
    st = _nf(g, 0)
    st = _nf(g, 0, 1)


def test_rows_not_sorted_and_larger_graph():
    _nf(W.shuffle_rows(W.grid8(96, 96, wmax=10000, seed=9), 1), 0)
    _nf(W.ring_lattice(1 << 18, 16, 1, 1000, seed=2), 0)


def test_invalid_inputs():
    import torch
    from gpu_util import dev32, dev64
    g = W.grid4(4, 4)
    off, tg, wt = dev64(g.offsets), dev32(g.targets), dev32(g.weights)
    dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
    with pytest.raises(pkg.PBHError) as e:
        pkg.sssp_nearfar(off, tg, wt, g.n, g.m, g.n, dist)
    assert e.value.code == pkg.PBH_EINVAL
    bad = g.targets.copy()
    bad[3] = 999
    with pytest.raises(pkg.PBHError) as e:
        pkg.sssp_nearfar(off, dev32(bad), wt, g.n, g.m, 0, dist)
    assert e.value.code == pkg.PBH_EINVAL
