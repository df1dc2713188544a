"""The paper's three GPU strategies, rebuilt as baselines (GPU only): vertex-parallel and
edge-parallel with one workgroup per source, and edge-parallel over the grid with
host-synchronised levels.  Each must give the oracle's BC (1e-9 relative, exact zeros) and
depth, for every workgroup size of the paper's block-size study."""
import sys

import numpy as np
import pytest

import oracle
from paper_1409_7764_amd import graphgen as gg

from helpers import rel_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bc():
    import torch
    from paper_1409_7764_amd import bcmi
    assert torch.cuda.is_available()
    bcmi.lib()
    return bcmi


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_cache = {}


def oracle_of(key, n, u, v, S=None):
    if key not in _cache:
        _cache[key] = oracle.bc(oracle.Graph(n, u, v), S)
    return _cache[key]


@pytest.mark.parametrize("wg", [64, 128, 256, 1024])
@pytest.mark.parametrize("strategy", [1, 2, 3])
def test_strategy_exact_ba(bc, strategy, wg):
    """The paper's workload: a BA digraph (each undirected edge as two directed ones)."""
    n, u, v = gg.barabasi_albert(300, 3, 11)
    want, _, st = oracle_of("ba300", n, u, v)
    g = bc.bc_build_csr(n, u, v)
    say("strategy", strategy, "wg", wg)
    got, info = bc.bc_paper_strategy(g, strategy, wg, info=True)
    assert info["path"] == 3 + strategy and info["n_sources"] == n
    assert info["levels_max"] == int(st[:, 3].max())
    rel_close(got.cpu().numpy(), want, what=f"strategy {strategy} wg {wg}")
    g.free()


@pytest.mark.parametrize("case", ["rmat10", "path", "lattice", "loops_dups"])
@pytest.mark.parametrize("strategy", [1, 2, 3])
def test_strategy_graph_shapes(bc, strategy, case):
    """Hubs (R-MAT), one vertex per level (path, closed form), many narrow levels (lattice),
    and an input with self-loops and repeated pairs (removed by the builder)."""
    if case == "rmat10":
        n, u, v = gg.rmat(10, 8, 10)
    elif case == "path":
        n, u, v = gg.directed_path(60)
    elif case == "lattice":
        n, u, v = gg.grid_random_orientation(16, 16, 2)
    else:
        n, u, v = gg.random_digraph(200, 1500, 3)
    want, _, st = oracle_of(case, n, u, v)
    if case == "path":
        assert np.array_equal(want, [float(i * (n - 1 - i)) for i in range(n)])
    g = bc.bc_build_csr(n, u, v)
    say("strategy", strategy, case)
    got, info = bc.bc_paper_strategy(g, strategy, 256, info=True)
    assert info["levels_max"] == int(st[:, 3].max())
    rel_close(got.cpu().numpy(), want, what=f"strategy {strategy} {case}")
    g.free()


@pytest.mark.parametrize("strategy", [1, 2, 3])
def test_strategy_sampled_multiset(bc, strategy):
    n, u, v = gg.barabasi_albert(500, 5, 12)
    S = np.concatenate([gg.uniform_sources(n, 120, 4), np.array([0, 0, 7], np.uint32)])
    want, _, _ = oracle.bc(oracle.Graph(n, u, v), S)
    g = bc.bc_build_csr(n, u, v)
    got, info = bc.bc_paper_strategy(g, strategy, 128, sources=S, info=True)
    assert info["n_sources"] == len(S)
    rel_close(got.cpu().numpy(), want, what=f"strategy {strategy} sampled")
    empty = bc.bc_paper_strategy(g, strategy, 128, sources=np.zeros(0, np.uint32))
    assert np.all(empty.cpu().numpy() == 0.0)
    g.free()


def test_strategy_rejects_bad_arguments(bc):
    n, u, v = gg.barabasi_albert(50, 2, 1)
    g = bc.bc_build_csr(n, u, v)
    for strategy, wg in [(0, 256), (4, 256), (1, 32), (2, 100), (3, 2048)]:
        with pytest.raises(bc.BcError) as e:
            bc.bc_paper_strategy(g, strategy, wg)
        assert e.value.code == bc.BC_E_INVAL
    with pytest.raises(bc.BcError) as e:
        bc.bc_paper_strategy(g, 1, 256, sources=np.array([3, n], np.uint32))
    assert e.value.code == bc.BC_E_RANGE
    g.free()
