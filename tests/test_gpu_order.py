"""The batching order built with the CSR (GPU only), checked against its definition.

The order only decides which sources share a batch; BC parity of the batched path is checked
elsewhere.  Here the device order must equal the documented one exactly: vertices ranked
outward from the hub along reversed edges, level by level, each level by (lowest successor
rank on the level before, out-degree bucket descending, id); unreached vertices last by
(out-degree bucket descending, id).
"""
import sys

import numpy as np
import pytest

from paper_1409_7764_amd import graphgen as gg

pytestmark = pytest.mark.gpu

LEVELS = 64


@pytest.fixture(scope="module")
def bc():
    import torch
    from paper_1409_7764_amd import bcmi
    assert torch.cuda.is_available()
    bcmi.lib()
    return bcmi


def expected_order(n, rp, col, cp, cr):
    outdeg = np.diff(rp)
    indeg = np.diff(cp)
    bucket = [32 - int(d).bit_length() for d in outdeg]   # count of leading zeros of a 32-bit degree
    cand = np.nonzero(outdeg > 0)[0]
    best = indeg[cand].max()
    hub = int(cand[indeg[cand] == best].min())
    dist = np.full(n, -1, np.int64)
    rank = np.full(n, -1, np.int64)
    dist[hub] = 0
    rank[hub] = 0
    order = [hub]
    frontier = [hub]
    for k in range(1, LEVELS + 1):
        new = set()
        for u in frontier:
            for v in cr[cp[u]:cp[u + 1]]:
                if dist[v] < 0:
                    dist[v] = k
                    new.add(int(v))
        if not new:
            break
        keys = []
        for v in new:
            succ = col[rp[v]:rp[v + 1]]
            par = min(int(rank[u]) for u in succ if dist[u] == k - 1)
            keys.append((par, bucket[v], v))
        keys.sort()
        for _, _, v in keys:
            rank[v] = len(order)
            order.append(v)
        frontier = [v for _, _, v in keys]
    rest = sorted((bucket[v], v) for v in range(n) if rank[v] < 0)
    order += [v for _, v in rest]
    return np.array(order, np.int64)


def in_star(n):
    u = np.arange(1, n, dtype=np.uint32)
    return n, u, np.zeros(n - 1, np.uint32)


@pytest.mark.parametrize("case", ["rmat12", "rmat15", "path200", "in_star", "grid20", "two_parts", "empty"])
def test_batching_order(bc, case):
    print("order case", case, flush=True)
    sys.stdout.flush()
    if case == "rmat12":
        n, u, v = gg.rmat(12, 8, 3)
    elif case == "rmat15":
        n, u, v = gg.rmat(15, 16, 5)
    elif case == "path200":   # longer than the ranked levels: most vertices fall to the rest
        n, u, v = gg.directed_path(200)
    elif case == "in_star":   # the largest in-degree has no out-edges: the hub is another vertex
        n, u, v = in_star(100)
    elif case == "grid20":
        n, u, v = gg.grid_random_orientation(20, 20, 4)
    elif case == "two_parts":   # a part that cannot reach the hub
        n1, u1, v1 = gg.rmat(9, 8, 1)
        n2, u2, v2 = gg.bidirectional_star(50)
        n = n1 + n2
        u = np.concatenate([u1, u2 + n1]).astype(np.uint32)
        v = np.concatenate([v1, v2 + n1]).astype(np.uint32)
    else:
        n, u, v = 10, np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    g = bc.bc_build_csr(n, u, v)
    got = g.order()
    if case == "empty":
        assert got is None
        return
    order, rank = (x.numpy() for x in got)
    rp, col, cp, cr = (x.numpy() for x in g.arrays())
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.array_equal(rank[order], np.arange(n))
    active = int((np.diff(rp) > 0).sum())
    assert np.all(np.diff(rp)[order[:active]] > 0)
    assert np.array_equal(order, expected_order(n, rp, col, cp, cr))
