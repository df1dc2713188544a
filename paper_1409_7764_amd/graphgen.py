"""Seeded synthetic graph generators (inputs only; no betweenness arithmetic).

Every generator returns ``(n, src, dst)`` with ``src``/``dst`` as ``uint32``
numpy arrays describing a directed multigraph in COO form.  Self-loops and
duplicate pairs may be present in the R-MAT output on purpose: the method is
defined on simple digraphs, and both the device CSR builder and the CPU
oracle remove them on their own.

The paper's workloads are scale-free directed graphs (Barabasi-Albert
preferential attachment with each undirected edge replaced by two directed
ones, section II-C).  The headline workloads here are R-MAT graphs with the
usual (a, b, c, d) = (0.57, 0.19, 0.19, 0.05) quadrant split, which have the
same power-law out-degree skew; a random-orientation lattice stands in for
high-diameter graphs.  A small Barabasi-Albert generator is included for the
paper's own graph family.

This module is shared by the tests and the benchmark on both sides of the
parity check, so it holds input generation only.
"""
from __future__ import annotations

import numpy as np

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def _as_coo(n: int, u, v):
    return int(n), np.ascontiguousarray(u, dtype=np.uint32), np.ascontiguousarray(v, dtype=np.uint32)


def rmat(scale: int, edge_factor: int, seed: int, abcd=RMAT_ABCD, relabel: bool = True):
    """Directed R-MAT graph with ``n = 2**scale`` and ``edge_factor * n`` samples.

    Each sample picks one quadrant per bit: (0,0) with prob a, (0,1) with b,
    (1,0) with c, (1,1) with d; the source bit is set for c and d, the
    destination bit for b and d.  A seeded uniform relabelling of vertex ids
    follows, so hubs are not clustered at small ids.  No noise, no resampling
    of self-loops or duplicates.
    """
    a, b, c, d = abcd
    n = 1 << scale
    m = edge_factor * n
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.zeros(m, dtype=np.uint32)
    v = np.zeros(m, dtype=np.uint32)
    t_ab, t_abc = a + b, a + b + c
    for bit in range(scale):
        r = rng.random(m, dtype=np.float32)
        src_bit = r >= t_ab                      # quadrants c, d
        dst_bit = ((r >= a) & (r < t_ab)) | (r >= t_abc)   # quadrants b, d
        u |= src_bit.astype(np.uint32) << np.uint32(bit)
        v |= dst_bit.astype(np.uint32) << np.uint32(bit)
        del r, src_bit, dst_bit
    if relabel:
        perm = rng.permutation(n).astype(np.uint32)
        u = perm[u]
        v = perm[v]
    return _as_coo(n, u, v)


def grid_random_orientation(rows: int, cols: int, seed: int):
    """Lattice ``rows x cols`` (id = r*cols + c), each lattice edge oriented at random (p = 1/2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r, c = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64), indexing="ij")
    ids = r * cols + c
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    a = np.concatenate([hu, vu])
    b = np.concatenate([hv, vv])
    flip = rng.random(a.shape[0]) < 0.5
    u = np.where(flip, b, a)
    v = np.where(flip, a, b)
    return _as_coo(rows * cols, u, v)


def uniform_sources(n: int, k: int, seed: int):
    """``k`` distinct vertex ids drawn uniformly from [0, n) without replacement (k capped at n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = min(int(k), int(n))
    return np.ascontiguousarray(rng.choice(n, size=k, replace=False).astype(np.uint32))


def random_digraph(n: int, m: int, seed: int, allow_loops: bool = True):
    """Uniform random multigraph with ``m`` sampled pairs (may hold loops / duplicates)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.integers(0, n, size=m)
    v = rng.integers(0, n, size=m)
    if not allow_loops:
        keep = u != v
        u, v = u[keep], v[keep]
    return _as_coo(n, u, v)


def barabasi_albert(n: int, beta: int, seed: int):
    """Preferential attachment: each new vertex links to ``beta`` distinct earlier vertices
    chosen with probability proportional to degree; each undirected edge becomes two
    directed edges, so m = 2*beta*(n - beta) (section II-C)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    targets = list(range(beta))
    repeated: list[int] = []
    us, vs = [], []
    for src in range(beta, n):
        for t in targets:
            us.append(src); vs.append(t)
            us.append(t); vs.append(src)
        repeated.extend(targets)
        repeated.extend([src] * beta)
        chosen: set[int] = set()
        while len(chosen) < beta:
            chosen.add(repeated[int(rng.integers(0, len(repeated)))])
        targets = sorted(chosen)
    return _as_coo(n, us, vs)


# --- small structured graphs with closed-form answers -----------------------------------

def directed_path(n: int):
    i = np.arange(n - 1)
    return _as_coo(n, i, i + 1)


def directed_cycle(n: int):
    i = np.arange(n)
    return _as_coo(n, i, (i + 1) % n)


def bidirectional_star(n: int, centre: int = 0):
    leaves = np.array([x for x in range(n) if x != centre])
    c = np.full(leaves.shape, centre)
    return _as_coo(n, np.concatenate([c, leaves]), np.concatenate([leaves, c]))


def out_star(n: int, centre: int = 0):
    leaves = np.array([x for x in range(n) if x != centre])
    return _as_coo(n, np.full(leaves.shape, centre), leaves)


def complete_digraph(n: int):
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = u != v
    return _as_coo(n, u[keep], v[keep])


def grid_dag(rows: int, cols: int):
    """Monotone lattice DAG: edges (r,c)->(r,c+1) and (r,c)->(r+1,c); id = r*cols + c."""
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    ids = r * cols + c
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return _as_coo(rows * cols, u, v)


def diamond_chain(k: int):
    """s=0 -> {a,b} -> j1 -> {a,b} -> j2 ... ; joint j_i has 2**i shortest paths from s.

    Vertex ids: joints are 3*i (i = 0..k), the two middle vertices of diamond i are
    3*i+1 and 3*i+2.  n = 3*k + 1.
    """
    us, vs = [], []
    for i in range(k):
        j, a, b, nxt = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        us += [j, j, a, b]
        vs += [a, b, nxt, nxt]
    return _as_coo(3 * k + 1, us, vs)


def wide_diamond_forest(copies: int, width: int, k: int):
    """`copies` chains of `k` diamonds with `width` middle vertices each; the last joint of
    every chain feeds one shared sink, which has one out-edge to a tail vertex.  Joint i of a
    chain has width**i shortest paths from the chain's first joint, while every vertex
    reaches the sink within 2k + 1 steps (a shallow graph with large path counts; the sink is
    the vertex of largest in-degree among those with out-edges).

    Chain c starts at b = c * (k * (width + 1) + 1): joint i is b + i * (width + 1), the
    middles of diamond i are b + i * (width + 1) + 1 .. + width.  The sink is vertex
    copies * (k * (width + 1) + 1), the tail the next one; n = that + 2.
    """
    per = k * (width + 1) + 1
    sink = copies * per
    us, vs = [], []
    for c in range(copies):
        b = c * per
        for i in range(k):
            j = b + i * (width + 1)
            nxt = j + width + 1
            for t in range(1, width + 1):
                us += [j, j + t]
                vs += [j + t, nxt]
        us.append(b + k * (width + 1))
        vs.append(sink)
    us.append(sink)
    vs.append(sink + 1)
    return _as_coo(sink + 2, us, vs)
