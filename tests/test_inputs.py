"""The seeded input recipes (CPU only): the same seed gives the same graph or source list,
and each generator produces the structure its recipe states."""
import numpy as np

from paper_1409_7764_amd import graphgen as gg


def test_rmat_is_seeded_and_sized():
    n, u, v = gg.rmat(10, 8, 3)
    n2, u2, v2 = gg.rmat(10, 8, 3)
    assert n == n2 == 1024 and len(u) == len(v) == 8 * 1024
    assert np.array_equal(u, u2) and np.array_equal(v, v2)
    _, u3, _ = gg.rmat(10, 8, 4)
    assert not np.array_equal(u, u3)
    assert u.max() < n and v.max() < n


def test_rmat_quadrant_probabilities():
    """Without the final relabelling, every bit of a sample is a quadrant draw: the source bit
    is set with probability c + d, the destination bit with b + d, both with d."""
    a, b, c, d = gg.RMAT_ABCD
    scale = 12
    _, u, v = gg.rmat(scale, 16, 9, relabel=False)
    m = len(u)
    for bit in range(scale):
        su = (u >> bit) & 1
        sv = (v >> bit) & 1
        se = 4 * np.sqrt(0.25 / m)   # four standard errors at worst
        assert abs(su.mean() - (c + d)) < se
        assert abs(sv.mean() - (b + d)) < se
        assert abs((su & sv).mean() - d) < se


def test_grid_orientation():
    rows, cols = 13, 17
    n, u, v = gg.grid_random_orientation(rows, cols, 1)
    assert n == rows * cols and len(u) == rows * (cols - 1) + cols * (rows - 1)
    ru, cu = u // cols, u % cols
    rv, cv = v // cols, v % cols
    assert np.all(np.abs(ru.astype(int) - rv) + np.abs(cu.astype(int) - cv) == 1)   # lattice neighbours
    und = np.sort(np.stack([u, v]), axis=0)
    assert len(np.unique(und[0].astype(np.int64) * n + und[1])) == len(u)             # each edge once
    forward = (u < v).mean()
    assert 0.4 < forward < 0.6
    assert np.array_equal(u, gg.grid_random_orientation(rows, cols, 1)[1])


def test_uniform_sources():
    s = gg.uniform_sources(1000, 300, 5)
    assert len(s) == 300 and len(np.unique(s)) == 300 and s.max() < 1000 and s.dtype == np.uint32
    assert np.array_equal(s, gg.uniform_sources(1000, 300, 5))
    assert not np.array_equal(s, gg.uniform_sources(1000, 300, 6))
    assert np.array_equal(np.sort(gg.uniform_sources(50, 80, 1)), np.arange(50))      # capped at n
