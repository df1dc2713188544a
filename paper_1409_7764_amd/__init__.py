"""bcmi: Brandes betweenness centrality on AMD MI355X (gfx950).

``bcmi``      -- binding of the C ABI in include/bc.h (libbcmi.so, HIP kernels)
``graphgen``  -- seeded synthetic input graphs (R-MAT, lattices, closed-form families)
"""
