"""Shared test utilities (comparison rules and an independent BFS certificate)."""
import numpy as np

BC_RTOL = 1e-9   # relative tolerance on FP64 dependencies and BC (all terms are >= 0)


def rel_close(got, want, tol=BC_RTOL, what="value"):
    """|got - want| <= tol * |want| elementwise; where want == 0, got must be exactly 0."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    zero = want == 0
    bad = np.nonzero(got[zero] != 0)[0]
    assert bad.size == 0, f"{what}: {bad.size} structural zeros differ (first at {np.nonzero(zero)[0][bad[0]]})"
    nz = ~zero
    if nz.any():
        err = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
        i = int(np.argmax(err))
        assert err[i] <= tol, f"{what}: max rel err {err[i]:.3e} at {np.nonzero(nz)[0][i]}"


def certificate(n, row_ptr, col, s, dist, sigma):
    """O(m) validity check of BFS distances and shortest-path counts from s, independent of
    both implementations: dist[s] = 0; dist[w] <= dist[v] + 1 along every edge out of a
    reached v; every reached w != s has an in-neighbour one level up; sigma[w] equals the
    sum of sigma over those in-neighbours; unreached vertices have sigma 0."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    dist = np.asarray(dist, dtype=np.int64)
    sig = [int(x) for x in sigma]
    assert dist[s] == 0 and sig[s] == 1
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    reached_src = dist[src] >= 0
    u, w = src[reached_src], col[reached_src]
    assert np.all(dist[w] >= 0), "edge from a reached vertex to an unreached one"
    assert np.all(dist[w] <= dist[u] + 1), "distance not a BFS labelling"
    tight = dist[w] == dist[u] + 1
    acc = [0] * n
    has_parent = np.zeros(n, dtype=bool)
    for a, b in zip(u[tight].tolist(), w[tight].tolist()):
        acc[b] += sig[a]
        has_parent[b] = True
    for v in range(n):
        if v == s:
            continue
        if dist[v] < 0:
            assert sig[v] == 0
        else:
            assert has_parent[v], f"vertex {v} has no parent"
            assert acc[v] == sig[v], f"sigma recurrence fails at {v}"
