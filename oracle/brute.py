"""Exhaustive shortest-path enumeration for tiny digraphs -- TEST INFRASTRUCTURE ONLY.

Independent of Brandes' method: for every ordered pair (s, t), all simple s->t paths are
listed by depth-first search, the shortest ones are kept, and each interior vertex v is
credited sigma_st(v)/sigma_st as an exact rational -- the definition of betweenness in
section I of the paper, written out with no recurrence.  Exponential; meant for n <= 8.
"""
from __future__ import annotations

from fractions import Fraction


def _simple_edges(n, src, dst):
    adj = [set() for _ in range(n)]
    for u, v in zip(src, dst):
        u, v = int(u), int(v)
        if u != v:
            adj[u].add(v)
    return [sorted(a) for a in adj]


def _all_simple_paths(adj, s, t):
    out = []
    stack = [(s, [s])]
    while stack:
        v, path = stack.pop()
        if v == t:
            out.append(path)
            continue
        for w in adj[v]:
            if w not in path:
                stack.append((w, path + [w]))
    return out


def brute_force(n, src, dst):
    """Return (dist, sigma, bc): dist[s][t] (-1 unreachable, 0 on the diagonal), sigma[s][t]
    (Python ints, sigma[s][s] = 1), bc[v] (Fractions)."""
    adj = _simple_edges(n, src, dst)
    dist = [[-1] * n for _ in range(n)]
    sigma = [[0] * n for _ in range(n)]
    bc = [Fraction(0)] * n
    for s in range(n):
        dist[s][s] = 0
        sigma[s][s] = 1
        for t in range(n):
            if t == s:
                continue
            paths = _all_simple_paths(adj, s, t)
            if not paths:
                continue
            best = min(len(p) for p in paths)
            shortest = [p for p in paths if len(p) == best]
            dist[s][t] = best - 1
            sigma[s][t] = len(shortest)
            through = [0] * n
            for p in shortest:
                for v in p[1:-1]:
                    through[v] += 1
            for v in range(n):
                if through[v]:
                    bc[v] += Fraction(through[v], len(shortest))
    return dist, sigma, bc
