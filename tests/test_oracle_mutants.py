"""Plant mistakes in a copy of the CPU oracle and check that the pins catch each one.

The copy lives in a temporary directory; the committed oracle is never modified.  Every
mutant is a plausible slip (a dropped term, a transposed operand, a wrong index or
comparison, a missing endpoint exclusion, a missing de-duplication or overflow check); the
unmodified copy must pass the same checks.
"""
import importlib.util
import math
import os
import shutil
import sys
from fractions import Fraction

import numpy as np
import pytest

from paper_1409_7764_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "drop_one_plus_delta": ("(1.0 + delta[w])", "(delta[w])"),
    "transposed_sigma_ratio": ("(sigma_f[v] / sigma_f[w])", "(sigma_f[w] / sigma_f[v])"),
    "endpoint_included": ("if ((uint32_t)v != s) mine[v] += delta[v];", "mine[v] += delta[v];"),
    "successor_test_ge": ("            if (dist[w] == dist[v] + 1)\n                acc",
                          "            if (dist[w] >= dist[v])\n                acc"),
    "no_dedup": ("if (i > 0 && pairs[i] == pairs[i - 1]) continue;", ""),
    "no_overflow_flag": ("&sum)) *overflow = 1;", "&sum)) {}"),
    "dist_plus_two": ("dist[w] = dist[v] + 1;", "dist[w] = dist[v] + 2;"),
    "double_count_adds_one": ("sigma_f[w] += sigma_f[v];", "sigma_f[w] += 1.0;"),
    "forward_order_accumulation": ("for (int64_t i = count - 1; i >= 0; --i) {",
                                   "for (int64_t i = 0; i < count; ++i) {"),
    # slips in the per-source work counters
    "levels_off_by_one": ("st->levels = (int64_t)deepest + 1;", "st->levels = (int64_t)deepest;"),
    "reached_excludes_source": ("st->reached = tail;", "st->reached = tail - 1;"),
    "dag_counted_before_test": ("            if (dist[w] == dist[v] + 1) {         /* (v,w) lies on a shortest path */\n"
                                "                ++dag;",
                                "            ++dag;\n"
                                "            if (dist[w] == dist[v] + 1) {"),
    "dag_counted_on_first_visit": ("                order[tail++] = w;\n", "                order[tail++] = w;\n                ++dag;\n"),
    "examined_per_vertex": [("            ++examined;\n", ""),
                            ("        uint32_t v = order[head++];\n", "        uint32_t v = order[head++];\n        ++examined;\n")],
    "recount_adds_counters": ("st->examined = examined;", "st->examined += examined;"),
}


def _load_copy(tmp, name, mutation):
    dst = os.path.join(tmp, name)
    shutil.copytree(os.path.join(ROOT, "oracle"), dst,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = os.path.join(dst, "brandes.c")
    text = open(src).read()
    if mutation is not None:
        for old, new in (mutation if isinstance(mutation, list) else [mutation]):
            assert text.count(old) == 1, f"mutation anchor not unique: {old!r}"
            text = text.replace(old, new)
        open(src, "w").write(text)
    spec = importlib.util.spec_from_file_location(name, os.path.join(dst, "__init__.py"),
                                                  submodule_search_locations=[dst])
    mod = importlib.util.module_from_spec(spec)
    sys.modules[name] = mod
    spec.loader.exec_module(mod)
    return mod


def _pin_failures(orc):
    from oracle.brute import brute_force
    fails = []

    def check(name, ok):
        if not ok:
            fails.append(name)

    def close(x, y, tol=1e-12):
        x, y = np.asarray(x, float), np.asarray(y, float)
        if x.shape != y.shape:
            return False
        z = y == 0
        return bool(np.all(x[z] == 0) and np.all(np.abs(x[~z] - y[~z]) <= tol * np.abs(y[~z])))

    # brute force on small random inputs with loops and duplicates
    rng = np.random.default_rng(99)
    for t in range(40):
        n = int(rng.integers(2, 7))
        m = int(rng.integers(1, 3 * n + 1))
        u, v = rng.integers(0, n, size=m), rng.integers(0, n, size=m)
        dist, sigma, bcx = brute_force(n, u, v)
        g = orc.Graph(n, u, v)
        check("brute_bc", close(orc.bc(g, threads=1)[0], [float(x) for x in bcx]))
        for s in range(n):
            r = orc.brandes_source(g, s)
            check("brute_dist", r["dist"].tolist() == dist[s])
            check("brute_sigma", r["sigma"].tolist() == sigma[s])
    # closed forms
    n = 9
    check("path", orc.bc(orc.Graph(*gg.directed_path(n)))[0].tolist() == [i * (n - 1 - i) for i in range(n)])
    check("star", orc.bc(orc.Graph(*gg.bidirectional_star(n)))[0].tolist() == [(n - 1) * (n - 2)] + [0] * (n - 1))
    g = orc.Graph(*gg.diamond_chain(64))
    check("diamond_overflow", orc.brandes_source(g, 0)["overflow"])
    g = orc.Graph(*gg.grid_dag(35, 35))
    r = orc.brandes_source(g, 0)
    want = [float(math.comb(i + j, i)) for i in range(35) for j in range(35)]
    check("grid_sigma_f", close(r["sigma_f"], want, 1e-13))
    # work counters: closed form on the overflowing grid DAG (every vertex reached, every
    # edge examined and on a shortest path, 69 levels), and the definitions on scipy's BFS
    # distances for every source of a small R-MAT graph
    check("grid_counters", (r["reached"], r["examined"], r["dag_edges"], r["levels"]) == (1225, 2380, 2380, 69))
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    n, u, v = gg.rmat(7, 8, 1)
    g = orc.Graph(n, u, v)
    a = csr_matrix((np.ones(g.m), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(n, n))
    d = shortest_path(a, method="D", directed=True, unweighted=True)
    _, _, stats = orc.bc(g, threads=2)
    outdeg = np.diff(g.row_ptr.astype(np.int64))
    src = np.repeat(np.arange(n), outdeg)
    col = g.col.astype(np.int64)
    for s in range(n):
        fin = np.isfinite(d[s])
        dag = int(np.sum(fin[src] & fin[col] & (d[s][col] == d[s][src] + 1)))
        want = [int(fin.sum()), int(outdeg[fin].sum()), dag, int(d[s][fin].max()) + 1]
        check("counters", stats[s].tolist() == want)
    return sorted(set(fails))


@pytest.fixture(scope="module")
def tmpdir_mod(tmp_path_factory):
    return str(tmp_path_factory.mktemp("oracle_mutants"))


def test_pristine_copy_passes(tmpdir_mod):
    orc = _load_copy(tmpdir_mod, "oracle_pristine", None)
    assert _pin_failures(orc) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmpdir_mod, name):
    orc = _load_copy(tmpdir_mod, "oracle_mut_" + name, MUTANTS[name])
    assert _pin_failures(orc), f"mutant {name} survived every pin"
