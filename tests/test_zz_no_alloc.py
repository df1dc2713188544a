"""The allocation-free entry point (bc_sampled_noalloc) against bc_sampled on the same kernel
(one source per workgroup, state in global memory), through the C ABI (GPU only).

Two and more calls in a row share the library's fixed per-device array, each later call on a
smaller graph than the one before, so a call that left its predecessor's state behind, or sized
its slots by the previous graph, shows up as a difference."""
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


def np_of(t):
    return t.detach().cpu().numpy()


def test_noalloc_equals_bc_sampled_on_calls_in_a_row(bc):
    import torch
    cases = [
        ("rmat14 (relabelled copy)", gg.rmat(14, 8, 21), 400),
        ("lattice 64x64 (counts past 2^64)", gg.grid_random_orientation(64, 64, 1), None),
        ("rmat10", gg.rmat(10, 8, 10), 100),
    ]
    per_source = bc.tuning(batched=-1, lds_max_n=-1)
    for rep in range(2):
        for name, (n, u, v), k in cases:
            say("noalloc", rep, name)
            g = bc.bc_build_csr(n, u, v)
            if k is None:
                S = np.arange(n, dtype=np.uint32)
            else:
                S = gg.uniform_sources(n, k, 5 + rep)
                S = np.concatenate([S, S[:7], np.zeros(2, np.uint32)])   # repeats: multiset
            out = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
            bc.bc_sampled_noalloc(g, S, out)
            torch.cuda.synchronize()
            got = np_of(out)
            want_dev = np_of(bc.bc_sampled(g, S, tuning=per_source))
            rel_close(got, want_dev, what=f"{name}: noalloc vs bc_sampled")
            want, _, _ = oracle.bc(oracle.Graph(n, u, v), S)
            rel_close(got, want, what=f"{name}: noalloc vs oracle")
            g.free()


def test_noalloc_empty_and_limits(bc):
    import torch
    n, u, v = gg.rmat(9, 8, 3)
    g = bc.bc_build_csr(n, u, v)
    out = torch.full((n,), 5.0, dtype=torch.float64, device="cuda")
    bc.bc_sampled_noalloc(g, np.zeros(0, np.uint32), out)
    torch.cuda.synchronize()
    assert np_of(out).tolist() == [0.0] * n
    g.free()
    # one vertex past the largest graph whose single state slot fits the fixed array
    big = 1_398_080
    g = bc.bc_build_csr(big, np.array([0, 1, 2], np.uint32), np.array([1, 2, 3], np.uint32))
    out = torch.empty(big, dtype=torch.float64, device="cuda")
    with pytest.raises(bc.BcError) as e:
        bc.bc_sampled_noalloc(g, np.array([0], np.uint32), out)
    assert e.value.code == bc.BC_E_RANGE and "1398079" in str(e.value)
    g.free()
    g = bc.bc_build_csr(big - 1, np.array([0, 1, 2], np.uint32), np.array([1, 2, 3], np.uint32))
    out = torch.full((big - 1,), 5.0, dtype=torch.float64, device="cuda")
    bc.bc_sampled_noalloc(g, np.array([0, 0, 1], np.uint32), out)
    torch.cuda.synchronize()
    got = np_of(out)
    # from 0: 1, 2 interior on the path 0->1->2->3 (twice); from 1: 2 interior once
    assert got[:4].tolist() == [0.0, 4.0, 3.0, 0.0] and not got[4:].any()
    g.free()
