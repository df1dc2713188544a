"""Serving and autotuning through the C ABI (GPU only): every request's result is the same
alone and in the mix (1e-9), and matches the oracle; requests that arrive while others run
overlap with them on the device; admission by footprint holds requests back or rejects them."""
import time

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


def wait(bc, srv, ticket, timeout=120.0):
    t0 = time.time()
    while True:
        info = bc.bc_serve_poll(srv, ticket)
        if info is not None:
            return info
        assert time.time() - t0 < timeout, "request did not finish"
        time.sleep(0.0005)


def msb_team_bytes(n):
    """Device state of one batched team: control block, masks 16n + counts 256n + psi 512n,
    bnx 8n, level masks of pulled levels 16n, staggers, level lists (8n + 64 entries of 20 B)
    and 1026 level offsets."""
    cap = 8 * n + 64
    return 128 + n * (16 + 8 + 16 + 256 + 512) + 5 * 37 * 512 * 8 + cap * 20 + 4 * (1024 + 2)


def footprint(n, m, k, path):
    """Admission footprint: CSR + CSC + output, plus the state of the request's path."""
    f = 2 * (4 * (n + 1) + 4 * m) + 8 * n
    if path == "global":
        f += min(k, 64) * (24 * n + 4)
    elif path == "batched":
        f += min((k + 63) // 64, 64) * msb_team_bytes(n)
    return f


def test_serve_alone_equals_mix(bc):
    import torch
    specs = [(6, 8, 1), (9, 4, 2), (12, 16, 3), (13, 8, 4), (14, 4, 5)]
    graphs, coo = [], []
    for sc, ef, seed in specs:
        n, u, v = gg.rmat(sc, ef, seed)
        graphs.append(bc.bc_build_csr(n, u, v))
        coo.append((n, u, v))
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(24):
        gi = int(rng.integers(0, len(graphs)))
        n = graphs[gi].n
        if rng.random() < 0.5 and n <= 4096:
            reqs.append((gi, None))
        else:
            reqs.append((gi, gg.uniform_sources(n, int(rng.integers(1, 300)), 100 + i)))
    # fewer than 64 sources on the larger graphs: one source per workgroup in global slots
    reqs += [(3, gg.uniform_sources(graphs[3].n, 10, 500)), (4, gg.uniform_sources(graphs[4].n, 37, 501))]
    alone = []
    for gi, S in reqs:
        g = graphs[gi]
        out = bc.bc_exact(g) if S is None else bc.bc_sampled(g, S)
        alone.append(out.cpu().numpy())
    srv = bc.bc_serve_create(64 << 30)
    outs = [torch.full((graphs[gi].n,), -1.0, dtype=torch.float64, device="cuda") for gi, _ in reqs]
    tickets = [bc.bc_serve_submit(srv, graphs[gi], S, out) for (gi, S), out in zip(reqs, outs)]
    infos = [wait(bc, srv, t) for t in tickets]
    assert {inf["path"] for inf in infos} == {0, 1, 2}   # LDS, global slots and batched in one mix
    for i, ((gi, S), out, inf) in enumerate(zip(reqs, outs, infos)):
        got = out.cpu().numpy()
        rel_close(got, alone[i], what=f"request {i} alone vs mix")
        k = graphs[gi].n if S is None else len(S)
        assert inf["n_sources"] == k
        assert inf["t_submit_ms"] <= inf["t_start_ms"] <= inf["t_done_ms"]
    # oracle on a few of them
    for i in [0, 1, 2, 3]:
        gi, S = reqs[i]
        n, u, v = coo[gi]
        want, _, _ = oracle.bc(oracle.Graph(n, u, v), S)
        rel_close(outs[i].cpu().numpy(), want, what=f"request {i} vs oracle")
    bc.bc_serve_destroy(srv)
    for g in graphs:
        g.free()


def test_serve_overlap_and_continuous_batching(bc):
    import torch
    n, u, v = gg.rmat(15, 16, 7)
    big = bc.bc_build_csr(n, u, v)
    n2, u2, v2 = gg.rmat(8, 8, 8)
    small = bc.bc_build_csr(n2, u2, v2)
    srv = bc.bc_serve_create(64 << 30)
    out_a = torch.empty(big.n, dtype=torch.float64, device="cuda")
    out_b = torch.empty(small.n, dtype=torch.float64, device="cuda")
    SA = np.tile(gg.uniform_sources(big.n, big.n, 1), 4)   # a multiset of 8 batched chunks
    ta = bc.bc_serve_submit(srv, big, SA, out_a)   # spans many ticks
    time.sleep(0.005)
    tb = bc.bc_serve_submit(srv, small, None, out_b)
    ib = wait(bc, srv, tb)
    ia = wait(bc, srv, ta)
    # B arrived while A was on the device, joined a tick before A finished, and finished first
    assert ib["t_submit_ms"] < ia["t_done_ms"]
    assert ib["t_start_ms"] < ia["t_done_ms"]
    assert ib["t_done_ms"] < ia["t_done_ms"]
    want_b, _, _ = oracle.bc(oracle.Graph(n2, u2, v2))
    rel_close(out_b.cpu().numpy(), want_b)
    rel_close(out_a.cpu().numpy(), bc.bc_sampled(big, SA).cpu().numpy())
    bc.bc_serve_destroy(srv)
    big.free()
    small.free()


def test_serve_batched_with_hand_off(bc):
    """An exact request on a shallow 5,482-vertex graph runs as batched chunks; sources whose
    counts pass 32 bits are handed to the per-source kernel within the same tick."""
    import torch
    n, u, v = gg.wide_diamond_forest(40, 16, 8)
    g = bc.bc_build_csr(n, u, v)
    srv = bc.bc_serve_create(64 << 30)
    out = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    info = wait(bc, srv, bc.bc_serve_submit(srv, g, None, out))
    assert info["path"] == 2 and info["n_sources"] == n
    want, _, _ = oracle.bc(oracle.Graph(n, u, v))
    rel_close(out.cpu().numpy(), want, what="served batched with hand-off")
    bc.bc_serve_destroy(srv)
    g.free()


def test_serve_admission_budget(bc):
    import torch
    n, u, v = gg.rmat(13, 8, 9)
    g = bc.bc_build_csr(n, u, v)
    f = footprint(g.n, g.m, 512, path="batched")   # 512 sources on an 8192-vertex R-MAT: batched
    srv = bc.bc_serve_create(int(1.5 * f))       # room for one request at a time
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in range(3)]
    S = [gg.uniform_sources(g.n, 512, 20 + i) for i in range(3)]
    ts = [bc.bc_serve_submit(srv, g, S[i], outs[i]) for i in range(3)]
    infos = [wait(bc, srv, t) for t in ts]
    assert all(i["path"] == 2 for i in infos)
    for a, b in zip(infos, infos[1:]):
        assert b["t_start_ms"] >= a["t_done_ms"]       # admitted only after the previous one left
    for i in range(3):
        rel_close(outs[i].cpu().numpy(), bc.bc_sampled(g, S[i]).cpu().numpy())
    tiny = bc.bc_serve_create(f // 2)
    with pytest.raises(bc.BcError) as e:       # larger than the whole budget
        bc.bc_serve_submit(tiny, g, None, outs[0])
    assert e.value.code == bc.BC_E_NOMEM
    bc.bc_serve_destroy(tiny)
    with pytest.raises(bc.BcError) as e:
        bc.bc_serve_submit(srv, g, np.array([g.n], np.uint32), outs[0])
    assert e.value.code == bc.BC_E_RANGE
    bc.bc_serve_destroy(srv)
    g.free()


def test_serve_destroy_with_work_queued(bc):
    import torch
    n, u, v = gg.rmat(12, 8, 11)
    g = bc.bc_build_csr(n, u, v)
    srv = bc.bc_serve_create(footprint(g.n, g.m, 64, False) * 2)
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in range(8)]
    for i in range(8):
        bc.bc_serve_submit(srv, g, gg.uniform_sources(g.n, 64, i), outs[i])
    bc.bc_serve_destroy(srv)      # cancels what was not admitted, finishes what runs
    g.free()


def test_autotune_keeps_results(bc):
    n, u, v = gg.rmat(14, 16, 12)
    g = bc.bc_build_csr(n, u, v)
    S = gg.uniform_sources(n, 200, 3)
    before = bc.bc_sampled(g, S).cpu().numpy()
    t = bc.bc_tune(g)
    assert t["wg_size"] in (64, 128, 256, 512, 1024)
    after, info = bc.bc_sampled(g, S, tuning=bc.tuning(**t), info=True)
    rel_close(after.cpu().numpy(), before, 1e-12)
    n2, u2, v2 = gg.rmat(9, 8, 12)
    g2 = bc.bc_build_csr(n2, u2, v2)
    t2 = bc.bc_tune(g2)
    assert t2["batched"] == -1          # small graphs stay on the LDS-resident path
    want, _, _ = oracle.bc(oracle.Graph(n2, u2, v2))
    rel_close(bc.bc_exact(g2).cpu().numpy(), want)
    g.free()
    g2.free()


def test_batch_resolves_tuned_knobs_per_class(bc):
    """bc_batch resolves each graph's knobs from the tuner's entry for its size class: after
    tuning one graph of two classes, a batch mixing them (and an untuned class) still equals
    the oracle, and equals the batch run before tuning."""
    import torch
    specs = [(9, 8, 300 + i) for i in range(6)] + [(11, 8, 310 + i) for i in range(4)] + [(13, 8, 320), (13, 8, 321)]
    graphs, wants = [], []
    for sc, ef, seed in specs:
        n, u, v = gg.rmat(sc, ef, seed)
        graphs.append(bc.bc_build_csr(n, u, v))
        wants.append(oracle.bc(oracle.Graph(n, u, v))[0])
    before = bc.bc_batch(graphs)
    torch.cuda.synchronize()
    for o, w in zip(before, wants):
        rel_close(o.cpu().numpy(), w, what="batch before tuning")
    bc.bc_tune(graphs[0])     # class of the scale-9 graphs (LDS-resident)
    bc.bc_tune(graphs[-1])    # class of the scale-13 graphs (global slots or batched candidates)
    for rep in range(2):      # a new plan, then its replay
        after, infos = bc.bc_batch(graphs, info=True)
        torch.cuda.synchronize()
        for i, (o, b, w) in enumerate(zip(after, before, wants)):
            rel_close(o.cpu().numpy(), w, what=f"batch after tuning, graph {i}")
            rel_close(o.cpu().numpy(), b.cpu().numpy(), 1e-11, what=f"tuned vs default, graph {i}")
            assert infos[i]["n_sources"] == graphs[i].n
    for g in graphs:
        g.free()


@pytest.mark.slow
def test_serve_bench_workload(bc):
    """The benchmark's served stream, replayed: 256 requests over a pool of 64 resident R-MAT
    graphs (scales 8 to 18, log-uniform n; edge factors 4 to 16), 70 % exact and 30 % on 256
    sampled sources, submitted at the same Poisson arrival times (2,000 per second).  Every
    sampled request, and every exact request on a graph of scale <= 14, equals the oracle; an
    exact request on a larger graph (10^10 to 10^12 edge visits, beyond the oracle's reach here)
    equals the same graph's bc_exact run alone, outside the server, which the oracle pins on
    other graphs."""
    import torch
    rng = np.random.default_rng(5)
    pool, coo, scales = [], [], []
    for i in range(64):
        sc = int(rng.integers(8, 19))
        ef = int(rng.integers(4, 17))
        n, u, v = gg.rmat(sc, ef, 5000 + i)
        coo.append((n, u, v))
        scales.append(sc)
        pool.append(bc.bc_build_csr(n, u, v))
    arrive = np.cumsum(rng.exponential(1.0 / 2000.0, size=256))
    reqs = []
    for i in range(256):
        gi = int(rng.integers(0, len(pool)))
        if rng.random() < 0.7:
            reqs.append((gi, None))
        else:
            reqs.append((gi, gg.uniform_sources(pool[gi].n, min(256, pool[gi].n), 77 + i)))
    outs = [torch.full((pool[gi].n,), -1.0, dtype=torch.float64, device="cuda") for gi, _ in reqs]
    torch.cuda.synchronize()
    srv = bc.bc_serve_create(200 << 30)
    tickets = []
    t0 = time.perf_counter()
    for (gi, S), out, at in zip(reqs, outs, arrive):
        while time.perf_counter() - t0 < at:
            pass
        tickets.append(bc.bc_serve_submit(srv, pool[gi], S, out))
    print("served stream: submitted", flush=True)
    infos = [wait(bc, srv, t, timeout=600.0) for t in tickets]
    bc.bc_serve_destroy(srv)
    print("served stream: done; checking", flush=True)
    exact = {}
    for i, ((gi, S), out, inf) in enumerate(zip(reqs, outs, infos)):
        n, u, v = coo[gi]
        if S is None:
            if gi not in exact:
                if scales[gi] <= 14:
                    exact[gi] = oracle.bc(oracle.Graph(n, u, v))[0]
                else:
                    exact[gi] = bc.bc_exact(pool[gi]).cpu().numpy()
            want = exact[gi]
        else:
            want = oracle.bc(oracle.Graph(n, u, v), S)[0]
        assert inf["n_sources"] == (n if S is None else len(S))
        rel_close(out.cpu().numpy(), want,
                  what=f"request {i} (graph {gi}, scale {scales[gi]}, {'exact' if S is None else 'sampled'})")
    for g in pool:
        g.free()
