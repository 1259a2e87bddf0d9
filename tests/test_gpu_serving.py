"""Serving on the GPU: every served colouring count equals the oracle's (exact below 2^53, 1e-12
relative above), every request's result is the same alone and in the mix (bit for bit), and the
per-batch cap on a request's colourings (which relieves head-of-line blocking) changes no value."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TWO53 = float(2 ** 53)
SEED_BASE = 50
POOL = [(10, 8), (11, 16), (12, 8), (9, 32)]


def _pool(cc):
    graphs, host = [], []
    for i, (s, ef) in enumerate(POOL):
        rp, cl = inputs.rmat_graph(s, ef, 100 + i)
        host.append((rp, cl))
        graphs.append(cc.Graph.from_numpy(rp, cl, hub_threshold=256, chunk=128))
    return graphs, host


def _requests(n=14, seed=4):
    from paper_1804_09764_amd.serving import Request
    rng = np.random.default_rng(seed)
    reqs = []
    for rid in range(n):
        k = int(rng.integers(5, 10))
        reqs.append(Request(rid=rid, graph_id=int(rng.integers(0, len(POOL))), tree_edges=inputs.pruefer_tree(k, rid),
                            B=int(rng.integers(2, 7)), seed=rid, arrival=0.002 * rid))
    return reqs


def _serve(cc, pool, reqs, cap):
    from paper_1804_09764_amd.serving import GpuExecutor, Server
    ex = GpuExecutor(pool, seed_base=SEED_BASE)
    budget = 3 * max(ex.slot_bytes(r) for r in reqs)
    srv = Server(ex, memory_budget=budget, max_inflight=2, max_colourings_per_batch=8, slot_colourings=cap)
    print(f"case: serving {len(reqs)} requests, budget {budget} bytes, cap {cap}", flush=True)
    done = srv.run(reqs)
    assert all(r.status == "done" for r in done), [(r.rid, r.status, r.error) for r in done]
    assert srv.stats.batches > 1 and srv.stats.max_inflight_bytes <= budget
    return srv


def test_served_results_equal_oracle_and_alone(dev):
    import torch
    import paper_1804_09764_amd as cc
    from paper_1804_09764_amd.serving import latency_summary

    pool, host = _pool(cc)
    reqs = _requests()
    _serve(cc, pool, reqs, cap=0)
    for r in reqs:
        g = pool[r.graph_id]
        rp, cl = host[r.graph_id]
        P = cc.Plan(r.tree_edges)
        # the oracle: the request's colourings (the hash colouring of its seed), Eq. 1 on the host
        Xo = np.array([oracle.count(rp, cl, oracle.colour(SEED_BASE + r.seed, b, g.n, P.k), r.tree_edges)
                       for b in range(r.B)])
        small = Xo < TWO53
        np.testing.assert_array_equal(r.X[small], Xo[small])
        assert np.all(np.abs(r.X[~small] - Xo[~small]) <= 1e-12 * Xo[~small])
        # alone: the same colourings in one packed count of their own
        C = cc.colour(g, P.k, seed=SEED_BASE + r.seed, first_iter=0, B=r.B)
        X = cc.count_packed(P, g, C)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(r.X, X.cpu().numpy())
        est, _ = cc.estimate(P, X.cpu().numpy())
        assert r.estimate == est
    s = latency_summary(reqs)
    assert s["n"] == 14 and s["p99_s"] >= s["p50_s"] > 0


def test_slot_cap_changes_no_value(dev):
    import paper_1804_09764_amd as cc
    pool, _ = _pool(cc)
    a = _requests()
    b = _requests()
    _serve(cc, pool, a, cap=0)
    srv = _serve(cc, pool, b, cap=2)
    assert max(srv.stats.batch_sizes) <= 8
    for ra, rb in zip(a, b):
        np.testing.assert_array_equal(ra.X, rb.X)
        assert ra.estimate == rb.estimate
