"""Serving on the GPU: every request's result is the same alone and in the mix (bit for bit), and
equals the one-colouring count (exact below 2^53, 1e-12 relative above)."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone(dev):
    import torch
    import paper_1804_09764_amd as cc
    from paper_1804_09764_amd.serving import GpuExecutor, Request, Server, latency_summary

    pool = [cc.Graph.from_numpy(*inputs.rmat_graph(s, ef, 100 + i), hub_threshold=256, chunk=128)
            for i, (s, ef) in enumerate([(10, 8), (11, 16), (12, 8), (9, 32)])]
    rng = np.random.default_rng(4)
    reqs = []
    for rid in range(14):
        k = int(rng.integers(5, 10))
        reqs.append(Request(rid=rid, graph_id=int(rng.integers(0, len(pool))), tree_edges=inputs.pruefer_tree(k, rid),
                            B=int(rng.integers(2, 7)), seed=rid, arrival=0.002 * rid))
    ex = GpuExecutor(pool, seed_base=50)
    budget = 3 * max(ex.slot_bytes(r) for r in reqs)
    srv = Server(ex, memory_budget=budget, max_inflight=2, max_colourings_per_batch=8)
    print(f"case: serving 14 requests, budget {budget} bytes", flush=True)
    done = srv.run(reqs)
    assert all(r.status == "done" for r in done), [(r.rid, r.status, r.error) for r in done]
    assert srv.stats.batches > 1 and srv.stats.max_inflight_bytes <= budget
    for r in reqs:
        g = pool[r.graph_id]
        P = cc.Plan(r.tree_edges)
        C = cc.colour(g, P.k, seed=50 + r.seed, first_iter=0, B=r.B)
        X = cc.count_packed(P, g, C)
        Xs = cc.count(P, g, C)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(r.X, X.cpu().numpy())
        xs = Xs.cpu().numpy()
        small = xs < 2.0 ** 53
        np.testing.assert_array_equal(r.X[small], xs[small])
        assert np.all(np.abs(r.X[~small] - xs[~small]) <= 1e-12 * xs[~small])
        est, _ = cc.estimate(P, X.cpu().numpy())
        assert r.estimate == est
    s = latency_summary(reqs)
    assert s["n"] == 14 and s["p99_s"] >= s["p50_s"] > 0
