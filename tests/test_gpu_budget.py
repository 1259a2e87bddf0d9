"""Counts within a device-memory budget (cc_count_budget): tables idle across the peak are parked
in host memory and come back before their first reader. The kernels and their order are those of
cc_count, so the counts must be bit-identical to cc_count's and equal to the oracle."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TWO53 = float(2 ** 53)


def assert_parity(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    small = ref < TWO53
    np.testing.assert_array_equal(gpu[small], ref[small])
    if (~small).any():
        assert (np.abs(gpu[~small] - ref[~small]) / ref[~small]).max() <= 1e-12


@pytest.mark.parametrize("k,seed,scale", [(12, 12, 11), (15, 15, 9), (10, 3, 11)])
def test_budget_parks_tables_and_matches(dev, k, seed, scale):
    import torch
    import paper_1804_09764_amd as cc
    rp, cl = inputs.rmat_graph(scale, 16, 4)
    n = len(rp) - 1
    G = cc.Graph.from_numpy(rp, cl, hub_threshold=64, chunk=64)
    T = inputs.pruefer_tree(k, seed)
    P = cc.Plan(T)
    full = cc.count_workspace_bytes(P, G)
    info = cc.count_budget_plan(P, G, 1 << 62)
    assert info["parked_tables"] == 0 and info["workspace_bytes"] <= full
    # the smallest budget the parking can meet, found by bisection over the unbounded workspace
    lo, hi = 0, full
    while hi - lo > full // 64:
        mid = (lo + hi) // 2
        try:
            cc.count_budget_plan(P, G, mid)
            hi = mid
        except cc.CCError:
            lo = mid
    info = cc.count_budget_plan(P, G, hi)
    print(f"case: budget k={k} scale={scale}: {full} -> {info}", flush=True)
    assert info["parked_tables"] >= 1 and info["workspace_bytes"] <= hi < full
    assert info["arena_columns"] < info["unbounded_columns"]
    colours = cc.colour(G, k, seed=9, first_iter=0, B=2)
    X0, V0 = cc.count(P, G, colours, per_vertex=True)
    X1, V1 = cc.count_budget(P, G, colours, budget=hi, per_vertex=True)
    X2 = cc.count_budget(P, G, colours, budget=hi)  # root counts in the workspace
    torch.cuda.synchronize()
    np.testing.assert_array_equal(V1.cpu().numpy(), V0.cpu().numpy())
    np.testing.assert_array_equal(X1.cpu().numpy(), X0.cpu().numpy())
    np.testing.assert_array_equal(X2.cpu().numpy(), X0.cpu().numpy())
    Ch = colours.cpu().numpy()
    Xo, Vo = oracle.count(rp, cl, Ch[0], T, root=P.info.root, per_vertex=True)
    assert_parity(V1.cpu().numpy()[0], Vo)
    assert_parity([float(X1.cpu()[0])], [Xo])


def test_budget_too_small_is_refused(dev):
    import paper_1804_09764_amd as cc
    rp, cl = inputs.rmat_graph(10, 16, 4)
    G = cc.Graph.from_numpy(rp, cl)
    P = cc.Plan(inputs.pruefer_tree(12, 12))
    with pytest.raises(cc.CCError) as e:
        cc.count_budget_plan(P, G, 1 << 20)
    assert e.value.status == -4
