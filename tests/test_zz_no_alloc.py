"""cc_count_noalloc (the count with the library's fixed device workspace) against cc_count through
the C ABI: two calls in a row, the second on a smaller input, both bit-identical to cc_count with a
caller workspace (the same kernels in the same order), and a count too large for the fixed
workspace refused with CC_ENOSPC."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def _case(cc, torch, dev, rp, cl, T, k, seed, B):
    G = cc.Graph.from_numpy(rp, cl, device=dev)
    P = cc.Plan(T)
    C = cc.colour(G, k, seed=seed, first_iter=0, B=B)
    X_ref, V_ref = cc.count(P, G, C, per_vertex=True)
    X = torch.full((B,), -1.0, dtype=torch.float64, device=dev)
    V = torch.full((B, G.n), -1.0, dtype=torch.float64, device=dev)
    cc.count_noalloc(P, G, C, out=X, vertex_out=V)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(X.cpu().numpy(), X_ref.cpu().numpy())
    np.testing.assert_array_equal(V.cpu().numpy(), V_ref.cpu().numpy())
    # without per-vertex output: the root counts go to the fixed workspace
    X2 = torch.full((B,), -1.0, dtype=torch.float64, device=dev)
    cc.count_noalloc(P, G, C, out=X2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(X2.cpu().numpy(), X_ref.cpu().numpy())
    return G, P


def test_noalloc_equals_count_twice_then_smaller(dev):
    import torch
    import paper_1804_09764_amd as cc
    print("case: no-alloc count, R-MAT 14 / 10-vertex tree, B = 3", flush=True)
    rp, cl = inputs.rmat_graph(14, 8, 11)
    _case(cc, torch, dev, rp, cl, inputs.pruefer_tree(10, 4), 10, 5, 3)
    print("case: no-alloc count, ER 500 / 5-path, B = 2 (smaller, after the larger one)", flush=True)
    rp, cl = inputs.er_graph(500, 2000, 3)
    _case(cc, torch, dev, rp, cl, inputs.path_tree(5), 5, 9, 2)


def test_noalloc_refuses_a_count_beyond_its_workspace(dev):
    import torch
    import paper_1804_09764_amd as cc
    rp, cl = inputs.rmat_graph(16, 16, 2)
    G = cc.Graph.from_numpy(rp, cl, device=dev)
    P = cc.Plan(inputs.pruefer_tree(12, 12))
    assert cc.count_workspace_bytes(P, G) > cc.CC_NOALLOC_SCRATCH_BYTES
    C = cc.colour(G, 12, seed=1, first_iter=0, B=1)
    X = torch.zeros(1, dtype=torch.float64, device=dev)
    with pytest.raises(cc.CCError) as e:
        cc.count_noalloc(P, G, C, out=X)
    assert e.value.status == -4 and "workspace" in str(e.value)
