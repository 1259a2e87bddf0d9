"""Batched counting: every instance of a batch equals its plain count bit for bit, in the
persistent single launch and in the level-by-level mode, alone and mixed with other instances."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


def _cc():
    import paper_1804_09764_amd as cc
    return cc


def _plain(cc, P, G, C):
    import torch
    X, V = cc.count(P, G, C.view(1, -1), per_vertex=True)
    torch.cuda.synchronize()
    return X.cpu().numpy()[0], V.cpu().numpy()[0]


@pytest.mark.parametrize("levels", [False, True])
def test_batch_equals_plain_mixed_instances(dev, levels):
    import torch
    cc = _cc()
    graphs = [cc.Graph.from_numpy(*inputs.rmat_graph(11, 16, 5), hub_threshold=128, chunk=64),
              cc.Graph.from_numpy(*inputs.er_graph(500, 2500, 2)),
              cc.Graph.from_numpy(*inputs.rmat_graph(9, 8, 3))]
    templates = [inputs.path_tree(5), inputs.pruefer_tree(7, 1), inputs.star_tree(4), inputs.pruefer_tree(9, 2),
                 np.zeros((0, 2), np.int32), inputs.path_tree(2)]
    plans = [cc.Plan(T) for T in templates]
    rng = np.random.default_rng(0)
    inst, want = [], []
    for i in range(24):
        G = graphs[i % len(graphs)]
        P = plans[int(rng.integers(len(plans)))]
        C = cc.colour(G, P.k, seed=100 + i, first_iter=i, B=1)[0]
        X = torch.empty(1, dtype=torch.float64, device=dev)
        V = torch.empty(G.n, dtype=torch.float64, device=dev) if i % 2 else None
        inst.append((P, G, C, X, V))
        want.append(_plain(cc, P, G, C))
    print(f"case: batch of {len(inst)} mixed instances, levels={levels}", flush=True)
    batch = cc.Batch(inst, levels=levels)
    batch.run()
    batch.check()
    for (P, G, C, X, V), (xw, vw) in zip(inst, want):
        assert float(X.cpu()[0]) == float(xw)
        if V is not None:
            np.testing.assert_array_equal(V.cpu().numpy(), vw)


def test_batch_all_trees_of_size_7_against_oracle(dev):
    import torch
    cc = _cc()
    rp, cl = inputs.rmat_graph(10, 16, 2)
    G = cc.Graph.from_numpy(rp, cl, hub_threshold=128, chunk=64)
    trees = inputs.all_trees(7)
    plans = [cc.Plan(T) for T in trees]
    C = cc.colour(G, 7, seed=7, first_iter=0, B=8)
    X, batch = cc.count_batched(plans, G, C)
    batch.check()
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    for t, T in enumerate(trees):
        for b in range(8):
            want = oracle.count(rp, cl, C[b].cpu().numpy(), T)
            assert Xh[t, b] == want or abs(Xh[t, b] - want) <= 1e-12 * want


def test_batch_reuse_and_empty(dev):
    import torch
    cc = _cc()
    G = cc.Graph.from_numpy(*inputs.er_graph(300, 900, 4))
    E = cc.Graph.from_numpy(np.zeros(1, np.int64), np.zeros(0, np.int32))
    P = cc.Plan(inputs.pruefer_tree(6, 6))
    C = cc.colour(G, 6, seed=3, first_iter=0, B=3)
    X = torch.empty(4, dtype=torch.float64, device=dev)
    inst = [(P, G, C[b], X[b:b + 1], None) for b in range(3)]
    inst.append((P, E, torch.empty(0, dtype=torch.uint8, device=dev), X[3:4], None))
    batch = cc.Batch(inst)
    ws = cc.Workspace()
    for rep in range(3):
        X.fill_(-1.0)
        batch.run(ws)
        batch.check()
        got = X.cpu().numpy()
        for b in range(3):
            assert got[b] == _plain(cc, P, G, C[b])[0]
        assert got[3] == 0.0
