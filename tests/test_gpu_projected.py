"""Projected passive rows (cc_tuning.proj_classes) against the oracle and the unprojected count.

A centre of colour c adds up only the entries of a neighbour's row whose colour set avoids c
(Section 2.1, Eq. 1: the active and passive sets of a split are disjoint). With projection on, a
wide split copies those entries of every row into one contiguous row per colour and runs its
centres colour class by colour class. The same terms reach each neighbour sum in the same order
when a passive row fits one pass of the gather, so counts must be bit-identical to the
unprojected path there, and exact below 2^53 (1e-12 relative above) against the oracle always.
"""
import json
import os

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TWO53 = float(2 ** 53)


def assert_parity(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape
    small = ref < TWO53
    np.testing.assert_array_equal(gpu[small], ref[small])
    if (~small).any():
        rel = np.abs(gpu[~small] - ref[~small]) / ref[~small]
        assert rel.max() <= 1e-12, rel.max()


def count(rp, cl, col, T, **tuning):
    import torch
    import paper_1804_09764_amd as cc
    G = cc.Graph.from_numpy(rp, cl, **tuning)
    P = cc.Plan(T)
    colours = torch.from_numpy(np.ascontiguousarray(col, dtype=np.uint8)).cuda().view(1, -1)
    X, V = cc.count(P, G, colours, per_vertex=True)
    torch.cuda.synchronize()
    return float(X.cpu()[0]), V.cpu().numpy()[0], P


def wide_splits(P):
    return [i for i in range(P.info.n_splits) if P.split_maps(i)["Wn"] > 0]


@pytest.mark.parametrize("k", [10, 11, 12])
def test_projected_equals_oracle_and_unprojected(dev, k):
    """R-MAT scale 11 (edge factor 16), cut rows of 64 entries: every class count per pass, one
    colour per pass up to all k colours in one pass."""
    rp, cl = inputs.rmat_graph(11, 16, 5)
    n = len(rp) - 1
    col = inputs.colours(n, k, 3)
    T = inputs.pruefer_tree(k, 40 + k)
    X0, V0, P = count(rp, cl, col, T, hub_threshold=64, chunk=64, proj_classes=-1)
    assert wide_splits(P), "the template has no wide passive rows"
    Xo, Vo = oracle.count(rp, cl, col, T, root=P.info.root, per_vertex=True)
    assert_parity(V0, Vo)
    for cls in (1, 3, 5, k):
        print(f"case: rmat11 k={k} proj_classes={cls}", flush=True)
        X, V, _ = count(rp, cl, col, T, hub_threshold=64, chunk=64, proj_classes=cls)
        np.testing.assert_array_equal(V, V0)
        assert X == X0
        assert_parity(V, Vo)
        assert_parity([X], [Xo])


def test_projected_light_rows_only(dev):
    """No cut rows (every row one task), four classes per pass."""
    rp, cl = inputs.rmat_graph(10, 32, 7)
    n = len(rp) - 1
    col = inputs.colours(n, 11, 9)
    T = inputs.pruefer_tree(11, 5)
    X0, V0, P = count(rp, cl, col, T, hub_threshold=100000, chunk=64, proj_classes=-1)
    X, V, _ = count(rp, cl, col, T, hub_threshold=100000, chunk=64, proj_classes=4)
    np.testing.assert_array_equal(V, V0)
    Xo, Vo = oracle.count(rp, cl, col, T, root=P.info.root, per_vertex=True)
    assert_parity(V, Vo)


def test_projected_invalid_colours(dev):
    """Vertices whose colour is not below k take part in no map and their rows are zero; the
    first pass writes them. Projected and unprojected counts agree bit for bit."""
    rp, cl = inputs.rmat_graph(10, 16, 3)
    n = len(rp) - 1
    k = 12
    col = inputs.colours(n, k, 4).copy()
    rng = np.random.default_rng(1)
    col[rng.choice(n, n // 10, replace=False)] = 200
    T = inputs.pruefer_tree(k, 12)
    X0, V0, _ = count(rp, cl, col, T, hub_threshold=64, chunk=64, proj_classes=-1)
    X, V, _ = count(rp, cl, col, T, hub_threshold=64, chunk=64, proj_classes=5)
    np.testing.assert_array_equal(V, V0)
    assert np.all(V[col >= k] == 0)


@pytest.mark.parametrize("k", [15, 16])
def test_projected_rows_over_several_gather_passes(dev, k):
    """k = 15, 16: passive rows of 2002..6435 entries, projected rows of 1287..3432, read in
    several column passes: exact against the oracle (the order of terms may differ from the
    unprojected count, which matters only above 2^53)."""
    rp, cl = inputs.er_graph(300, 3000, 4)
    col = inputs.colours(300, k, 3)
    T = inputs.pruefer_tree(k, 7)
    X, V, P = count(rp, cl, col, T, hub_threshold=64, chunk=64, proj_classes=3)
    assert wide_splits(P)
    Xo, Vo = oracle.count(rp, cl, col, T, root=P.info.root, per_vertex=True)
    assert Xo < TWO53
    assert_parity(V, Vo)
    assert X == Xo


def test_projected_rmat20_u12_against_golden(dev):
    """R-MAT scale 20 / 12-vertex tree with projection forced (three classes per pass, the
    default degree split): X and the 2000 stored oracle per-vertex counts."""
    import torch
    import paper_1804_09764_amd as cc
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rmat20_u12.json")))
    G0, T0 = g["graph"], g["template"]
    rp, col = inputs.rmat_graph_gpu(G0["scale"], G0["edge_factor"], G0["seed"], device=dev)
    G = cc.Graph(rp, col, proj_classes=3)
    T = inputs.pruefer_tree(T0["k"], T0["seed"])
    colours = torch.from_numpy(inputs.colours(rp.numel() - 1, T0["k"], g["colouring"]["seed"])).to(dev).view(1, -1)
    P = cc.Plan(T, root=T0["root"])
    assert wide_splits(P)
    X, V = cc.count(P, G, colours, per_vertex=True)
    torch.cuda.synchronize()
    assert_parity([float(X.cpu()[0])], [float(g["X"])])
    Vh = V.cpu().numpy()[0]
    assert_parity(Vh[np.asarray(g["vertices"])], np.asarray(g["vertex_counts"], dtype=np.float64))


def test_auto_projection_skips_low_degree_graphs(dev):
    """On R-MAT scale 20, edge factor 16 (30 entries per row on average) copying rows costs more
    than it saves: the byte model projects nothing."""
    import paper_1804_09764_amd as cc
    rp, col = inputs.rmat_graph_gpu(20, 16, 1, device=dev)
    G = cc.Graph(rp, col)
    for k, seed in ((12, 12), (15, 15)):
        P = cc.Plan(inputs.pruefer_tree(k, seed))
        assert wide_splits(P)
        assert cc.count_projection(P, G) == [0] * P.info.n_splits
