"""Parity at the benchmark sizes, in the launch configuration bench.py times (default tuning).

* R-MAT scale 20 / 12-vertex tree: X and 2000 sampled per-vertex counts against the oracle's values
  stored in tests/golden/rmat20_u12.json (written by tests/golden/make_golden.py, oracle only).
* R-MAT scale 23, edge factor 256: per-vertex closed forms on sampled vertices (the oracle's
  per-vertex definitions evaluated one by one on the host: the edge, the 3-path and the 4-star
  rooted at their centres), the exact total for the edge, and, for the 12-vertex tree, invariance
  of X under the choice of root (a property that holds at any size).
"""
import json
import math
import os

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat20_u12.json")
TWO53 = float(2 ** 53)


def _close(gpu, ref):
    gpu, ref = float(gpu), float(ref)
    if ref < TWO53:
        assert gpu == ref, (gpu, ref)
    else:
        assert abs(gpu - ref) <= 1e-12 * ref, (gpu, ref, abs(gpu - ref) / ref)


def test_rmat20_u12_against_golden(dev):
    import torch
    import paper_1804_09764_amd as cc
    g = json.load(open(GOLDEN))
    G0, T0 = g["graph"], g["template"]
    rp, col = inputs.rmat_graph_gpu(G0["scale"], G0["edge_factor"], G0["seed"], device=dev)
    assert col.numel() == G0["nnz"]
    G = cc.Graph(rp, col)
    T = inputs.pruefer_tree(T0["k"], T0["seed"])
    colours = torch.from_numpy(inputs.colours(rp.numel() - 1, T0["k"], g["colouring"]["seed"])).to(dev).view(1, -1)
    P = cc.Plan(T, root=T0["root"])
    print("case: R-MAT 20 / 12-tree against the stored oracle values", flush=True)
    X, V = cc.count(P, G, colours, per_vertex=True)
    torch.cuda.synchronize()
    _close(X.cpu()[0], float(g["X"]))
    Vh = V.cpu().numpy()[0]
    for v, want in zip(g["vertices"], g["vertex_counts"]):
        _close(Vh[v], float(want))
    # the planner's own root gives the same total
    X2 = cc.count(cc.Plan(T), G, colours)
    torch.cuda.synchronize()
    _close(X2.cpu()[0], float(g["X"]))


def _neighbour_colour_counts(rp, col, colours, v, k):
    return np.bincount(colours[col[rp[v]:rp[v + 1]]], minlength=k).astype(np.int64)


def test_rmat23_ef256_closed_forms_and_invariance(dev):
    import torch
    import paper_1804_09764_amd as cc
    rp_d, col_d = inputs.rmat_graph_gpu(23, 256, 3, device=dev)
    n = rp_d.numel() - 1
    G = cc.Graph(rp_d, col_d, trust=True)
    rp = rp_d.cpu().numpy()
    col = col_d.cpu().numpy()
    deg = np.diff(rp)
    rng = np.random.default_rng(11)
    sample = np.unique(np.concatenate([np.argsort(-deg, kind="stable")[:20], rng.choice(n, 500, replace=False)]))

    # edge (k = 2), rooted at either end: per-vertex count of neighbours with the other colour
    c2 = cc.colour(G, 2, seed=5, first_iter=0, B=1)
    X, V = cc.count(cc.Plan(inputs.path_tree(2), root=0), G, c2, per_vertex=True)
    torch.cuda.synchronize()
    ch = c2.cpu().numpy()[0]
    Vh = V.cpu().numpy()[0]
    for v in sample:
        assert Vh[v] == float(np.sum(ch[col[rp[v]:rp[v + 1]]] != ch[v]))
    src_col = np.repeat(ch, deg)
    assert float(X.cpu()[0]) == float(np.sum(src_col != ch[col]))
    del src_col

    # 3-path rooted at its middle: ordered pairs of neighbours with two different colours, both
    # different from the centre's
    c3 = cc.colour(G, 3, seed=6, first_iter=0, B=1)
    _, V = cc.count(cc.Plan(inputs.path_tree(3), root=1), G, c3, per_vertex=True)
    torch.cuda.synchronize()
    ch = c3.cpu().numpy()[0]
    Vh = V.cpu().numpy()[0]
    for v in sample:
        nc = _neighbour_colour_counts(rp, col, ch, v, 3)
        others = [int(nc[c]) for c in range(3) if c != ch[v]]
        _close(Vh[v], 2 * others[0] * others[1])

    # 4-star rooted at its centre: 3! * product of the neighbour counts of the three other colours
    c4 = cc.colour(G, 4, seed=7, first_iter=0, B=1)
    _, V = cc.count(cc.Plan(inputs.star_tree(4), root=0), G, c4, per_vertex=True)
    torch.cuda.synchronize()
    ch = c4.cpu().numpy()[0]
    Vh = V.cpu().numpy()[0]
    for v in sample:
        nc = _neighbour_colour_counts(rp, col, ch, v, 4)
        _close(Vh[v], 6 * math.prod(int(nc[c]) for c in range(4) if c != ch[v]))

    # the 12-vertex benchmark tree: the total does not depend on the root or the partition
    T = inputs.pruefer_tree(12, 12)
    c12 = cc.colour(G, 12, seed=777, first_iter=0, B=1)
    print("case: R-MAT 23 ef256, 12-tree, two roots", flush=True)
    Pa = cc.Plan(T)
    # the byte model projects the 462- and 330-entry passive rows (the p = 6 and p = 5 splits)
    proj = cc.count_projection(Pa, G)
    assert [i for i, c in enumerate(proj) if c > 0] == [i for i, sp in enumerate(Pa.splits) if sp[2] >= 5]
    Xa = cc.count(Pa, G, c12)
    Xb = cc.count(cc.Plan(T, root=0), G, c12)
    # projected and unprojected counts agree bit for bit (each row fits one pass of the gather)
    Xc = cc.count(Pa, cc.Graph(rp_d, col_d, trust=True, proj_classes=-1), c12)
    torch.cuda.synchronize()
    a, b = float(Xa.cpu()[0]), float(Xb.cpu()[0])
    assert a > TWO53 and abs(a - b) <= 1e-12 * a
    assert float(Xc.cpu()[0]) == a


def test_c2_batched_against_oracle(dev):
    """R-MAT scale 18 (edge factor 16, seed 2), all 11 trees with 7 vertices x 64 colourings, counted
    as bench.py's batched leg does (one multi-template packed count, default tuning) and as one
    packed count per tree: sampled colourings against the oracle."""
    import torch
    import paper_1804_09764_amd as cc
    import oracle
    rp_d, col_d = inputs.rmat_graph_gpu(18, 16, 2, device=dev)
    G = cc.Graph(rp_d, col_d)
    rp, col = rp_d.cpu().numpy(), col_d.cpu().numpy()
    C = cc.colour(G, 7, seed=777, first_iter=0, B=64)
    Ch = C.cpu().numpy()
    trees = inputs.all_trees(7)
    plans = [cc.Plan(T) for T in trees]
    Xm = cc.Multi(plans).count(G, C)
    torch.cuda.synchronize()
    Xm = Xm.cpu().numpy()
    for t, (T, P) in enumerate(zip(trees, plans)):
        X = cc.count_packed(P, G, C)
        torch.cuda.synchronize()
        Xh = X.cpu().numpy()
        for b in ((0, 63) if t < 3 else (t,)):
            print(f"case: R-MAT 18 tree {t} colouring {b} against the oracle", flush=True)
            want = oracle.count(rp, col, Ch[b], T)
            _close(Xm[t, b], want)
            _close(Xh[b], want)


def test_c3b_rmat20_u15_root_invariance(dev):
    """R-MAT scale 20 / 15-vertex tree (seed 15): the total does not depend on the root."""
    import torch
    import paper_1804_09764_amd as cc
    rp_d, col_d = inputs.rmat_graph_gpu(20, 16, 1, device=dev)
    G = cc.Graph(rp_d, col_d)
    T = inputs.pruefer_tree(15, 15)
    c = cc.colour(G, 15, seed=777, first_iter=0, B=1)
    print("case: R-MAT 20, 15-tree, planner root and root 0", flush=True)
    Xa = cc.count(cc.Plan(T), G, c)
    Xb = cc.count(cc.Plan(T, root=0), G, c)
    torch.cuda.synchronize()
    a, b = float(Xa.cpu()[0]), float(Xb.cpu()[0])
    assert a > TWO53 and abs(a - b) <= 1e-12 * a
