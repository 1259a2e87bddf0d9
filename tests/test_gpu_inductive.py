"""Inductive single-step parity: every split of the plan, checked one step at a time.

A split of the dynamic program (Section 2.1, Eq. 1) computes the table of T_i from the tables of
T_i' and T_i'' alone. For each split the GPU runs the count up to that split and stops
(cc_count_inspect); its input tables are read back for sampled centre vertices and all of their
neighbours, expanded from the colour-anchored storage (cc_plan_table_get, cc_entry_order) to full
colex rows over the k colours, and the oracle applies Eq. 1 once (oracle.step) to the GPU's own
inputs. Its result must equal the GPU's output table entry by entry (every C(k, s) entry per
sampled vertex, the zeros of the sets without col(v) included): bit for bit below 2^53, within
1e-12 relative above. With the leaves fixed by the colouring, the splits checked this way cover the
whole computation by induction, at sizes where the whole count cannot be recomputed on the host.

Workloads: ER n=1000 / 5-path (every vertex, every split: the helper itself against a case the
full count pins), R-MAT scale 23, edge factor 256 / 12-vertex tree (seed 12) and R-MAT scale 20,
edge factor 16 / 15-vertex tree (seed 15), in bench.py's launch configuration (default tuning).
Sampled centres per split: the highest-degree vertex, cut rows (more neighbours than the hub
threshold) at log-spaced degrees, and uniform vertices, about 1000 in all.
"""
import math

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TWO53 = float(2 ** 53)


def _colex_masks(K, m):
    """Masks of m colours out of K in colex order (= increasing numeric order)."""
    return [x for x in range(1 << K) if bin(x).count("1") == m]


def dest_map(k, t):
    """dest[c][j] = colex rank over all k colours (the oracle's set index) of the set stored at
    position j of a row anchored at colour c, for sets of t colours."""
    import paper_1804_09764_amd as cc
    K = k - 1
    masks = _colex_masks(K, t - 1)
    order = cc.entry_order(k, t - 1)
    full_rank = {m: r for r, m in enumerate(_colex_masks(k, t))}
    out = np.zeros((k, len(order)), dtype=np.int64)
    for c in range(k):
        for j, r in enumerate(order):
            R = masks[r]
            lo = R & ((1 << c) - 1)
            S = lo | ((R >> c) << (c + 1)) | (1 << c)
            out[c, j] = full_rank[S]
    return out


def full_rows(plan, graph, ws, table, vertices, colours_dev, k):
    """Full colex rows (len(vertices) x C(k, t)) of table `table` for `vertices`, as float64 on the
    host; table -1 is a single vertex (one-hot at its colour)."""
    import torch
    import paper_1804_09764_amd as cc
    idx = torch.as_tensor(vertices, dtype=torch.int64, device=colours_dev.device)
    cols = colours_dev.reshape(-1).index_select(0, idx).to(torch.int64)
    if table < 0:
        out = torch.zeros((len(vertices), k), dtype=torch.float64, device=idx.device)
        out.scatter_(1, cols.unsqueeze(1), 1.0)
        return out.cpu().numpy()
    d = cc.table_desc(plan, graph, table)
    t = d["size"]
    region = ws[d["offset"]:d["offset"] + graph.n * d["stride"] * 8].view(torch.float64).view(graph.n, d["stride"])
    rows = region.index_select(0, idx)[:, :d["width"]]
    dest = torch.as_tensor(dest_map(k, t), device=idx.device)
    out = torch.zeros((len(vertices), math.comb(k, t)), dtype=torch.float64, device=idx.device)
    out.scatter_(1, dest.index_select(0, cols), rows)
    return out.cpu().numpy()


def sample_centres(rp, hub_threshold, n_uniform, n_cut, seed):
    deg = np.diff(rp)
    n = len(deg)
    rng = np.random.default_rng(seed)
    picks = [int(np.argmax(deg))]
    cut = np.flatnonzero(deg > hub_threshold)
    if len(cut):
        order = cut[np.argsort(deg[cut], kind="stable")]
        for q in np.unique(np.geomspace(1, len(order), n_cut).astype(np.int64) - 1):
            picks.append(int(order[q]))
    picks += [int(v) for v in rng.choice(n, min(n, n_uniform), replace=False)]
    return np.unique(np.asarray(picks, dtype=np.int64))


def assert_step(gpu, ref, what):
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    small = ref < TWO53
    bad = np.flatnonzero(gpu[small] != ref[small])
    assert len(bad) == 0, (what, "entries below 2^53 differ", len(bad), gpu[small][bad[:5]], ref[small][bad[:5]])
    if (~small).any():
        rel = np.abs(gpu[~small] - ref[~small]) / ref[~small]
        assert rel.max() <= 1e-12, (what, "relative error", rel.max())


def check_split(plan, graph, rp, col, colours_dev, split, centres, ws_holder):
    """Run to `split`, expand the GPU's inputs for the centres and their neighbours, apply Eq. 1
    once on the host, compare with the GPU's output rows."""
    import torch
    import paper_1804_09764_amd as cc
    k = plan.k
    s, a, p = plan.splits[split]
    m = plan.split_maps(split)
    ws, V = cc.count_inspect(plan, graph, colours_dev, split, workspace=ws_holder)
    torch.cuda.synchronize()
    lens = (rp[centres + 1] - rp[centres]).astype(np.int64)
    nbrs = np.concatenate([col[rp[v]:rp[v + 1]] for v in centres]) if len(centres) else np.zeros(0, np.int32)
    uniq, inv = np.unique(nbrs, return_inverse=True)
    nbr_ptr = np.zeros(len(centres) + 1, dtype=np.int64)
    nbr_ptr[1:] = np.cumsum(lens)
    A = full_rows(plan, graph, ws, m["act"], centres, colours_dev, k)
    P = full_rows(plan, graph, ws, m["pas"], uniq, colours_dev, k)
    ref = oracle.step(k, s, a, nbr_ptr, inv.astype(np.int32), A, P)
    del P
    if m["out"] == -2:
        gpu = V.index_select(0, torch.as_tensor(centres, device=V.device)).cpu().numpy().reshape(-1, 1)
    else:
        gpu = full_rows(plan, graph, ws, m["out"], centres, colours_dev, k)
    assert_step(gpu, ref, f"split {split} (s={s}, a={a}, p={p})")
    return len(centres), int(lens.sum()), len(uniq)


def test_c0_every_split_every_vertex(dev):
    """ER n=1000 / 5-path: every split, every vertex (the expansion helper on a case that the full
    count already pins against brute force)."""
    import torch
    import paper_1804_09764_amd as cc
    rp, col = inputs.er_graph(1000, 5000, 1)
    G = cc.Graph.from_numpy(rp, col, device=dev)
    C = torch.from_numpy(inputs.colours(1000, 5, 7)).to(dev)
    ws = cc.Workspace()
    for root in (-1, 0, 2):
        P = cc.Plan(inputs.path_tree(5), root=root)
        for i in range(P.info.n_splits):
            print(f"case: C0 root {root} split {i} {P.splits[i]}", flush=True)
            check_split(P, G, rp, col, C, i, np.arange(1000), ws)
    # a template with a combine over several pairs and a passive part of three vertices
    P = cc.Plan(np.array([[0, 1], [1, 2], [2, 3], [1, 4], [4, 5], [0, 6]], dtype=np.int32))
    C7 = torch.from_numpy(inputs.colours(1000, 7, 8)).to(dev)
    for i in range(P.info.n_splits):
        print(f"case: C0 7-tree split {i} {P.splits[i]}", flush=True)
        check_split(P, G, rp, col, C7, i, np.arange(1000), ws)


@pytest.fixture(scope="module")
def c3a(dev):
    import paper_1804_09764_amd as cc
    print("case: building R-MAT 23 ef 256", flush=True)
    rp_d, col_d = inputs.rmat_graph_gpu(23, 256, 3, device=dev)
    G = cc.Graph(rp_d, col_d, trust=True)
    P = cc.Plan(inputs.pruefer_tree(12, 12))
    C = cc.colour(G, 12, seed=777, first_iter=0, B=1)[0]
    rp, col = rp_d.cpu().numpy(), col_d.cpu().numpy()
    centres = sample_centres(rp, G.info["hub_threshold"], n_uniform=990, n_cut=9, seed=23)
    yield dict(G=G, P=P, C=C, rp=rp, col=col, centres=centres, ws=cc.Workspace())


@pytest.mark.parametrize("split", range(8))
def test_c3a_rmat23_ef256_u12_single_step(c3a, split):
    P = c3a["P"]
    if split >= P.info.n_splits:
        pytest.skip("the plan runs fewer splits")
    print(f"case: R-MAT 23 ef256 12-tree split {split} {P.splits[split]}", flush=True)
    nv, ne, nu = check_split(P, c3a["G"], c3a["rp"], c3a["col"], c3a["C"], split, c3a["centres"], c3a["ws"])
    print(f"checked {nv} centres, {ne} neighbour entries, {nu} distinct neighbours", flush=True)


@pytest.fixture(scope="module")
def c3b(dev):
    import paper_1804_09764_amd as cc
    rp_d, col_d = inputs.rmat_graph_gpu(20, 16, 1, device=dev)
    G = cc.Graph(rp_d, col_d)
    P = cc.Plan(inputs.pruefer_tree(15, 15))
    C = cc.colour(G, 15, seed=777, first_iter=0, B=1)[0]
    rp, col = rp_d.cpu().numpy(), col_d.cpu().numpy()
    centres = sample_centres(rp, G.info["hub_threshold"], n_uniform=990, n_cut=9, seed=20)
    yield dict(G=G, P=P, C=C, rp=rp, col=col, centres=centres, ws=cc.Workspace())


@pytest.mark.parametrize("split", range(11))
def test_c3b_rmat20_u15_single_step(c3b, split):
    P = c3b["P"]
    if split >= P.info.n_splits:
        pytest.skip("the plan runs fewer splits")
    print(f"case: R-MAT 20 15-tree split {split} {P.splits[split]}", flush=True)
    nv, ne, nu = check_split(P, c3b["G"], c3b["rp"], c3b["col"], c3b["C"], split, c3b["centres"], c3b["ws"])
    print(f"checked {nv} centres, {ne} neighbour entries, {nu} distinct neighbours", flush=True)


def test_c3a_colouring_matches_oracle(c3a):
    """The leaves of the induction: the colouring on the device is the oracle's."""
    n = len(c3a["rp"]) - 1
    assert np.array_equal(c3a["C"].cpu().numpy(), oracle.colour(777, 0, n, 12))
