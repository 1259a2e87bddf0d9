"""GPU parity: the HIP path (through the C ABI) against the oracle, element by element.

Counts below 2^53 must be bit-identical; above, within 1e-12 relative (all terms are non-negative
integers, so every entry whose exact value is below 2^53 is exact in any summation order).
"""
import math

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TWO53 = float(2 ** 53)


def _cc():
    import paper_1804_09764_amd as cc
    return cc


def assert_parity(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape
    small = ref < TWO53
    np.testing.assert_array_equal(gpu[small], ref[small])
    if (~small).any():
        rel = np.abs(gpu[~small] - ref[~small]) / ref[~small]
        assert rel.max() <= 1e-12, rel.max()


def gpu_count(rp, cl, col, T, root=-1, hub_threshold=0, chunk=0, flags=0, cols_per_lane=0):
    import torch
    cc = _cc()
    G = cc.Graph.from_numpy(rp, cl, hub_threshold=hub_threshold, chunk=chunk, cols_per_lane=cols_per_lane)
    P = cc.Plan(T, root=root, flags=flags)
    colours = torch.from_numpy(np.ascontiguousarray(col, dtype=np.uint8)).cuda().view(1, -1)
    X, V = cc.count(P, G, colours, per_vertex=True)
    torch.cuda.synchronize()
    return float(X.cpu()[0]), V.cpu().numpy()[0], P, G


def check_case(rp, cl, col, T, root=-1, **kw):
    Xg, Vg, P, G = gpu_count(rp, cl, col, T, root=root, **kw)
    Xo, Vo = oracle.count(rp, cl, col, T, root=P.info.root, per_vertex=True)
    assert_parity(Vg, Vo)
    assert_parity([Xg], [Xo])
    return Xg, P, G


def test_c0_er1000_path5_bit_exact(dev):
    print("case: ER n=1000 m=5000 seed 1, P5, colours seed 7", flush=True)
    rp, cl = inputs.er_graph(1000, 5000, 1)
    col = inputs.colours(1000, 5, 7)
    T = inputs.path_tree(5)
    brute = oracle.brute_count(rp, cl, col, T, root=0)
    for root in (-1, 0, 2):
        Xg, _, _ = check_case(rp, cl, col, T, root=root)
        assert Xg == brute


@pytest.mark.parametrize("seed", [1, 2])
def test_tiny_all_trees_all_roots(dev, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(8, 14))
    rp, cl = inputs.er_graph(n, 2 * n, seed)
    for k in range(1, 8):
        for ti, T in enumerate(inputs.all_trees(k)):
            col = inputs.colours(n, k, seed * 1000 + k * 10 + ti)
            for root in range(k):
                print(f"case: tiny n={n} k={k} tree={ti} root={root}", flush=True)
                check_case(rp, cl, col, T, root=root)


def test_closed_forms(dev):
    # star K_{1,m}: (k-1)! * prod of leaf colour counts
    m = 40
    rp, cl = inputs.star_graph(m)
    for k in (3, 5, 7):
        col = inputs.colours(m + 1, k, k)
        c0 = int(col[0])
        nq = np.bincount(col[1:], minlength=k)
        want = math.factorial(k - 1) * math.prod(int(nq[q]) for q in range(k) if q != c0)
        Xg, _, _, _ = gpu_count(rp, cl, col, inputs.star_tree(k))
        assert Xg == want
    # cycle with col(i) = i mod k: the k-path has 2n maps
    for k in (3, 4, 6):
        n = 5 * k
        rp, cl = inputs.cycle_graph(n)
        col = (np.arange(n) % k).astype(np.uint8)
        assert gpu_count(rp, cl, col, inputs.path_tree(k))[0] == 2 * n
    # clique K_k, distinct colours: every tree has k! maps
    for k in (4, 7, 9):
        rp, cl = inputs.clique_graph(k)
        col = np.arange(k, dtype=np.uint8)
        for T in inputs.all_trees(k)[:6]:
            assert gpu_count(rp, cl, col, T)[0] == math.factorial(k)


@pytest.mark.parametrize("k", [3, 5, 8, 10])
def test_hub_chunks_match_oracle(dev, k):
    """Rows longer than the hub threshold are cut into chunks; results stay element-exact."""
    rp, cl = inputs.rmat_graph(11, 16, 5)
    col = inputs.colours(len(rp) - 1, k, 3)
    T = inputs.pruefer_tree(k, 40 + k)
    print(f"case: rmat11 hubs k={k}", flush=True)
    X1, P1, G1 = check_case(rp, cl, col, T, hub_threshold=64, chunk=64)
    assert G1.info["n_hubs"] > 0 and G1.info["n_chunks"] > G1.info["n_hubs"]
    X2, _, G2 = check_case(rp, cl, col, T, hub_threshold=100000, chunk=64)
    assert G2.info["n_hubs"] == 0
    assert X1 == X2 or abs(X1 - X2) <= 1e-12 * X2


@pytest.mark.parametrize("k", [11, 12, 13])
def test_wide_tables(dev, k):
    """k = 12..13: passive rows wider than 512 doubles take several column passes."""
    rp, cl = inputs.rmat_graph(8, 8, 2)
    col = inputs.colours(len(rp) - 1, k, 1)
    for seed in (12, 13):
        T = inputs.pruefer_tree(k, seed)
        for cols in (0, 1, 2, 8):
            print(f"case: rmat8 wide k={k} seed={seed} cols_per_lane={cols}", flush=True)
            check_case(rp, cl, col, T, hub_threshold=128, chunk=64, cols_per_lane=cols)
    check_case(rp, cl, col, inputs.path_tree(k))


@pytest.mark.parametrize("k", [14, 16])
def test_k_up_to_16(dev, k):
    rp, cl = inputs.er_graph(60, 240, k)
    col = inputs.colours(60, k, 2)
    print(f"case: er60 k={k}", flush=True)
    check_case(rp, cl, col, inputs.path_tree(k))
    check_case(rp, cl, col, inputs.pruefer_tree(k, 3))


def test_above_2_53(dev):
    """Dense graph with counts far above 2^53: relative 1e-12 there, exact below."""
    rp, cl = inputs.clique_graph(80)
    col = inputs.colours(80, 12, 5)
    Xg, _, _ = check_case(rp, cl, col, inputs.path_tree(12))
    assert Xg > TWO53
    rp, cl = inputs.rmat_graph(10, 32, 7)
    col = inputs.colours(len(rp) - 1, 9, 5)
    check_case(rp, cl, col, inputs.pruefer_tree(9, 1), hub_threshold=64, chunk=64)


def test_colour_kernel_matches_oracle_colouring(dev):
    import torch
    cc = _cc()
    rp, cl = inputs.er_graph(5000, 10000, 3)
    G = cc.Graph.from_numpy(rp, cl)
    for k in (1, 5, 12, 16):
        C = cc.colour(G, k, seed=1234, first_iter=7, B=3)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        for b in range(3):
            np.testing.assert_array_equal(got[b], oracle.colour(1234, 7 + b, 5000, k))


def test_batch_and_determinism(dev):
    import torch
    cc = _cc()
    rp, cl = inputs.rmat_graph(12, 16, 9)
    n = len(rp) - 1
    G = cc.Graph.from_numpy(rp, cl, hub_threshold=256, chunk=128)
    T = inputs.pruefer_tree(9, 9)
    P = cc.Plan(T)
    C = cc.colour(G, 9, seed=5, first_iter=0, B=4)
    X1, V1 = cc.count(P, G, C, per_vertex=True)
    X2 = cc.count(P, G, C)
    singles = [cc.count(P, G, C[b:b + 1].contiguous()) for b in range(4)]
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)
    for b in range(4):
        assert torch.equal(singles[b], X1[b:b + 1])
    Xo = [oracle.count(rp, cl, C[b].cpu().numpy(), T) for b in range(4)]
    assert_parity(X1.cpu().numpy(), Xo)


def test_graph_validation_rejects_bad_csr(dev):
    import torch
    cc = _cc()
    rp, cl = inputs.cycle_graph(10)
    bad = cl.copy()
    bad[0] = 0  # self-loop
    with pytest.raises(cc.CCError):
        cc.Graph.from_numpy(rp, bad)
    rp2, cl2 = inputs.csr_from_edges(5, [(0, 1), (1, 2), (3, 4)])
    c3 = cl2.copy()
    c3[-1] = 2  # asymmetric
    with pytest.raises(cc.CCError):
        cc.Graph.from_numpy(rp2, c3)
    rp4 = rp2.copy()
    rp4[2] = rp4[3] + 1  # decreasing offsets
    with pytest.raises(cc.CCError):
        cc.Graph.from_numpy(rp4, cl2)
    c5 = cl2.copy()
    c5[0] = 99  # out of range
    with pytest.raises(cc.CCError):
        cc.Graph.from_numpy(rp2, c5)
    cc.Graph.from_numpy(rp2, cl2)  # the good one passes
    torch.cuda.synchronize()


def test_empty_and_degenerate(dev):
    import torch
    cc = _cc()
    # isolated vertices only
    rp = np.zeros(11, dtype=np.int64)
    cl = np.zeros(0, dtype=np.int32)
    G = cc.Graph.from_numpy(rp, cl)
    for k in (1, 2, 5):
        T = inputs.path_tree(k)
        P = cc.Plan(T)
        C = cc.colour(G, k, 1, 0, 2)
        X = cc.count(P, G, C)
        torch.cuda.synchronize()
        assert X.cpu().tolist() == ([10.0, 10.0] if k == 1 else [0.0, 0.0])
    # k larger than any embedding can reach
    rp, cl = inputs.path_graph(5)
    col = np.arange(5, dtype=np.uint8) % 3
    assert gpu_count(rp, cl, col, inputs.path_tree(6))[0] == 0.0


def test_estimate_tracks_true_count(dev):
    import torch
    cc = _cc()
    rp, cl = inputs.er_graph(40, 110, 8)
    T = inputs.pruefer_tree(5, 4)
    copies = oracle.brute_count(rp, cl, None, T, root=0) / oracle.aut(T)
    G = cc.Graph.from_numpy(rp, cl)
    P = cc.Plan(T)
    C = cc.colour(G, 5, seed=11, first_iter=0, B=4000)
    X = cc.count(P, G, C)
    torch.cuda.synchronize()
    est, se = cc.estimate(P, X.cpu().numpy())
    assert abs(est - copies) < 5 * se


@pytest.mark.parametrize("offset", [0, 1, 3])
def test_column_alignment_and_ragged_tail(dev, offset):
    """The plain count gathers each CSR entry's neighbour colour once per colouring, four entries
    per thread when the column array is 16-byte aligned and one per thread otherwise; nnz here is
    2 mod 4, so the aligned path also runs its tail. Column views 0, 4 and 12 bytes past a 16-byte
    boundary all equal the oracle."""
    import torch
    cc = _cc()
    rp, cl = inputs.rmat_graph(10, 16, 9)
    nnz = len(cl)
    assert nnz % 4 == 2
    big = torch.zeros(nnz + 8, dtype=torch.int32, device="cuda")
    big[offset:offset + nnz] = torch.from_numpy(cl).cuda()
    col_view = big[offset:offset + nnz]
    assert col_view.data_ptr() % 16 == 4 * offset
    G = cc.Graph(torch.from_numpy(rp).cuda(), col_view, hub_threshold=64, chunk=64)
    k = 7
    T = inputs.pruefer_tree(k, 4)
    P = cc.Plan(T)
    cols = np.stack([inputs.colours(len(rp) - 1, k, s) for s in (21, 22)])
    X, V = cc.count(P, G, torch.from_numpy(cols).cuda(), per_vertex=True)
    torch.cuda.synchronize()
    for b in range(2):
        print(f"case: column offset {offset} colouring {b}", flush=True)
        Xo, Vo = oracle.count(rp, cl, cols[b], T, root=P.info.root, per_vertex=True)
        assert_parity(V.cpu().numpy()[b], Vo)
        assert_parity([float(X[b])], [Xo])


def test_shared_and_unshared_plans_agree(dev):
    """A template with equal branches: the plan that runs each equal branch once and the plan that
    runs every split both match the oracle."""
    cc = _cc()
    legs = np.array([(0, 1), (1, 2), (0, 3), (3, 4), (0, 5), (5, 6), (6, 7)], dtype=np.int32)
    rp, cl = inputs.rmat_graph(11, 16, 8)
    col = inputs.colours(len(rp) - 1, 8, 9)
    shared = cc.Plan(legs, root=0)
    assert shared.info.n_splits < 7
    print("case: spider k=8, shared and unshared plans", flush=True)
    Xs, _, _ = check_case(rp, cl, col, legs, root=0, hub_threshold=64, chunk=64)
    Xf, _, _ = check_case(rp, cl, col, legs, root=0, hub_threshold=64, chunk=64, flags=cc.CC_PLAN_NO_SHARING)
    assert Xs == Xf or abs(Xs - Xf) <= 1e-12 * Xf
