"""Host-side checks of libcc.so without a GPU: exported symbols, planner logic, error paths.

Nothing here launches a kernel; cc_plan_create / cc_plan_info_get / cc_estimate are host-only.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import inputs
import oracle
import paper_1804_09764_amd as cc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "cc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = cc.lib()
    names = _declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert sorted(cc.EXPORTS) == names


def test_plan_rejects_bad_templates():
    """k = 1 is accepted; non-trees, k > 16, duplicate edges and bad roots are rejected."""
    p = cc.Plan(np.zeros((0, 2)), bind=False)
    assert p.info.k == 1 and p.info.n_splits == 0
    with pytest.raises(cc.CCError) as e:
        cc.Plan([[0, 1], [1, 2], [2, 0]], bind=False)  # k=4: a triangle plus an isolated vertex
    assert e.value.status == -1
    with pytest.raises(cc.CCError) as e:
        cc.Plan(inputs.path_tree(17), bind=False)
    assert e.value.status == -2
    with pytest.raises(cc.CCError):
        cc.Plan([[0, 1], [0, 1]], bind=False)
    with pytest.raises(cc.CCError):
        cc.Plan(inputs.path_tree(4), root=4, bind=False)


@pytest.mark.parametrize("k", range(1, 11))
def test_aut_matches_oracle(k):
    for T in inputs.all_trees(k):
        assert cc.Plan(T, bind=False).info.aut == oracle.aut(T)


@pytest.mark.parametrize("k", [12, 13, 14, 15, 16])
def test_aut_large_random_trees(k):
    for seed in range(3):
        T = inputs.pruefer_tree(k, seed)
        assert cc.Plan(T, bind=False).info.aut == oracle.aut(T)
    assert cc.Plan(inputs.star_tree(k), bind=False).info.aut == math.factorial(k - 1)


@pytest.mark.parametrize("k", range(2, 17))
def test_partition_invariants(k):
    for seed in range(5):
        T = inputs.pruefer_tree(k, seed)
        for root in (-1, 0, k - 1):
            p = cc.Plan(T, root=root, bind=False, flags=cc.CC_PLAN_NO_SHARING)
            assert p.info.n_splits == k - 1
            assert p.splits[-1][0] == k
            for s, a, pp in p.splits:
                assert s == a + pp and a >= 1 and pp >= 1
            # the passive sizes are the subtree sizes of the non-root vertices
            assert sorted(pp for _, _, pp in p.splits) == sorted(_subtree_sizes(T, p.info.root))


@pytest.mark.parametrize("k", range(2, 17))
def test_shared_splits_are_a_subset(k):
    """With sharing (the default), the splits that run are a sub-multiset of the partition's, the
    root split is last, and the table arena is no larger; the reference partition never shares."""
    from collections import Counter
    for seed in range(5):
        T = inputs.pruefer_tree(k, seed)
        for root in (0, k - 1):
            full = cc.Plan(T, root=root, bind=False, flags=cc.CC_PLAN_NO_SHARING)
            p = cc.Plan(T, root=root, bind=False)
            assert p.splits[-1] == full.splits[-1]
            assert not (Counter(p.splits) - Counter(full.splits))
            assert p.info.table3_memory == full.info.table3_memory
        ref = cc.Plan(T, bind=False, flags=cc.CC_PLAN_CENTRE_SMALLEST)
        assert ref.info.n_splits == k - 1
    # two equal branches below the root: the branch's splits run once
    legs = [(0, 1), (1, 2), (0, 3), (3, 4), (0, 5), (5, 6)]
    p = cc.Plan(np.array(legs, dtype=np.int32), root=0, bind=False)
    assert p.info.n_splits < 6


def _subtree_sizes(T, root):
    k = len(T) + 1
    adj = [[] for _ in range(k)]
    for u, v in T:
        adj[u].append(v)
        adj[v].append(u)
    sizes = []

    def dfs(x, par):
        s = 1
        for y in adj[x]:
            if y != par:
                s += dfs(y, x)
        if par >= 0:
            sizes.append(s)
        return s

    dfs(root, -1)
    return sizes


def test_table3_bookkeeping():
    """The paper's Table 3: u3-1 = (3, 6), u5-2 = (25, 70), u12-1 = (4082, 24552) are reproduced by
    end-rooted paths, counting every split sub-template except T itself."""
    for k, want in [(3, (3, 6)), (5, (25, 70)), (12, (4082, 24552))]:
        p = cc.Plan(inputs.path_tree(k), root=0, bind=False)
        assert (p.info.table3_memory, p.info.table3_compute) == want


def test_units_reference_partition():
    # the 5-path rooted at its centre: passive subtrees 2, 1, 2, 1 -> C(5,2)+1+C(5,2)+1 = 22
    assert cc.Plan(inputs.path_tree(5), bind=False).info.units_per_edge == 22
    # a star with k-1 leaves: k-1 passive single vertices
    assert cc.Plan(inputs.star_tree(9), bind=False).info.units_per_edge == 8
    # the 12-path end-rooted plan still reports units of the centre-rooted reference partition
    a = cc.Plan(inputs.path_tree(12), root=0, bind=False).info.units_per_edge
    b = cc.Plan(inputs.path_tree(12), bind=False).info.units_per_edge
    assert a == b


def test_estimate_host():
    T = inputs.pruefer_tree(6, 3)
    p = cc.Plan(T, bind=False)
    X = [10.0, 20.0, 30.0, 40.0]
    est, se = cc.estimate(p, X)
    f = 6 ** 6 / math.factorial(6) / p.info.aut
    assert math.isclose(est, 25.0 * f, rel_tol=1e-15)
    assert math.isclose(se, np.std(X, ddof=1) / 2 * f, rel_tol=1e-12)
    assert math.isclose(est, oracle.estimate(6, int(p.info.aut), X), rel_tol=1e-15)
    mom = cc.estimate_median_of_means(p, [1.0, 3.0, 10.0, 10.0, 100.0, 200.0], 3)
    assert math.isclose(mom, 10.0 * f, rel_tol=1e-15)
    with pytest.raises(cc.CCError):
        cc.estimate_median_of_means(p, [1.0, 2.0, 3.0], 2)


def test_iterations_driver():
    """Sample sizes of the (epsilon, delta) driver and their argument checks."""
    for k, eps, delta in ((1, 0.5, 0.5), (3, 0.5, 0.1), (7, 0.2, 0.05), (12, 0.1, 0.01), (16, 0.9, 0.9)):
        s, t = cc.iterations(k, eps, delta)
        assert s == math.ceil(4 * math.exp(k) / eps ** 2)
        assert t == max(1, math.ceil(8 * math.log(1 / delta)))
    # monotone: tighter epsilon or delta, larger k -> more samples
    assert cc.iterations(5, 0.1, 0.1)[0] > cc.iterations(5, 0.2, 0.1)[0]
    assert cc.iterations(5, 0.1, 0.01)[1] > cc.iterations(5, 0.1, 0.1)[1]
    assert cc.iterations(6, 0.1, 0.1)[0] > cc.iterations(5, 0.1, 0.1)[0]
    for bad in ((0, 0.1, 0.1), (17, 0.1, 0.1), (5, 0.0, 0.1), (5, 1.0, 0.1), (5, 0.1, 0.0), (5, 0.1, 1.0)):
        with pytest.raises(cc.CCError):
            cc.iterations(*bad)


def _line_skips(sets, K):
    """Lines of 16 entries that a reader anchored on colour x may skip (all sets hold x), summed
    over the K colours x."""
    return sum(all(sets[j] >> x & 1 for j in range(l, min(l + 16, len(sets))))
               for x in range(K) for l in range(0, len(sets), 16))


@pytest.mark.parametrize("k", [5, 8, 12, 16])
def test_entry_order(k):
    """Table rows are stored in a permutation of colex order; rows of at most 16 entries keep colex
    order, and the grouped order lets readers skip at least as many 128-byte lines as colex."""
    K = k - 1
    for m in range(0, k):
        o = cc.entry_order(k, m)
        W = math.comb(K, m)
        assert sorted(o.tolist()) == list(range(W))
        if W <= 16:
            assert o.tolist() == list(range(W))
            continue
        colex = [x for x in range(1 << K) if bin(x).count("1") == m]
        stored = [colex[r] for r in o]
        assert _line_skips(stored, K) >= _line_skips(colex, K)
        if m >= 1 and math.comb(K - 1, m - 1) >= 16:
            # 16 sets share a colour, so the first line is made of such sets
            common = (1 << K) - 1
            for x in stored[:16]:
                common &= x
            assert common != 0, (k, m)
    for bad in ((0, 0), (17, 1), (5, -1), (5, 5)):
        with pytest.raises(cc.CCError):
            cc.entry_order(*bad)
    with pytest.raises(cc.CCError):
        cc._check(cc.lib().cc_entry_order(5, 2, None, 6))


def test_entry_order_line_counts():
    """Expected 128-byte lines a reader fetches per row (bench.py's line model over the library's
    order): 21.7 of 29 for the 462-entry rows of 12-vertex templates (25.4 in colex order), 17.5 of
    21 for the 330-entry rows (19.2 in colex order)."""
    import bench
    assert abs(bench.needed_lines(12, 6) - 21.727) < 1e-3
    assert abs(bench.needed_lines(12, 5) - 17.455) < 1e-3
    K = 11
    for p, colex_lines in ((6, 25.36), (5, 19.18)):
        colex = [x for x in range(1 << K) if bin(x).count("1") == p - 1]
        total = sum(any(not (colex[j] >> x) & 1 for j in range(l, min(l + 16, len(colex))))
                    for x in range(K) for l in range(0, len(colex), 16))
        assert abs(total / K - colex_lines) < 0.01
        assert bench.needed_lines(12, p) < total / K


def test_epsilon_delta_estimate_on_brute_force():
    """Algorithm 1 end to end on the host: the driver's sample sizes, colourful counts of each
    colouring (oracle), the median of group means; the result is within epsilon of the number of
    copies counted by brute force (a statistical pin; seeds fixed)."""
    rp, cl = inputs.er_graph(14, 30, 5)
    for T in (inputs.path_tree(3), inputs.star_tree(4)):
        k = len(T) + 1
        copies = oracle.brute_count(rp, cl, None, T, root=0) / oracle.aut(T)
        eps, delta = 0.5, 0.1
        s, t = cc.iterations(k, eps, delta)
        X = [oracle.count(rp, cl, oracle.colour(77, j, 14, k), T) for j in range(s * t)]
        p = cc.Plan(T, bind=False)
        est = cc.estimate_median_of_means(p, X, t)
        assert abs(est - copies) <= eps * copies, (est, copies)


def test_multi_template_sharing_counts():
    """Equal rooted sub-templates are computed once: fewer splits run than the templates hold, and
    one template alone never runs more splits than it has."""
    for k in (5, 7, 8):
        plans = [cc.Plan(T, bind=False) for T in inputs.all_trees(k)]
        info = cc.Multi(plans).info
        assert info["splits"] == sum(len(p.splits) for p in plans)
        assert info["steps"] < info["splits"]
        for p in plans:
            one = cc.Multi([p]).info
            assert one["steps"] <= len(p.splits)
    # every template's root split runs, each exactly once, and steps refer to real splits
    plans = [cc.Plan(T, bind=False) for T in inputs.all_trees(7)]
    m = cc.Multi(plans)
    steps = m.steps
    assert len(steps) == m.info["steps"] and len(set(steps)) == len(steps)
    for p_i, p in enumerate(plans):
        assert (p_i, len(p.splits) - 1) in steps
    assert all(0 <= j < len(plans[p_i].splits) for p_i, j in steps)
    # a spider with three equal legs, planned without sharing: the multi-template count computes
    # the leg's tables once
    legs = [(0, 1), (1, 2), (0, 3), (3, 4), (0, 5), (5, 6)]
    p = cc.Plan(np.array(legs, dtype=np.int32), root=0, bind=False, flags=cc.CC_PLAN_NO_SHARING)
    assert cc.Multi([p]).info["steps"] < len(p.splits)
    with pytest.raises(cc.CCError):
        cc.Multi([cc.Plan(inputs.path_tree(4), bind=False), cc.Plan(inputs.path_tree(5), bind=False)])


def test_no_cpu_fallback_in_product():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1804_09764_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt
                assert "liboracle" not in txt
