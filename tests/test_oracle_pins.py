"""Pins for the oracle against facts fixed by the paper and by combinatorics (no GPU).

Each test pins the oracle to something other than itself: brute-force enumeration, the exact
all-colourings identity, closed forms on cycles / stars / cliques, the Cayley identity for
automorphism counts, the paper's worked example and its over-count remark.
"""
import json
import math
import os
from itertools import combinations, product

import numpy as np
import pytest

import inputs
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _colex_index(mask: int, k: int) -> int:
    """Position of `mask` among the masks of equal popcount in increasing numeric order."""
    pc = bin(mask).count("1")
    return sum(1 for m in range(mask) if bin(m).count("1") == pc)


# ---------------------------------------------------------------- P1: brute force -------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_tiny_all_trees(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 12))
    m = int(rng.integers(n, min(3 * n, n * (n - 1) // 2)))
    rp, cl = inputs.er_graph(n, m, seed)
    for k in range(1, 7):
        for T in inputs.all_trees(k):
            col = inputs.colours(n, k, seed * 100 + k)
            for root in range(k):
                for rule in (0, 1):
                    X, pv = oracle.count(rp, cl, col, T, root=root, rule=rule, per_vertex=True)
                    b, bpv = oracle.brute_count(rp, cl, col, T, root=root, per_vertex=True)
                    assert X == b
                    np.testing.assert_array_equal(pv, bpv.astype(np.float64))


def test_brute_force_c0_path5():
    """ER n=1000, m=5000, the 5-vertex path, one uniform colouring with 5 colours."""
    rp, cl = inputs.er_graph(1000, 5000, 1)
    col = inputs.colours(1000, 5, 7)
    T = inputs.path_tree(5)
    for root in (0, 2):
        X, pv = oracle.count(rp, cl, col, T, root=root, per_vertex=True)
        b, bpv = oracle.brute_count(rp, cl, col, T, root=root, per_vertex=True)
        assert X == b > 0
        np.testing.assert_array_equal(pv, bpv.astype(np.float64))


def test_brute_force_random_trees_k8():
    rp, cl = inputs.er_graph(40, 120, 11)
    for seed in range(4):
        T = inputs.pruefer_tree(8, seed)
        col = inputs.colours(40, 8, seed)
        X = oracle.count(rp, cl, col, T)
        assert X == oracle.brute_count(rp, cl, col, T, root=3)


# ---------------------------------------------------------------- P2: all colourings ---------

@pytest.mark.parametrize("n,k", [(7, 4), (6, 5), (8, 3)])
def test_all_colourings_identity(n, k):
    """sum over all k^n colourings of X(col) = k! * k^(n-k) * #injective homomorphisms(T, G).

    An injective map of the k template vertices is colourful in exactly k! * k^(n-k) of the k^n
    colourings (its k images take distinct colours in k! ways, the other n-k vertices are free).
    """
    rp, cl = inputs.er_graph(n, min(2 * n, n * (n - 1) // 2), n * 10 + k)
    for T in inputs.all_trees(k):
        inj = oracle.brute_count(rp, cl, None, T, root=0)
        total = 0
        for colouring in product(range(k), repeat=n):
            total += oracle.count(rp, cl, np.array(colouring, dtype=np.uint8), T)
        assert total == math.factorial(k) * k ** (n - k) * inj


# ---------------------------------------------------------------- P3: closed forms -----------

@pytest.mark.parametrize("k,reps", [(3, 2), (4, 3), (5, 2), (6, 1)])
def test_cycle_closed_form(k, reps):
    n = k * reps
    rp, cl = inputs.cycle_graph(n)
    col = (np.arange(n) % k).astype(np.uint8)
    assert oracle.count(rp, cl, col, inputs.path_tree(k)) == 2 * n
    for T in inputs.all_trees(k):
        if max(np.bincount(T.reshape(-1), minlength=k)) >= 3:
            assert oracle.count(rp, cl, col, T) == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_star_closed_form(seed):
    m = 17
    rp, cl = inputs.star_graph(m)
    for k in (3, 4, 5, 6):
        col = inputs.colours(m + 1, k, seed + 10 * k)
        c0 = int(col[0])
        nq = np.bincount(col[1:], minlength=k)
        want = math.factorial(k - 1) * math.prod(int(nq[q]) for q in range(k) if q != c0)
        assert oracle.count(rp, cl, col, inputs.star_tree(k)) == want
        # the 3-vertex path: middle at the centre, two leaves of different colours (ordered)
        col3 = inputs.colours(m + 1, 3, seed)
        c0 = int(col3[0])
        nq = np.bincount(col3[1:], minlength=3)
        others = [q for q in range(3) if q != c0]
        want3 = 2 * int(nq[others[0]]) * int(nq[others[1]])
        assert oracle.count(rp, cl, col3, inputs.path_tree(3)) == want3


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7])
def test_clique_closed_form(k):
    rp, cl = inputs.clique_graph(k)
    col = np.arange(k, dtype=np.uint8)
    for T in inputs.all_trees(k):
        assert oracle.count(rp, cl, col, T) == math.factorial(k)


def test_k1_and_k2():
    rp, cl = inputs.er_graph(300, 900, 4)
    assert oracle.count(rp, cl, np.zeros(300, np.uint8), np.zeros((0, 2), np.int32)) == 300
    col = inputs.colours(300, 2, 9)
    src = np.repeat(np.arange(300), np.diff(rp))
    want = int(np.sum(col[src] != col[cl]))
    assert oracle.count(rp, cl, col, inputs.path_tree(2)) == want


# ---------------------------------------------------------------- P5: automorphisms ----------

@pytest.mark.parametrize("k", range(1, 9))
def test_aut_matches_enumeration(k):
    for T in inputs.all_trees(k):
        assert oracle.aut(T) == oracle.brute_aut(T)


@pytest.mark.parametrize("k", range(1, 11))
def test_cayley_identity(k):
    """sum over non-isomorphic trees of k!/|Aut(T)| = number of labelled trees = k^(k-2)."""
    total = sum(math.factorial(k) // oracle.aut(T) for T in inputs.all_trees(k))
    assert total == (k ** (k - 2) if k >= 2 else 1)


def test_aut_k7_multiset():
    assert sorted(oracle.aut(T) for T in inputs.all_trees(7)) == [1, 2, 2, 2, 4, 6, 6, 8, 12, 24, 720]


# ---------------------------------------------------------------- P8: paper fragments --------

def test_worked_example_fragment():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    k, a, p = g["k"], g["active_size"], g["passive_size"]
    cid = g["colours"]

    def idx(names):
        return _colex_index(sum(1 << cid[x] for x in names), k)

    act = np.zeros((1, math.comb(k, a)))
    for names, val in g["active_counts"]:
        act[0, idx(names)] = val
    pas = np.zeros((1, math.comb(k, p)))
    for names, val in g["passive_counts"]:
        pas[0, idx(names)] = val
    out = oracle.step(k, a + p, a, np.array([0, 1]), np.array([0]), act, pas)
    assert out[0, 0] == g["expected_full_set_count"]


def test_three_path_overcount_is_two():
    """The 3-path rooted at its centre counts every embedding twice (its two leaves swap)."""
    rp, cl = inputs.er_graph(25, 70, 5)
    col = inputs.colours(25, 3, 1)
    T = inputs.path_tree(3)
    X = oracle.count(rp, cl, col, T, root=1)
    adj = {v: set(cl[rp[v]:rp[v + 1]].tolist()) for v in range(25)}
    copies = set()
    for mid in range(25):
        for x, y in combinations(sorted(adj[mid]), 2):
            if len({int(col[mid]), int(col[x]), int(col[y])}) == 3:
                copies.add((mid, x, y))
    assert oracle.aut(T) == 2
    assert X == 2 * len(copies)


# ---------------------------------------------------------------- P4: statistical smoke -------

def test_estimate_unbiased_smoke():
    n = 24
    rp, cl = inputs.er_graph(n, 50, 3)
    T = inputs.pruefer_tree(4, 2)
    k = 4
    copies = oracle.brute_count(rp, cl, None, T, root=0) // oracle.aut(T)
    ests = []
    for it in range(3000):
        col = oracle.colour(99, it, n, k)
        X = oracle.count(rp, cl, col, T)
        ests.append(oracle.estimate(k, oracle.aut(T), [X]))
    ests = np.array(ests)
    se = ests.std() / math.sqrt(len(ests))
    assert abs(ests.mean() - copies) < 5 * se + 1e-9
    # the library-level estimate is the mean, scaled once
    assert math.isclose(oracle.estimate(k, oracle.aut(T), [2.0, 4.0]),
                        3.0 * k ** k / math.factorial(k) / oracle.aut(T), rel_tol=1e-15)


def test_colouring_is_uniform_and_counter_based():
    a = oracle.colour(5, 3, 200000, 12)
    assert a.max() == 11 and a.min() == 0
    h = np.bincount(a, minlength=12) / len(a)
    assert np.all(np.abs(h - 1 / 12) < 0.005)
    # prefix stable: colour of v does not depend on n
    np.testing.assert_array_equal(oracle.colour(5, 3, 1000, 12), a[:1000])
    assert not np.array_equal(oracle.colour(5, 4, 1000, 12), a[:1000])
