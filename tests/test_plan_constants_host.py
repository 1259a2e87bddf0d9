"""The planner's constant tables, read back on the host, reproduce the oracle's counts.

A plain evaluation of Eq. 1 (Section 2.1) in numpy that takes every map from the plan's device
constants (split lists, output-to-N maps, fold maps, colour-set masks, in the tables' storage
order) must equal the oracle exactly, per vertex. The masks must agree with the fold maps' drop
rule, the packed layout's maps must name the same colour sets as the fold maps, and the count
through the packed maps (neighbour sums over all k colours) must equal the oracle too. No GPU:
these are the tables the kernels read, checked before any kernel runs.
"""
from math import comb

import numpy as np
import pytest

import inputs
import oracle
import paper_1804_09764_amd as cc

NO = 0xFFFF


def _u16(C, off, count):
    return np.frombuffer(C[off:off + 2 * count].tobytes(), dtype=np.uint16).astype(np.int64)


def _u32(C, off, count):
    return np.frombuffer(C[off:off + 4 * count].tobytes(), dtype=np.uint32).astype(np.int64)


def host_count(P, rp, cl, col):
    """X and per-vertex root counts from the plan's constants (all colours valid)."""
    k = P.k
    K = k - 1
    C = P.constants()
    n = len(rp) - 1
    tables = {}
    for i, (s, a, p) in enumerate(P.splits):
        m = P.split_maps(i)
        Wp, Ws, Nw = comb(K, p - 1), comb(K, s - 1), comb(K, p)
        N = np.zeros((n, Nw))
        fold = _u16(C, m["fold_off"], k * k * Wp).reshape(k, k, Wp) if p >= 2 else None
        Tp = tables[m["pas"]] if p >= 2 else None
        for v in range(n):
            cv = int(col[v])
            for u in cl[rp[v]:rp[v + 1]]:
                cu = int(col[u])
                if cu == cv:
                    continue
                if p == 1:
                    N[v, cu - (cu > cv)] += 1.0
                else:
                    f = fold[cu, cv]
                    keep = f != NO
                    np.add.at(N[v], f[keep], Tp[u][keep])
        if a == 1:
            O = N[:, _u32(C, m["split_off"], Ws)]
        else:
            npairs = comb(s - 1, p)
            pairs = _u32(C, m["split_off"], npairs * Ws).reshape(npairs, Ws)
            O = (tables[m["act"]][:, pairs & 0xFFFF] * N[:, pairs >> 16]).sum(axis=1)
        if m["out"] == -2:
            return float(O[:, 0].sum()), O[:, 0]
        tables[m["out"]] = O
    raise AssertionError("no split writes the full template")


def host_count_packed(P, rp, cl, col):
    """The same count through the packed layout's maps: neighbour sums over all k colours
    (C(k, p) entries, FM places passive entry j of a neighbour of colour c), entries whose set
    holds col(v) skipped by the mask, and E reading them back per output entry."""
    k = P.k
    K = k - 1
    C = P.constants()
    n = len(rp) - 1
    tables = {}
    for i, (s, a, p) in enumerate(P.splits):
        m = P.split_maps(i)
        Wp, Ws, Nw, Cf = comb(K, p - 1), comb(K, s - 1), comb(K, p), comb(k, p)
        E = _u16(C, m["emap_off"], k * Nw).reshape(k, Nw)
        FM = _u16(C, m["full_off"], k * Wp).reshape(k, Wp) if p >= 2 else None
        mask = _u16(C, m["mask_off"], Wp) if p >= 2 else None
        Tp = tables[m["pas"]] if p >= 2 else None
        Nf = np.zeros((n, Cf))
        for v in range(n):
            cv = int(col[v])
            for u in cl[rp[v]:rp[v + 1]]:
                c = int(col[u])
                if c == cv:
                    continue
                if p == 1:
                    Nf[v, c] += 1.0          # the full-space rank of {c} is c
                else:
                    need = ((mask >> (cv - (cv > c))) & 1) == 0
                    np.add.at(Nf[v], FM[c][need], Tp[u][need])
        Ev = E[np.asarray(col, dtype=np.int64)]                             # [n, Nw]: E[col(v)]
        if a == 1:
            O = Nf[np.arange(n)[:, None], Ev[:, :Ws]]
        else:
            npairs = comb(s - 1, p)
            pairs = _u32(C, m["split_off"], npairs * Ws).reshape(npairs, Ws)
            A = tables[m["act"]][:, pairs & 0xFFFF]                           # [n, npairs, Ws]
            O = (A * Nf[np.arange(n)[:, None, None], Ev[:, pairs >> 16]]).sum(axis=1)
        if m["out"] == -2:
            return float(O[:, 0].sum()), O[:, 0]
        tables[m["out"]] = O
    raise AssertionError("no split writes the full template")


CASES = [(k, T) for k in (2, 3, 5, 7) for T in inputs.all_trees(k)] + \
        [(k, T) for k in (9, 10, 11) for T in (inputs.path_tree(k), inputs.star_tree(k),
                                                inputs.pruefer_tree(k, 1), inputs.pruefer_tree(k, 2))]


@pytest.mark.parametrize("flags", [0, cc.CC_PLAN_NO_SHARING])
def test_constants_reproduce_oracle(flags):
    rp, cl = inputs.er_graph(24, 80, 5)
    n = len(rp) - 1
    for ci, (k, T) in enumerate(CASES):
        col = oracle.colour(100 + ci, 0, n, k)
        P = cc.Plan(T, bind=False, flags=flags)
        X, V = host_count(P, rp, cl, col)
        Xo, Vo = oracle.count(rp, cl, col, T, root=P.info.root, per_vertex=True)
        assert Xo < 2 ** 53
        np.testing.assert_array_equal(V, Vo, err_msg=f"k={k} case {ci}")
        assert X == Xo


def test_packed_maps_reproduce_oracle():
    rp, cl = inputs.er_graph(24, 80, 6)
    n = len(rp) - 1
    for ci, (k, T) in enumerate(CASES):
        col = oracle.colour(200 + ci, 0, n, k)
        P = cc.Plan(T, bind=False)
        X, V = host_count_packed(P, rp, cl, col)
        Xo, Vo = oracle.count(rp, cl, col, T, root=P.info.root, per_vertex=True)
        np.testing.assert_array_equal(V, Vo, err_msg=f"k={k} case {ci}")
        assert X == Xo


def test_constants_every_root():
    rp, cl = inputs.er_graph(20, 60, 8)
    n = len(rp) - 1
    T = inputs.pruefer_tree(10, 7)
    col = oracle.colour(3, 0, n, 10)
    for root in range(10):
        P = cc.Plan(T, root=root, bind=False)
        X, V = host_count(P, rp, cl, col)
        Xo, Vo = oracle.count(rp, cl, col, T, root=root, per_vertex=True)
        np.testing.assert_array_equal(V, Vo)
        assert X == Xo


@pytest.mark.parametrize("k", [6, 9, 12, 14])
def test_masks_and_packed_maps_agree_with_fold_maps(k):
    K = k - 1
    P = cc.Plan(inputs.pruefer_tree(k, 3), bind=False)
    C = P.constants()
    for i, (s, a, p) in enumerate(P.splits):
        if p < 2:
            continue
        m = P.split_maps(i)
        Wp, Ws, Nw = comb(K, p - 1), comb(K, s - 1), comb(K, p)
        fold = _u16(C, m["fold_off"], k * k * Wp).reshape(k, k, Wp)
        mask = _u16(C, m["mask_off"], Wp)
        FM = _u16(C, m["full_off"], k * Wp).reshape(k, Wp)
        E = _u16(C, m["emap_off"], k * Nw).reshape(k, Nw)
        if a == 1:
            # E runs over output positions; position r holds N's entry omap[r]
            omap = _u32(C, m["split_off"], Ws)
            pos_of = np.empty(Nw, dtype=np.int64)
            pos_of[omap] = np.arange(Ws)
        for cu in range(k):
            for cv in range(k):
                if cu == cv:
                    continue
                x = cv - (cv > cu)
                dropped = fold[cu, cv] == NO
                np.testing.assert_array_equal(dropped, (mask >> x) & 1 == 1)
                f = fold[cu, cv][~dropped]
                q = pos_of[f] if a == 1 else f
                np.testing.assert_array_equal(FM[cu][~dropped], E[cv][q])


def _colex_masks(K, m):
    return [x for x in range(1 << K) if bin(x).count("1") == m]


def _squeeze(mask, c):
    """The set `mask` written over the colours other than c (bit c removed, higher bits shifted)."""
    return (mask & ((1 << c) - 1)) | ((mask >> (c + 1)) << c)


@pytest.mark.parametrize("k", [10, 12, 14])
def test_projected_maps_name_the_needed_sets(k):
    """Projected rows: for a neighbour of colour cu and a centre of colour cv, entry j is the j-th
    colour set Q (|Q| = p, cu in Q, cv not in Q) in colex order; its source is the position of
    Q \\ {cu} in the neighbour's stored row and its target the rank of Q among the p-sets over the
    colours other than cv. Derived here from the sets, not from the fold map."""
    K = k - 1
    P = cc.Plan(inputs.pruefer_tree(k, 3), bind=False)
    C = P.constants()
    seen = 0
    for i, (s, a, p) in enumerate(P.splits):
        m = P.split_maps(i)
        Wp = comb(K, p - 1)
        if p < 2 or Wp <= 64:
            assert m["Wn"] == 0 and m["proj_src_off"] == -1
            continue
        seen += 1
        Wn = comb(k - 2, p - 1)
        assert m["Wn"] == Wn
        src = _u16(C, m["proj_src_off"], k * k * Wn).reshape(k, k, Wn)
        dst = _u16(C, m["proj_fold_off"], k * k * Wn).reshape(k, k, Wn)
        order = cc.entry_order(k, p - 1)
        pos_of_rank = np.empty(len(order), dtype=np.int64)
        pos_of_rank[order] = np.arange(len(order))
        row_rank = {x: r for r, x in enumerate(_colex_masks(K, p - 1))}
        n_rank = {x: r for r, x in enumerate(_colex_masks(K, p))}
        for cu in range(k):
            for cv in range(k):
                if cu == cv:
                    continue
                Qs = [Q for Q in _colex_masks(k, p) if (Q >> cu) & 1 and not (Q >> cv) & 1]
                assert len(Qs) == Wn
                want_src = [pos_of_rank[row_rank[_squeeze(Q & ~(1 << cu), cu)]] for Q in Qs]
                want_dst = [n_rank[_squeeze(Q, cv)] for Q in Qs]
                np.testing.assert_array_equal(src[cu, cv], want_src)
                np.testing.assert_array_equal(dst[cu, cv], want_dst)
    assert seen > 0


def host_count_projected(P, rp, cl, col):
    """Eq. 1 with every wide neighbour sum read through the projected rows: a centre of colour cv
    adds, for each neighbour u, the row proj[cv][u] = T[u][src[col(u), cv]] at N[dst[col(u), cv]]."""
    k = P.k
    K = k - 1
    C = P.constants()
    n = len(rp) - 1
    tables = {}
    for i, (s, a, p) in enumerate(P.splits):
        m = P.split_maps(i)
        Wp, Ws, Nw = comb(K, p - 1), comb(K, s - 1), comb(K, p)
        N = np.zeros((n, Nw))
        Tp = tables[m["pas"]] if p >= 2 else None
        if m["Wn"] > 0:
            Wn = m["Wn"]
            src = _u16(C, m["proj_src_off"], k * k * Wn).reshape(k, k, Wn)
            dst = _u16(C, m["proj_fold_off"], k * k * Wn).reshape(k, k, Wn)
        elif p >= 2:
            fold = _u16(C, m["fold_off"], k * k * Wp).reshape(k, k, Wp)
        for v in range(n):
            cv = int(col[v])
            for u in cl[rp[v]:rp[v + 1]]:
                cu = int(col[u])
                if cu == cv:
                    continue
                if p == 1:
                    N[v, cu - (cu > cv)] += 1.0
                elif m["Wn"] > 0:
                    N[v, dst[cu, cv]] += Tp[u][src[cu, cv]]
                else:
                    f = fold[cu, cv]
                    keep = f != NO
                    np.add.at(N[v], f[keep], Tp[u][keep])
        if a == 1:
            O = N[:, _u32(C, m["split_off"], Ws)]
        else:
            npairs = comb(s - 1, p)
            pairs = _u32(C, m["split_off"], npairs * Ws).reshape(npairs, Ws)
            O = (tables[m["act"]][:, pairs & 0xFFFF] * N[:, pairs >> 16]).sum(axis=1)
        if m["out"] == -2:
            return float(O[:, 0].sum()), O[:, 0]
        tables[m["out"]] = O
    raise AssertionError("no split writes the full template")


def test_projected_rows_reproduce_oracle():
    rp, cl = inputs.er_graph(24, 80, 9)
    n = len(rp) - 1
    cases = [(k, T) for k in (9, 10, 11, 12) for T in (inputs.path_tree(k), inputs.star_tree(k),
                                                        inputs.pruefer_tree(k, 4))]
    wide = 0
    for ci, (k, T) in enumerate(cases):
        col = oracle.colour(300 + ci, 0, n, k)
        P = cc.Plan(T, bind=False)
        wide += sum(P.split_maps(i)["Wn"] > 0 for i in range(P.info.n_splits))
        X, V = host_count_projected(P, rp, cl, col)
        Xo, Vo = oracle.count(rp, cl, col, T, root=P.info.root, per_vertex=True)
        np.testing.assert_array_equal(V, Vo, err_msg=f"k={k} case {ci}")
        assert X == Xo
    assert wide >= 6
