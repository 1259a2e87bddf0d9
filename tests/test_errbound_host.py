"""The guaranteed error bound of the FP64 counts (paper_1804_09764_amd.errbound) on the benchmark
configurations, and the roundings of the blocked sum it models."""
import math

import inputs
import paper_1804_09764_amd as cc
from paper_1804_09764_amd import errbound as eb


def walked_blocked_len(n):
    """Longest chain of roundings in the blocked order, by walking it: every addition a + b with both
    sides nonzero rounds once, and each term's count grows by one for each rounding of a sum it is
    part of (the first addition of each accumulator is onto zero and exact)."""
    def add(acc, part):  # acc, part: lists of (term, roundings)
        if not acc:
            return list(part)
        return [(i, d + 1) for i, d in acc + part]
    total = []
    for g in range(0, n, 256):
        gs = []
        for b in range(g, min(n, g + 256), 16):
            bs = []
            for i in range(b, min(n, b + 16)):
                bs = add(bs, [(i, 0)])
            gs = add(gs, bs)
        total = add(total, gs)
    return max((d for _, d in total), default=0)


def test_blocked_len_values():
    assert eb.blocked_len(0) == 0 and eb.blocked_len(1) == 0
    assert eb.blocked_len(2) == 1
    assert eb.blocked_len(16) == 15
    assert eb.blocked_len(17) == 16          # a second run: 15 inside the first, 1 between runs
    assert eb.blocked_len(256) == 30
    assert eb.blocked_len(257) == 31          # a second group
    assert eb.blocked_len(690) == 32          # the largest cut row of R-MAT 23 / ef 256 (chunks of 2048)
    assert eb.blocked_len(3432) == 15 + 15 + 13
    for n in list(range(0, 40)) + [255, 256, 257, 511, 512, 513, 690, 1000, 3432]:
        assert eb.blocked_len(n) == walked_blocked_len(n), n


def _bound(T, n, maxdeg, tau, c, path="plain"):
    P = cc.Plan(T, bind=False)
    return eb.plan_bound(P, dict(n=n, max_degree=maxdeg, hub_threshold=tau, chunk=c), path)


def test_bound_headline_configs_below_tolerance():
    # R-MAT 23 / ef 256 (largest degree 1 411 364, default hub threshold 4096, chunks of 2048),
    # 12-vertex tree; R-MAT 20 / ef 16 (largest degree below 2^17, 1024 / 512), 15- and 12-vertex trees
    c3a = _bound(inputs.pruefer_tree(12, 12), 2 ** 23, 1411364, 4096, 2048)
    c3b = _bound(inputs.pruefer_tree(15, 15), 2 ** 20, 1 << 17, 1024, 512)
    c1 = _bound(inputs.pruefer_tree(12, 12), 2 ** 20, 1 << 17, 1024, 512)
    for b in (c3a, c3b, c1):
        assert b["X_rel"] < 0.5e-12, b["X_rel"]
        # the local terms the budget is made of
        for r in b["splits"]:
            assert r["L_split"] <= 64 and r["L_nbr"] <= 63 + r["p"] * 64


def test_bound_batched_config_below_tolerance():
    # R-MAT 18 / ef 16, every 7-vertex tree, packed rows (terms in CSR order per entry)
    for T in inputs.all_trees(7):
        b = _bound(T, 2 ** 18, 1 << 15, 1024, 512, "packed")
        assert b["X_rel"] < 1e-12, b["X_rel"]


def test_bound_grows_with_hub_threshold_on_packed_rows():
    """Packed rows add a light row's terms one by one: the bound follows the hub threshold, and at
    the 4096 default of graphs above 2^28 entries it exceeds 1e-12 for the 12-vertex tree (the plain
    path, whose runs are folded per 64-entry block, stays far below)."""
    T = inputs.pruefer_tree(12, 12)
    small = _bound(T, 2 ** 23, 1411364, 1024, 512, "packed")["X_rel"]
    large = _bound(T, 2 ** 23, 1411364, 4096, 2048, "packed")["X_rel"]
    assert small < 1e-12 < large
    assert _bound(T, 2 ** 23, 1411364, 4096, 2048, "plain")["X_rel"] < 0.25e-12


def test_bound_sums_every_use_of_a_shared_table():
    """A sub-template table read twice contributes its error twice: the bound on the shared plan
    equals the bound on the unshared partition with the same splits."""
    T = inputs.pruefer_tree(12, 12)
    shared = cc.Plan(T, bind=False)
    full = cc.Plan(T, bind=False, root=shared.info.root, flags=cc.CC_PLAN_NO_SHARING)
    gi = dict(n=2 ** 20, max_degree=1 << 16, hub_threshold=1024, chunk=512)
    assert full.info.n_splits >= shared.info.n_splits
    assert math.isclose(eb.plan_bound(shared, gi)["X_rel"], eb.plan_bound(full, gi)["X_rel"])
