"""Host-side checks of the degree-split autotuner's candidate grid and record keys (no GPU)."""
import json
import math

import inputs
import paper_1804_09764_amd as cc
from paper_1804_09764_amd import autotune


def test_candidates_grid():
    c = autotune.default_chunk(10 ** 6)
    assert c == 512 and autotune.default_chunk(1 << 28) == 2048
    cand = autotune.candidates(10 ** 6, 100000)
    assert cand[0] == (2 * c, c)                       # the library default first
    assert len(cand) == len(set(cand)) == 9
    for tau, ch in cand:
        assert ch % 64 == 0 and ch >= 64 and tau >= ch
    assert {ch for _, ch in cand} == {256, 512, 1024}


def test_candidates_collapse_when_no_row_is_cut():
    # largest degree 300: every tau >= 300 cuts no row, so those candidates merge
    cand = autotune.candidates(10 ** 5, 300)
    assert cand == [(1024, 512), (256, 256), (300, 256), (512, 512), (1024, 1024)]


def test_record_key_separates_what_decides_the_choice():
    P12 = cc.Plan(inputs.pruefer_tree(12, 12), bind=False)
    P7 = cc.Plan(inputs.pruefer_tree(7, 1), bind=False)
    k1 = autotune.record_key(P12, 1 << 20, 31 << 20, 60000, "gpu")
    assert k1 == autotune.record_key(P12, 1 << 20, 31 << 20, 50000, "gpu")   # same log2 bucket
    assert k1 != autotune.record_key(P12, 1 << 20, 31 << 20, 20000, "gpu")
    assert k1 != autotune.record_key(P7, 1 << 20, 31 << 20, 60000, "gpu")
    assert k1 != autotune.record_key(P12, 1 << 20, 31 << 20, 60000, "other")
    d = json.loads(k1)
    assert d["k"] == 12 and d["passive_widths"] == [math.comb(11, p - 1) for (_, _, p) in P12.splits]
