"""GPU: the degree-split autotuner times every candidate, keeps the fastest, caches the record,
and a graph prepared with the chosen parameters counts exactly as the oracle."""
import json

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


def test_tune_choice_cache_and_parity(dev, tmp_path):
    import torch
    import paper_1804_09764_amd as cc
    from paper_1804_09764_amd import autotune
    rp, cl = inputs.rmat_graph(10, 16, 4)
    rp_d = torch.from_numpy(rp).cuda()
    cl_d = torch.from_numpy(cl).cuda()
    T = inputs.pruefer_tree(7, 5)
    P = cc.Plan(T)
    cache = str(tmp_path / "tune.json")
    print("case: autotune rmat10 k=7", flush=True)
    rec = autotune.tune(P, rp_d, cl_d, seed=3, repeats=1, cache_path=cache)
    max_degree = int(np.diff(rp).max())
    cand = autotune.candidates(len(cl), max_degree)
    assert len(rec.timings) == len(cand)
    assert rec.ms == min(rec.timings.values()) and (rec.hub_threshold, rec.chunk) in cand
    stored = json.load(open(cache))
    assert len(stored) == 1
    again = autotune.tune(P, rp_d, cl_d, seed=3, repeats=1, cache_path=cache)  # served from the cache
    assert again == rec
    G = cc.Graph(rp_d, cl_d, hub_threshold=rec.hub_threshold, chunk=rec.chunk)
    col = oracle.colour(3, 0, len(rp) - 1, 7)
    X = cc.count(P, G, torch.from_numpy(col).cuda())
    torch.cuda.synchronize()
    assert float(X.cpu()[0]) == oracle.count(rp, cl, col, T)
