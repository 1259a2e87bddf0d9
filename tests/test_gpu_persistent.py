"""The multi-template packed count in one persistent launch (cc_count_packed_multi_persistent) and
the batched path's autotuner (autotune.tune_multi).

The persistent launch runs the same device code on the same tiles as the launch-per-split count,
so its counts must be bit-identical to cc_count_packed_multi, and equal to the oracle on sampled
colourings (exact below 2^53, 1e-12 relative above)."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TWO53 = float(2 ** 53)


def _close(gpu, ref):
    if ref < TWO53:
        assert gpu == ref, (gpu, ref)
    else:
        assert abs(gpu - ref) <= 1e-12 * ref, (gpu, ref)


@pytest.mark.parametrize("k,B,tune", [(5, 7, {}), (7, 64, {}), (7, 33, {"hub_threshold": 64, "chunk": 64}),
                                      (6, 16, {"packed_tile": 128}), (5, 1, {}),
                                      (6, 130, {"hub_threshold": 64, "chunk": 64})])
def test_persistent_equals_launch_per_split_and_oracle(dev, k, B, tune):
    import torch
    import paper_1804_09764_amd as cc
    rp, cl = inputs.rmat_graph(11, 16, 6)
    G = cc.Graph.from_numpy(rp, cl, **tune)
    trees = inputs.all_trees(k)
    plans = [cc.Plan(T) for T in trees]
    m = cc.Multi(plans)
    C = cc.colour(G, k, seed=21, first_iter=0, B=B)
    print(f"case: persistent multi k={k} B={B} tuning={tune}", flush=True)
    X1 = m.count(G, C)
    X2 = m.count(G, C, persistent=True)
    X3 = m.count(G, C, persistent=True)  # a second call reuses the descriptors
    torch.cuda.synchronize()
    x1, x2, x3 = X1.cpu().numpy(), X2.cpu().numpy(), X3.cpu().numpy()
    np.testing.assert_array_equal(x2, x1)
    np.testing.assert_array_equal(x3, x1)
    Ch = C.cpu().numpy()
    for t, T in enumerate(trees):
        b = (t * 5) % B
        _close(float(x2[t, b]), oracle.count(rp, cl, Ch[b], T))


def test_persistent_rmat18_trees7x64_against_oracle(dev):
    """The batched benchmark configuration: R-MAT 18 (edge factor 16, seed 2), the 11 trees with 7
    vertices, 64 colourings; sampled colourings against the oracle."""
    import torch
    import paper_1804_09764_amd as cc
    rp_d, col_d = inputs.rmat_graph_gpu(18, 16, 2, device=dev)
    G = cc.Graph(rp_d, col_d)
    trees = inputs.all_trees(7)
    m = cc.Multi([cc.Plan(T) for T in trees])
    C = cc.colour(G, 7, seed=777, first_iter=0, B=64)
    Xp = m.count(G, C, persistent=True)
    Xm = m.count(G, C)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Xp.cpu().numpy(), Xm.cpu().numpy())
    rp, col = rp_d.cpu().numpy(), col_d.cpu().numpy()
    Ch = C.cpu().numpy()
    Xh = Xp.cpu().numpy()
    for t in (0, 5, 10):
        print(f"case: R-MAT 18 persistent tree {t} against the oracle", flush=True)
        _close(float(Xh[t, 63 - t]), oracle.count(rp, col, Ch[63 - t], trees[t]))


def test_persistent_refuses_wide_splits(dev):
    import paper_1804_09764_amd as cc
    rp, cl = inputs.er_graph(200, 800, 3)
    G = cc.Graph.from_numpy(rp, cl)
    m = cc.Multi([cc.Plan(inputs.path_tree(12))])
    C = cc.colour(G, 12, seed=1, first_iter=0, B=4)
    with pytest.raises(cc.CCError) as e:
        m.count(G, C, persistent=True)
    assert e.value.status == -2


def test_tune_multi_choice_and_parity(dev, tmp_path):
    import torch
    import paper_1804_09764_amd as cc
    from paper_1804_09764_amd import autotune
    rp, cl = inputs.rmat_graph(11, 16, 8)
    rp_d, cl_d = torch.from_numpy(rp).cuda(), torch.from_numpy(cl).cuda()
    trees = inputs.all_trees(6)
    plans = [cc.Plan(T) for T in trees]
    cache = str(tmp_path / "tune.json")
    print("case: tune_multi rmat11 k=6 B=16", flush=True)
    rec = autotune.tune_multi(plans, rp_d, cl_d, B=16, seed=4, repeats=1, cache_path=cache)
    assert rec.ms == min(rec.timings.values())
    assert len(rec.timings) == len(autotune.candidates(len(cl), int(np.diff(rp).max()))) + len(autotune.TILES) - 1
    assert autotune.tune_multi(plans, rp_d, cl_d, B=16, seed=4, repeats=1, cache_path=cache) == rec
    G = cc.Graph(rp_d, cl_d, hub_threshold=rec.hub_threshold, chunk=rec.chunk, packed_tile=rec.packed_tile)
    C = cc.colour(G, 6, seed=4, first_iter=0, B=16)
    X = cc.Multi(plans).count(G, C, persistent=True)
    torch.cuda.synchronize()
    Ch = C.cpu().numpy()
    for t, T in enumerate(trees):
        _close(float(X.cpu().numpy()[t, t]), oracle.count(rp, cl, Ch[t], T))
