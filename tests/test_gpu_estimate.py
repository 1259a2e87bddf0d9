"""Algorithm 1 end to end on the GPU: the (epsilon, delta) driver's sample sizes (cc_iterations),
the colourings (cc_color), the colourful counts (cc_count_packed, cc_count) and the median of
group means (cc_estimate_median_of_means). Every colouring's count must equal the oracle's, and
the estimate must lie within epsilon of the number of copies found by brute force (a statistical
pin of the method, Section 2.1; seeds fixed, so the run is deterministic)."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["path3", "star4"])
def test_epsilon_delta_estimate_on_the_gpu(dev, which):
    import torch
    import paper_1804_09764_amd as cc
    rp, cl = inputs.er_graph(14, 30, 5)
    T = inputs.path_tree(3) if which == "path3" else inputs.star_tree(4)
    k = len(T) + 1
    copies = oracle.brute_count(rp, cl, None, T, root=0) / oracle.aut(T)
    eps, delta = 0.5, 0.1
    s, t = cc.iterations(k, eps, delta)
    total = s * t
    print(f"case: {which} k={k} colourings {s} x {t} groups", flush=True)
    G = cc.Graph.from_numpy(rp, cl)
    P = cc.Plan(T)
    C = cc.colour(G, k, seed=77, first_iter=0, B=total)
    X = torch.empty(total, dtype=torch.float64, device=dev)
    step = cc.CC_MAX_PACKED
    for b0 in range(0, total, step):
        cc.count_packed(P, G, C[b0:b0 + step], out=X[b0:b0 + step])
    Xp = cc.count(P, G, C[:64])
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    Ch = C.cpu().numpy()
    Xo = np.array([oracle.count(rp, cl, Ch[j], T) for j in range(total)])
    np.testing.assert_array_equal(Xh, Xo)
    np.testing.assert_array_equal(Xp.cpu().numpy(), Xo[:64])
    # the colouring kernel is the oracle's hash colouring
    for j in (0, 1, total - 1):
        np.testing.assert_array_equal(Ch[j], oracle.colour(77, j, 14, k))
    est = cc.estimate_median_of_means(P, Xh, t)
    assert abs(est - copies) <= eps * copies, (est, copies)
