"""Input generators: C builder equals its numpy twin; graphs are simple and symmetric."""
import numpy as np
import pytest

import inputs


@pytest.mark.parametrize("scale,ef,seed", [(4, 8, 1), (9, 16, 2), (12, 4, 3)])
def test_rmat_c_equals_numpy(scale, ef, seed):
    a = inputs.rmat_graph(scale, ef, seed)
    b = inputs.rmat_graph_np(scale, ef, seed)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    inputs.check_csr(*a)


def test_rmat_is_skewed_and_relabelled():
    rp, cl = inputs.rmat_graph(14, 16, 1)
    deg = np.diff(rp)
    assert deg.max() > 20 * deg.mean()
    # hubs are spread over the id range, not piled at low ids
    top = np.argsort(deg)[-50:]
    assert top.min() < (1 << 13) < top.max()


def test_er_graph():
    rp, cl = inputs.er_graph(1000, 5000, 1)
    inputs.check_csr(rp, cl)
    assert len(cl) == 10000


def test_check_csr_rejects():
    rp, cl = inputs.cycle_graph(6)
    inputs.check_csr(rp, cl)
    bad = cl.copy()
    bad[0] = 0  # self loop at vertex 0
    with pytest.raises(ValueError):
        inputs.check_csr(rp, bad)
    rp2, cl2 = inputs.csr_from_edges(4, [(0, 1), (1, 2)])
    cl3 = cl2.copy()
    cl3[-1] = 3  # breaks symmetry
    with pytest.raises(ValueError):
        inputs.check_csr(rp2, cl3)


def test_tree_counts_oeis_a000055():
    assert [len(inputs.all_trees(k)) for k in range(1, 13)] == [1, 1, 1, 2, 3, 6, 11, 23, 47, 106, 235, 551]


@pytest.mark.parametrize("k", [1, 2, 3, 7, 12, 15])
def test_pruefer_is_tree(k):
    e = inputs.pruefer_tree(k, 12)
    assert e.shape == (k - 1, 2)
    parent = list(range(k))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v in e:
        ru, rv = find(int(u)), find(int(v))
        assert ru != rv
        parent[ru] = rv


@pytest.mark.gpu
@pytest.mark.parametrize("scale,ef,seed", [(6, 4, 1), (12, 16, 2), (15, 64, 3), (16, 8, 4)])
def test_rmat_gpu_builder_equals_cpu(scale, ef, seed):
    import torch
    rp_g, col_g = inputs.rmat_graph_gpu(scale, ef, seed, device="cuda:0")
    rp, cl = inputs.rmat_graph(scale, ef, seed)
    np.testing.assert_array_equal(rp_g.cpu().numpy(), rp)
    np.testing.assert_array_equal(col_g.cpu().numpy(), cl)
