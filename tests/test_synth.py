"""Invariants of the seeded workload generators (no solver arithmetic)."""

import numpy as np
import pytest

import dwn_synth as ds
from dwn_synth.generate import steady_input

from helpers import tiny_problem


@pytest.mark.parametrize("name,K,mu_tail", [("small", 19, 4), ("dwn128", 2429, 128),
                                            ("dwn2048", 30717, 2048)])
def test_tree_sizes(name, K, mu_tail):
    P = ds.config_problem(name)
    assert P.tree.K == K
    assert P.tree.nodes_per_stage[-1] == mu_tail
    assert P.tree.nodes_per_stage.sum() == K


def test_batch_tree_sizes():
    Ks = [ds.config_problem("batch64", i).tree.K for i in range(64)]
    assert set(Ks) <= {349, 669, 1277, 2429, 4605}
    assert len(set(Ks)) > 1


@pytest.mark.parametrize("name", ["small", "dwn128"])
def test_tree_structure(name):
    t = ds.config_problem(name).tree
    off = np.concatenate([[0], np.cumsum(t.nodes_per_stage)])
    assert t.anc[0] == -1
    for s in range(1, t.N):
        nodes = np.arange(off[s], off[s + 1])
        par = t.anc[nodes]
        # parents lie in the previous stage and are non-decreasing (contiguous children)
        assert par.min() >= off[s - 1] and par.max() < off[s]
        assert np.all(np.diff(par) >= 0)
    # probabilities: children sum to the parent, stage sums to one
    sums = np.zeros(t.K)
    np.add.at(sums, t.anc[1:], t.prob[1:])
    nonleaf = np.arange(off[t.N - 1])
    assert np.allclose(sums[nonleaf], t.prob[nonleaf], rtol=1e-13)
    for s in range(t.N):
        assert abs(t.prob[off[s]:off[s + 1]].sum() - 1.0) < 1e-12


def test_network_dimensions_and_rank():
    net = ds.config_problem("dwn128").net
    assert (net.nx, net.nu, net.nd, net.ns) == (63, 114, 88, 17)
    assert net.is_pump.sum() == 75
    assert np.linalg.matrix_rank(net.E) == 17
    # every tank has a source pump
    for t in range(net.nx):
        assert any(net.B[t, i] > 0 and k == "src_tank" for i, k in enumerate(net.kind))
    # mixing nodes have disjoint input sets
    assert np.all((net.E != 0).sum(axis=0) <= 1)


def test_steady_input_feasible():
    P = ds.config_problem("dwn128")
    net = P.net
    q = P.q
    assert np.all(q >= net.umin) and np.all(q <= net.umax)
    assert np.abs(net.E @ q + net.Ed @ P.data.demand[0]).max() < 1e-12
    assert np.abs(net.B @ q + net.Gd @ P.data.demand[0]).max() < 1e-12


def test_node_feasibility_every_node():
    """Every node's mass balance is feasible inside the input box."""
    for name in ["small", "dwn128"]:
        P = ds.config_problem(name)
        net = P.net
        row_dem = -(P.data.demand @ net.Ed.T)  # (K, ns)
        cap = (net.E > 0) @ net.umax
        assert np.all(row_dem >= 0) and np.all(row_dem <= cap[None, :])


def test_seeded_reproducible():
    a = ds.config_problem("dwn128")
    b = ds.config_problem("dwn128")
    assert np.array_equal(a.net.B, b.net.B)
    assert np.array_equal(a.data.demand, b.data.demand)
    assert np.array_equal(a.tree.prob, b.tree.prob)


def test_irregular_tree_leaves_last_stage():
    P = tiny_problem(N=5, irregular=True, seed=3)
    t = P.tree
    off = np.concatenate([[0], np.cumsum(t.nodes_per_stage)])
    has_child = np.zeros(t.K, bool)
    has_child[t.anc[1:]] = True
    assert np.all(has_child[:off[t.N - 1]])
    assert not np.any(has_child[off[t.N - 1]:])
