"""GPU: scenario-tree construction from sampled error paths (tapg_tree_build)
against the oracle's forward-selection tree on the same seeded paths: the
tree's structure, representatives and values exactly, probabilities to
rounding; a tree built from 10^4 paths (the paper's sample size) feeds a
solve that matches the oracle."""

import os
import sys
import time

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O
from dwn_synth.problem import NodeData, Problem, ScenarioTree
from paper_1904_10548_amd import tapg

from gpu_helpers import add_tree, make_solver

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("M,H,nd,branching,uniform", [
    (600, 8, 88, [1, 4, 2, 2, 2, 2, 1, 1], True),
    (300, 6, 3, [1, 3, 3, 2, 1, 1], False),
    (40, 4, 2, [1, 40, 40, 40], True),
])
def test_tree_build_matches_oracle(M, H, nd, branching, uniform):
    """Every pick and every assignment is an argmin of FP64 sums that the two
    sides add in different orders; on these seeded paths the closest pair of
    distinct candidates differs by 2e-5 (relative), far above either order's
    rounding, and exactly equal totals (two-path clusters with equal
    probabilities) go to the lower position on both sides, so the structure
    must agree exactly."""
    paths = ds.make_error_paths(M, H, nd, seed=M + H)
    if uniform:
        prob = np.full(M, 1.0 / M)
    else:
        w = np.random.default_rng(1).uniform(0.5, 1.5, M)
        prob = w / w.sum()
    say("tree build", M, H, nd + 1, branching)
    g = tapg.tapg_tree_build(paths, branching, prob=None if uniform else prob)
    ref = O.build_tree(paths, prob, branching)
    assert np.array_equal(g["nodes_per_stage"], ref.nodes_per_stage)
    assert np.array_equal(g["anc"], ref.anc)
    assert np.array_equal(g["rep"], ref.rep)
    assert np.array_equal(g["value"], ref.value)
    assert np.allclose(g["prob"], ref.prob, rtol=1e-13, atol=1e-16)


def test_tree_from_ten_thousand_paths_feeds_a_solve():
    """10^4 error paths reduced to the 128-scenario shape of the benchmark
    tree (4, then 2 up to 128, H = 24): the result is a valid tree (every
    node's children's probabilities add up to its own), and a solve on it
    matches the oracle element by element."""
    base = ds.config_problem("dwn128")
    net = base.net
    M, H = 10000, 24
    br = [1, 4] + [2] * 5 + [1] * 17
    paths = ds.make_error_paths(M, H, net.nd, seed=2024)
    t0 = time.perf_counter()
    g = tapg.tapg_tree_build(paths, br)
    dt = time.perf_counter() - t0
    mu, anc, pr = g["nodes_per_stage"], g["anc"], g["prob"]
    K = int(mu.sum())
    say("tree from 10^4 paths", K, "nodes in", round(dt, 3), "s")
    assert list(mu) == [1, 4, 8, 16, 32, 64] + [128] * 18 and K == 2429
    sums = np.zeros(K)
    np.add.at(sums, anc[1:], pr[1:])
    inner = np.arange(K - 128)
    assert np.allclose(sums[inner], pr[inner], rtol=1e-12)
    # node data: the benchmark tree's forecast at each stage times the errors
    stage = np.repeat(np.arange(H), mu)
    fd = np.zeros((H, net.nd))
    fp = np.zeros(H)
    bst = np.repeat(np.arange(H), base.tree.nodes_per_stage)
    for s in range(H):
        fd[s] = base.data.demand[bst == s].mean(axis=0)
        fp[s] = base.data.price[bst == s].mean()
    demand = fd[stage] * np.exp(g["value"][:, :net.nd])
    price = fp[stage] * (1.0 + g["value"][:, net.nd])
    tree = ScenarioTree(N=H, nodes_per_stage=mu.astype(np.int64), anc=anc.astype(np.int64),
                        prob=pr / pr[0])
    P = Problem(net=net, tree=tree, data=NodeData(demand=demand, price=price),
                weights=base.weights, p=base.p, q=base.q, name="dwn-built")
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, sf, 60))
    iters = 30
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=iters) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
    ref = O.apg(P, gamma, sf, iters)
    assert np.abs(u - ref.u).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())
    J = O.primal_cost(P, ref.u, ref.x)
    assert abs(res.cost - J) <= 1e-6 * max(1.0, abs(J))
