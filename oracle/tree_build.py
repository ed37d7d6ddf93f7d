"""Scenario-tree construction from sampled error paths by forward selection.

TEST INFRASTRUCTURE (CPU oracle).

The paper builds its trees from sampled prediction-error paths with the
scenario reduction of Heitsch and Roemisch (Sec. 2.3, Sec. 6.2: 10^4
Monte-Carlo scenarios reduced to a tree).  Reading used here (stage by stage,
the forward construction):

* stage 0: one root holding every sample path (the error at stage 0 is
  zero: observed demand and price);
* stage t >= 1: every node v of stage t-1 holds a cluster C_v of sample
  paths; forward selection picks n_v = min(b_t, |C_v|) representatives of
  C_v by their stage-t values, each member of C_v joins its nearest
  representative (ties: the one selected first), and every representative
  becomes a child of v, in the order selected, whose value is the
  representative's stage-t value and whose probability is the summed
  probability of its members;
* forward selection on a set with probabilities p_k and costs
  c(k, u) = |x_k - x_u|_2: with D_k = +inf initially, repeat n times:
  u = argmin over unselected u of sum_k p_k min(D_k, c(k, u)) (ties: the
  lowest index in the set's order), then D_k = min(D_k, c(k, u)).  The sum
  is the transport (Kantorovich) cost of moving every member to its nearest
  selected point.

Returns the tree in breadth-first order with contiguous children.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def distances(x: np.ndarray) -> np.ndarray:
    """Euclidean distances between the rows of x (one row at a time)."""
    m = x.shape[0]
    C = np.empty((m, m))
    for i in range(m):
        e = x - x[i]
        C[i] = np.sqrt(np.sum(e * e, axis=1))
    return C


def forward_selection(x: np.ndarray, p: np.ndarray, n: int):
    """Indices (into the rows of x) of the n points picked, in order, and the
    transport cost after each pick."""
    m = x.shape[0]
    C = distances(x)
    D = np.full(m, np.inf)
    chosen, costs = [], []
    for _ in range(min(n, m)):
        total = np.sum(p[:, None] * np.minimum(D[:, None], C), axis=0)
        total[chosen] = np.inf
        u = int(np.argmin(total))
        chosen.append(u)
        costs.append(float(total[u]))
        D = np.minimum(D, C[:, u])
    return chosen, costs


def nearest(x: np.ndarray, reps: list) -> np.ndarray:
    """For every row of x, the position in reps of its nearest representative
    (ties: the earlier one)."""
    C = distances(x)[:, reps]
    return np.argmin(C, axis=1)


@dataclass
class BuiltTree:
    nodes_per_stage: np.ndarray
    anc: np.ndarray
    prob: np.ndarray
    value: np.ndarray      # (K, d) the node's error value
    rep: np.ndarray        # (K,) the sample path whose value the node carries
    members: list          # per node, the sample paths it holds


def build_tree(samples: np.ndarray, prob: np.ndarray, branching) -> BuiltTree:
    """samples (M, H, d), prob (M,), branching[t] = children per node at
    stage t for t = 1..H-1 (branching[0] is ignored: one root)."""
    M, H, d = samples.shape
    anc, pr, val, rep, mem = [-1], [float(np.sum(prob))], [samples[0, 0].copy()], [0], \
        [np.arange(M)]
    mu = [1]
    first = 0
    for t in range(1, H):
        for v in range(first, first + mu[-1]):
            cl = mem[v]
            x = samples[cl, t, :]
            chosen, _ = forward_selection(x, prob[cl], int(branching[t]))
            who = nearest(x, chosen)
            for j, u in enumerate(chosen):
                sel = cl[who == j]
                anc.append(v)
                pr.append(float(np.sum(prob[sel])))
                val.append(samples[cl[u], t].copy())
                rep.append(int(cl[u]))
                mem.append(sel)
        first += mu[-1]
        mu.append(len(anc) - first)
    return BuiltTree(nodes_per_stage=np.asarray(mu), anc=np.asarray(anc), prob=np.asarray(pr),
                     value=np.asarray(val), rep=np.asarray(rep), members=mem)
