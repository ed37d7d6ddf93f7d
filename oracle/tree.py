"""Scenario-tree bookkeeping (paper Sec. 2.3: stages, children ``child(j,i)``,
ancestor ``anc(j,i)``, node probability ``p_j^i``).

Test infrastructure: part of the CPU oracle.
"""

from __future__ import annotations

import numpy as np


class TreeIndex:
    """Derived index structures of a breadth-first scenario tree.

    ``stage[n]`` is the stage of node n, ``nodes(s)`` the node ids of stage s,
    ``children[n]`` the child ids of node n, ``scenarios()`` the root-to-leaf
    paths (one per leaf).
    """

    def __init__(self, tree):
        self.N = int(tree.N)
        self.K = int(tree.K)
        self.anc = np.asarray(tree.anc, dtype=np.int64)
        self.prob = np.asarray(tree.prob, dtype=np.float64)
        mu = np.asarray(tree.nodes_per_stage, dtype=np.int64)
        self.mu = mu
        self.offset = np.concatenate([[0], np.cumsum(mu)])
        self.stage = np.repeat(np.arange(self.N), mu)
        self.children = [[] for _ in range(self.K)]
        for n in range(1, self.K):
            self.children[self.anc[n]].append(n)

    def nodes(self, s: int) -> np.ndarray:
        return np.arange(self.offset[s], self.offset[s + 1])

    def leaves(self) -> np.ndarray:
        return self.nodes(self.N - 1)

    def path(self, leaf: int) -> list:
        """Node ids from the root to ``leaf``."""
        out = [leaf]
        while self.anc[out[-1]] >= 0:
            out.append(int(self.anc[out[-1]]))
        return out[::-1]
