"""Plain data containers for one stochastic MPC instance.

No solver arithmetic lives here: only arrays and their shapes.  Every matrix
is a dense, row-major float64 numpy array.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Network:
    """Linear tank dynamics and mass balance of a flow-based network.

    ``x+ = A x + B u + Gd d`` with ``x`` the tank volumes (nx), ``u`` the
    pump/valve flows (nu) and ``d`` the demands (nd); the mixing nodes give
    ``E u + Ed d = 0`` (ns rows).  ``is_pump`` marks inputs whose flow costs
    electricity (pumps); the other inputs are valves.
    """

    A: np.ndarray
    B: np.ndarray
    Gd: np.ndarray
    E: np.ndarray
    Ed: np.ndarray
    xmin: np.ndarray
    xmax: np.ndarray
    xs: np.ndarray
    umin: np.ndarray
    umax: np.ndarray
    is_pump: np.ndarray
    # generator metadata: per input one of src_tank, tank_row, src_row, tank_tank
    kind: tuple = ()

    @property
    def nx(self) -> int:
        return self.A.shape[0]

    @property
    def nu(self) -> int:
        return self.B.shape[1]

    @property
    def nd(self) -> int:
        return self.Gd.shape[1]

    @property
    def ns(self) -> int:
        return self.E.shape[0]


@dataclass
class ScenarioTree:
    """Scenario tree over the decision stages ``0..N-1``.

    Nodes are numbered breadth-first: all nodes of stage ``j`` come before
    those of stage ``j+1`` and the children of a node are contiguous and in
    the order of their parents.  ``anc[0] = -1`` (root).  ``prob[n]`` is the
    probability of reaching node ``n`` from the root.
    """

    N: int
    nodes_per_stage: np.ndarray  # (N,) int64
    anc: np.ndarray  # (K,) int64
    prob: np.ndarray  # (K,) float64

    @property
    def K(self) -> int:
        return int(self.anc.shape[0])

    @property
    def n_scenarios(self) -> int:
        return int(self.nodes_per_stage[-1])


@dataclass
class NodeData:
    """Uncertain quantities carried by every node: demand ``d_n`` (nd) and
    the scalar electricity price ``pi_n``."""

    demand: np.ndarray  # (K, nd)
    price: np.ndarray  # (K,)


@dataclass
class Weights:
    """Tuning weights of the stage cost and the soft penalties.

    The economic cost of node ``n`` is ``W_alpha (alpha0 + price_n *
    c_energy)' u_n``; the smoothing cost is ``du' W_u du``; the soft
    penalties are ``W_x dist(x | [xmin, xmax])`` and ``W_s dist(x | [xs, inf))``.
    """

    W_alpha: float
    W_u: np.ndarray  # (nu, nu) SPD
    W_s: float
    W_x: float
    alpha0: np.ndarray  # (nu,)
    c_energy: np.ndarray  # (nu,)


@dataclass
class Problem:
    """One stochastic MPC instance: network, tree, node data, weights and
    the initial condition ``x_{k|k} = p``, ``u_{k-1|k} = q``."""

    net: Network
    tree: ScenarioTree
    data: NodeData
    weights: Weights
    p: np.ndarray  # (nx,)
    q: np.ndarray  # (nu,)
    name: str = ""
    meta: dict = field(default_factory=dict)
