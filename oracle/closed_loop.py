"""Closed-loop receding-horizon simulation (paper Sec. 6.3).

TEST INFRASTRUCTURE (CPU oracle).

At every sampling instant k = 0..H_s-1: the scenario tree's node data at k
(root = the observed demand and price), one solve of the stochastic MPC
problem from the plant state x_k and the previous input (the dual APG of
:mod:`oracle.apg`, warm started from the previous dual), the root input u_k
applied, and the plant moved with the observed demand d_k:

    x_{k+1} = A x_k + B u_k + Gd d_k.

Performance indices (Sec. 6.3): KPI_E = (1/H_s) sum_k (alpha0 + alpha_k)'u_k
with alpha_k = pi_k c_E, KPI_S = sum_k |max(xs - x_{k+1}, 0)|_1 (KPI_tau, the
worst solve time, is a measurement and has no oracle).
"""

from __future__ import annotations

import copy
from dataclasses import dataclass

import numpy as np

from .apg import apg


@dataclass
class LoopResult:
    x: np.ndarray        # (H_s + 1, nx)
    u: np.ndarray        # (H_s, nu)
    iters: np.ndarray    # (H_s,)
    kpi_E: float
    kpi_S: float
    root_states: np.ndarray  # (H_s, nx): x_hat at the root of each solve


def closed_loop(problem, inputs, H_s: int, gamma: float, factors, max_iter: int,
                tol: float | None = None, warm_start: bool = True) -> LoopResult:
    """``inputs.tree_data(net, tree, k) -> (demand, price)`` gives the tree's
    data at instant k (see :mod:`dwn_synth.closed_loop`)."""
    net, w = problem.net, problem.weights
    x = np.array(problem.p, dtype=np.float64)
    q = np.array(problem.q, dtype=np.float64)
    y = None
    xs, us, its, roots = [x.copy()], [], [], []
    kE = kS = 0.0
    for k in range(H_s):
        d, pr = inputs.tree_data(net, problem.tree, k)
        Pk = copy.copy(problem)
        Pk.data = copy.copy(problem.data)
        Pk.data.demand, Pk.data.price = d, pr
        Pk.p, Pk.q = x, q
        r = apg(Pk, gamma, factors, max_iter, tol=tol,
                y0=y if (warm_start and y is not None) else None)
        u = r.u[0].copy()
        x_next = net.A @ x + net.B @ u + net.Gd @ d[0]
        kE += float((w.alpha0 + pr[0] * w.c_energy) @ u) / H_s
        kS += float(np.sum(np.maximum(net.xs - x_next, 0.0)))
        xs.append(x_next)
        us.append(u)
        its.append(r.iters)
        roots.append(r.x[0].copy())
        x, q, y = x_next, u, r.y
    return LoopResult(x=np.asarray(xs), u=np.asarray(us), iters=np.asarray(its), kpi_E=kE,
                      kpi_S=kS, root_states=np.asarray(roots))
