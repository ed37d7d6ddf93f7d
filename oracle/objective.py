"""Primal cost, constraint violations and the dual objective.

TEST INFRASTRUCTURE (CPU oracle).

* Primal cost (problem SMPC, Sec. 3.2): the expected stage cost
  ``sum_n p_n [W_alpha (alpha0 + alpha_n)'u_n + du_n' W_u du_n]`` plus the
  unweighted soft penalties ``V_s = sum_n W_x dist(x_n | [xmin, xmax]) +
  W_s dist(x_n | [xs, inf))`` with Euclidean norms.  The hard input box is
  not part of the cost; its violation is reported separately.
* Duality gap of a dual point (``split_gap``) from the two objectives.
* Dual objective (Sec. 4.2, problem D): ``F(y) = f*(-H'y) + g*(y)`` with
  ``f*(-H'y) = -[f(x_hat(y)) + <y, H x_hat(y)>]`` and
  ``g*(y) = sum_n sigma_X(y1_n) + xs'y2_n + sigma_U(y3_n)`` on its domain
  ``|y1_n| <= W_x``, ``|y2_n| <= W_s``, ``y2_n <= 0``.
"""

from __future__ import annotations

import numpy as np

from .dual_gradient import dual_gradient, stage_linear_costs
from .prox import proj_box, proj_lower
from .tree import TreeIndex


def _parents(problem, u, x):
    anc = np.asarray(problem.tree.anc)
    upar = np.where(anc[:, None] >= 0, u[np.maximum(anc, 0)], problem.q[None, :])
    xpar = np.where(anc[:, None] >= 0, x[np.maximum(anc, 0)], problem.p[None, :])
    return upar, xpar


def smooth_cost(problem, u: np.ndarray) -> float:
    """``f`` without its indicators: ``sum_n p_n (c_n'u_n + du_n'W_u du_n)``."""
    prob = np.asarray(problem.tree.prob)
    upar, _ = _parents(problem, u, np.zeros((u.shape[0], problem.net.nx)))
    du = u - upar
    c = stage_linear_costs(problem)
    quad = np.einsum("ni,ij,nj->n", du, problem.weights.W_u, du)
    return float(np.sum(prob * (np.sum(c * u, axis=1) + quad)))


def soft_penalty(problem, x: np.ndarray) -> float:
    """``V_s``: unweighted sum over nodes of the two distance penalties."""
    net, w = problem.net, problem.weights
    d1 = np.linalg.norm(x - proj_box(x, net.xmin, net.xmax), axis=1)
    d2 = np.linalg.norm(x - proj_lower(x, net.xs), axis=1)
    return float(np.sum(w.W_x * d1 + w.W_s * d2))


def primal_cost(problem, u: np.ndarray, x: np.ndarray) -> float:
    return smooth_cost(problem, u) + soft_penalty(problem, x)


def violations(problem, u: np.ndarray, x: np.ndarray):
    """``(viol_box, viol_eq)``: max distance of any ``u_n`` to the input box
    (inf-norm), and the max of the mass-balance and dynamics residuals."""
    net, d = problem.net, problem.data.demand
    vbox = float(np.max(np.maximum(np.maximum(net.umin - u, u - net.umax), 0.0)))
    mass = np.max(np.abs(u @ net.E.T + d @ net.Ed.T))
    upar, xpar = _parents(problem, u, x)
    dyn = np.max(np.abs(x - xpar @ net.A.T - u @ net.B.T - d @ net.Gd.T))
    return vbox, float(max(mass, dyn))


def split_residual(hx: np.ndarray, t: np.ndarray) -> float:
    return float(np.max(np.abs(hx - t)))


def _support_box(y, lo, hi):
    return np.sum(np.maximum(y * hi, y * lo), axis=-1)


def g_conj(problem, y: np.ndarray, slack: float = 1e-9) -> float:
    """``g*(y)``; ``+inf`` outside its domain (checked with a relative slack)."""
    net, w = problem.net, problem.weights
    nx, nu = net.nx, net.nu
    y1, y2, y3 = y[:, :nx], y[:, nx:2 * nx], y[:, 2 * nx:2 * nx + nu]
    if np.any(np.linalg.norm(y1, axis=1) > w.W_x * (1 + slack)):
        return np.inf
    if np.any(np.linalg.norm(y2, axis=1) > w.W_s * (1 + slack)) or np.any(y2 > slack * w.W_s):
        return np.inf
    val = _support_box(y1, net.xmin, net.xmax).sum()
    val += float(np.sum(y2 @ net.xs))
    val += _support_box(y3, net.umin, net.umax).sum()
    return float(val)


def g_value(problem, z: np.ndarray, slack: float = 1e-9) -> float:
    """``g(z)`` of the split form (Sec. 4.1, eq. g): per node
    ``W_x dist(z1|[xmin,xmax]) + W_s dist(z2|[xs,inf))`` plus the indicator
    of ``z3`` in the input box (``+inf`` outside it, with a relative slack)."""
    net, w = problem.net, problem.weights
    nx, nu = net.nx, net.nu
    z1, z2, z3 = z[:, :nx], z[:, nx:2 * nx], z[:, 2 * nx:2 * nx + nu]
    span = np.maximum(1.0, np.abs(net.umax - net.umin))
    if np.any(z3 < net.umin - slack * span) or np.any(z3 > net.umax + slack * span):
        return np.inf
    d1 = np.linalg.norm(z1 - proj_box(z1, net.xmin, net.xmax), axis=1)
    d2 = np.linalg.norm(z2 - proj_lower(z2, net.xs), axis=1)
    return float(np.sum(w.W_x * d1 + w.W_s * d2))


def split_gap(problem, y: np.ndarray, gamma: float, factors):
    """Duality gap of a dual point ``y`` at the primal pair ``y`` determines
    (Sec. 4.2, Fenchel dual and strong duality): with ``x' = x_hat(y)`` and
    ``t = prox_{g/gamma}(y/gamma + H x')`` (the split variable of one more
    proximal-gradient step from ``y``),

        G(y) = f(x') + g(t) + F(y),   F(y) = f*(-H'y) + g*(y).

    Weak duality and Fenchel-Young give ``G(y) >= <y, t - H x'>``, and ``G = 0``
    at a dual optimum.  Returns ``(G, F)``."""
    from .prox import prox_gconj

    u, x = dual_gradient(problem, y, factors)
    hx = np.concatenate([x, x, u], axis=1)
    _, t = prox_gconj(y + gamma * hx, gamma, problem.net, problem.weights)
    F = dual_objective(problem, y, factors)
    return smooth_cost(problem, u) + g_value(problem, t) + F, F


def dual_objective(problem, y: np.ndarray, factors) -> float:
    """``F(y) = f*(-H'y) + g*(y)`` (to be minimised)."""
    u, x = dual_gradient(problem, y, factors)
    hx = np.concatenate([x, x, u], axis=1)
    fstar = -(smooth_cost(problem, u) + float(np.sum(y * hx)))
    return fstar + g_conj(problem, y)


def scenario_sum_cost(problem, u: np.ndarray) -> float:
    """Brute-force ``E[V]``: the sum over scenarios (root-to-leaf paths) of the
    leaf probability times the path's stage costs."""
    tidx = TreeIndex(problem.tree)
    c = stage_linear_costs(problem)
    W = problem.weights.W_u
    total = 0.0
    for leaf in tidx.leaves():
        path = tidx.path(int(leaf))
        prev = problem.q
        acc = 0.0
        for n in path:
            du = u[n] - prev
            acc += float(c[n] @ u[n] + du @ W @ du)
            prev = u[n]
        total += tidx.prob[leaf] * acc
    return total
