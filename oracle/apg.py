"""Accelerated proximal gradient on the Fenchel dual (paper Sec. 4.3).

TEST INFRASTRUCTURE (CPU oracle).

Iteration (eqs. apg:1, apg:2, read with ``y^{nu+1}`` on the left of the
second equation):

    w^nu     = y^nu + beta_nu (y^nu - y^{nu-1})
    y^{nu+1} = prox_{gamma g*}( w^nu + gamma H x_hat(w^nu) )

with ``y^0 = y^{-1} = 0`` (or a warm start for both), and
``beta_nu = theta_nu (1/theta_{nu-1} - 1)``, ``theta_0 = theta_{-1} = 1``,
``theta_{nu+1} = (sqrt(theta_nu^4 + 4 theta_nu^2) - theta_nu^2) / 2``.

Termination: the split residual ``r = H x_hat(w^nu) - t`` where
``t = prox_{g/gamma}(v/gamma)``, equal to ``(y^{nu+1} - w^nu)/gamma``; the
run stops after the first iteration whose ``max |r|`` is at most ``tol``.
The returned primal is ``x_hat(w^{nu*})`` of that last iteration.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .dual_gradient import dual_gradient, particular_inputs, stage_linear_costs
from .prox import prox_gconj


def theta_next(theta: float) -> float:
    """``theta_{nu+1} = (sqrt(theta^4 + 4 theta^2) - theta^2) / 2``."""
    t2 = theta * theta
    return 0.5 * (np.sqrt(t2 * t2 + 4.0 * t2) - t2)


def beta_sequence(n: int) -> np.ndarray:
    """``beta_0 .. beta_{n-1}`` of the theta recursion."""
    out = np.zeros(n)
    th_prev, th = 1.0, 1.0
    for i in range(n):
        out[i] = th * (1.0 / th_prev - 1.0)
        th_prev, th = th, theta_next(th)
    return out


@dataclass
class APGResult:
    u: np.ndarray
    x: np.ndarray
    y: np.ndarray
    y_prev: np.ndarray
    iters: int
    res: float
    converged: bool
    res_hist: list = field(default_factory=list)
    t: np.ndarray | None = None


def hx_blocks(u: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``H(x, u) = (x, x, u)`` node by node (Sec. 4.1, eq. H)."""
    return np.concatenate([x, x, u], axis=1)


def apg(problem, gamma: float, factors, max_iter: int, tol: float | None = None,
        beta_rule: str = "paper", y0: np.ndarray | None = None,
        callback=None) -> APGResult:
    """Run the dual APG.  ``beta_rule='zero'`` gives the plain dual proximal
    gradient (every ``beta = 0``).  ``callback(nu, y_new, w, u, x)`` is called
    after every iteration (tests use it to follow the dual objective)."""
    net, wts = problem.net, problem.weights
    K = problem.tree.K
    m = 2 * net.nx + net.nu
    ubar = particular_inputs(net, problem.data.demand)
    clin = stage_linear_costs(problem)
    y = np.zeros((K, m)) if y0 is None else np.array(y0, dtype=np.float64)
    y_prev = y.copy()
    th_prev, th = 1.0, 1.0
    hist = []
    u = x = t = None
    res = np.inf
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        beta = th * (1.0 / th_prev - 1.0) if beta_rule == "paper" else 0.0
        w = y + beta * (y - y_prev)
        u, x = dual_gradient(problem, w, factors, ubar=ubar, cost_lin=clin)
        hx = hx_blocks(u, x)
        y_new, t = prox_gconj(w + gamma * hx, gamma, net, wts)
        res = float(np.max(np.abs(hx - t))) if hx.size else 0.0
        hist.append(res)
        if callback is not None:
            callback(it - 1, y_new, w, u, x)
        y_prev, y = y, y_new
        th_prev, th = th, theta_next(th)
        if tol is not None and res <= tol:
            converged = True
            break
    return APGResult(u=u, x=x, y=y, y_prev=y_prev, iters=it, res=res,
                     converged=converged, res_hist=hist, t=t)
