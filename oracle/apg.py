"""Accelerated proximal gradient on the Fenchel dual (paper Sec. 4.3).

TEST INFRASTRUCTURE (CPU oracle).

Iteration (eqs. apg:1, apg:2, read with ``y^{nu+1}`` on the left of the
second equation):

    w^nu     = y^nu + beta_nu (y^nu - y^{nu-1})
    y^{nu+1} = prox_{gamma g*}( w^nu + gamma H x_hat(w^nu) )

with ``y^0 = y^{-1} = 0`` (or a warm start for both), and
``beta_nu = theta_nu (1/theta_{nu-1} - 1)``, ``theta_0 = theta_{-1} = 1``,
``theta_{nu+1} = (sqrt(theta_nu^4 + 4 theta_nu^2) - theta_nu^2) / 2``.

Other choices the paper names (Sec. 4.3): ``theta_nu = 2/(nu+2)`` for
``nu >= 1`` (``beta_rule='simple'``), and ``beta = 0`` throughout, the plain
dual proximal gradient (``beta_rule='zero'``).

Averaged primal (Sec. 4.3, which cites the averaged iterate of accelerated
dual gradient projection for its ``O(1/nu^2)`` primal rate):
``xbar^nu = (1 - theta_nu) xbar^{nu-1} + theta_nu x_hat(w^nu)`` with the
iteration's own ``theta_nu`` (``theta_0 = 1``, so ``xbar^0 = x_hat(w^0)``); for
``beta_rule='zero'`` the weights are ``theta_nu = 1/(nu+1)``, the running mean.

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


def theta_of(rule: str, nu: int, theta: float) -> float:
    """``theta_{nu}`` from ``theta_{nu-1} = theta`` under the given rule."""
    if rule == "paper":
        return theta_next(theta)
    if rule == "simple":
        return 2.0 / (nu + 2.0)
    if rule == "zero":
        return 1.0 / (nu + 1.0)
    raise ValueError(rule)


def beta_sequence(n: int, rule: str = "paper") -> np.ndarray:
    """``beta_0 .. beta_{n-1}`` (``theta_0 = theta_{-1} = 1``)."""
    out = np.zeros(n)
    th_prev, th = 1.0, 1.0
    for i in range(n):
        out[i] = 0.0 if rule == "zero" else th * (1.0 / th_prev - 1.0)
        th_prev, th = th, theta_of(rule, i + 1, th)
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
    u_avg: np.ndarray | None = None
    x_avg: np.ndarray | None = None


def hx_blocks(u: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``H(x, u) = (x, x, u)`` node by node (Sec. 4.1, eq. H)."""
    return np.concatenate([x, x, u], axis=1)


def apg(problem, gamma: float, factors, max_iter: int, tol: float | None = None,
        beta_rule: str = "paper", y0: np.ndarray | None = None,
        callback=None, average: bool = False) -> APGResult:
    """Run the dual APG.  ``beta_rule`` is ``'paper'`` (the theta recursion),
    ``'simple'`` (``theta_nu = 2/(nu+2)``) or ``'zero'`` (every ``beta = 0``,
    the plain dual proximal gradient).  ``average=True`` also returns the
    averaged primal.  ``callback(nu, y_new, w, u, x)`` is called after every
    iteration (tests use it to follow the dual objective); a true return value
    stops the run there (counted as converged)."""
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
    ua = xa = None
    res = np.inf
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        beta = 0.0 if beta_rule == "zero" else th * (1.0 / th_prev - 1.0)
        w = y + beta * (y - y_prev)
        u, x = dual_gradient(problem, w, factors, ubar=ubar, cost_lin=clin)
        if average:
            if ua is None:  # theta_0 = 1
                ua, xa = u.copy(), x.copy()
            else:
                ua = (1.0 - th) * ua + th * u
                xa = (1.0 - th) * xa + th * x
        hx = hx_blocks(u, x)
        y_new, t = prox_gconj(w + gamma * hx, gamma, net, wts)
        res = float(np.max(np.abs(hx - t))) if hx.size else 0.0
        hist.append(res)
        stop = callback(it - 1, y_new, w, u, x) if callback is not None else False
        y_prev, y = y, y_new
        th_prev, th = th, theta_of(beta_rule, it, th)
        if (tol is not None and res <= tol) or stop:
            converged = True
            break
    return APGResult(u=u, x=x, y=y, y_prev=y_prev, iters=it, res=res,
                     converged=converged, res_hist=hist, t=t, u_avg=ua, x_avg=xa)
