"""Lipschitz constant of the dual gradient (step size ``gamma = 1/L``).

TEST INFRASTRUCTURE (CPU oracle).

The smooth part of the dual, ``y -> f*(-H'y)``, has gradient
``-H x_hat(y)`` (Sec. 4.2, eq. dual-gradient), which is affine in ``y``.
Its linear part ``y -> -H x_hat_0(y)`` (``x_hat_0``: the dual gradient of the
same tree with all data, prices and initial conditions set to zero) is a
symmetric positive semidefinite operator; ``L`` is its largest eigenvalue.
The paper does not state its step size; ``gamma = 1/L`` is the standard
choice for the accelerated method.
"""

from __future__ import annotations

import copy

import numpy as np

from .dual_gradient import dual_gradient


def _zero_data(problem):
    z = copy.copy(problem)
    z.data = copy.copy(problem.data)
    z.weights = copy.copy(problem.weights)
    z.data.demand = np.zeros_like(problem.data.demand)
    z.data.price = np.zeros_like(problem.data.price)
    z.weights.alpha0 = np.zeros_like(problem.weights.alpha0)
    z.p = np.zeros_like(problem.p)
    z.q = np.zeros_like(problem.q)
    return z


def dual_operator(problem, factors):
    """``v -> -H x_hat_0(v)`` as a function on (K, 2nx+nu) arrays."""
    z = _zero_data(problem)

    def op(v):
        u, x = dual_gradient(z, v, factors)
        return -np.concatenate([x, x, u], axis=1)

    return op


def dual_hessian_dense(problem, factors) -> np.ndarray:
    """The operator as a dense matrix, one column per unit vector (tiny trees)."""
    K = problem.tree.K
    m = 2 * problem.net.nx + problem.net.nu
    op = dual_operator(problem, factors)
    M = np.zeros((K * m, K * m))
    for j in range(K * m):
        e = np.zeros(K * m)
        e[j] = 1.0
        M[:, j] = op(e.reshape(K, m)).ravel()
    return M


def lipschitz_dense(problem, factors) -> float:
    M = dual_hessian_dense(problem, factors)
    return float(np.linalg.eigvalsh(0.5 * (M + M.T)).max())


def lipschitz_power(problem, factors, iters: int = 200, seed: int = 0) -> float:
    """Power iteration from a seeded random start; returns ``|M v| / |v|`` of
    the last iterate (a lower bound that converges to ``L``)."""
    K = problem.tree.K
    m = 2 * problem.net.nx + problem.net.nu
    op = dual_operator(problem, factors)
    v = np.random.default_rng(seed).standard_normal((K, m))
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        mv = op(v)
        lam = float(np.linalg.norm(mv))
        if lam == 0.0:
            return 0.0
        v = mv / lam
    return lam
