"""Dual gradient of the scenario-tree MPC: ``x_hat(w) = argmin_x f(x) + <w, Hx>``.

TEST INFRASTRUCTURE (CPU oracle).

The paper (Sec. 4.3, "Accelerated proximal algorithm on the dual", and
Sec. 4.4, "Implementation") computes ``grad f*(-H'w)`` by dynamic
programming over the tree, a Riccati-type recursion from the last stage to
stage 0 with all nodes of a stage independent; it defers the details to
other work.  This module states that recursion from the problem itself.

Problem (Sec. 4.1, eqs. f, Phi_1, Phi_2, H): with ``a_n = w1_n + w2_n`` and
``b_n = w3_n``,

    minimise  sum_n p_n [ c_n'u_n + (u_n - u_anc)'W_u(u_n - u_anc) ]
              + sum_n [ a_n'x_n + b_n'u_n ]
    s.t.      x_n = A x_anc + B u_n + Gd d_n,   E u_n + Ed d_n = 0,

with ``c_n = W_alpha (alpha0 + pi_n c_E)`` (Sec. 3.1, economic cost),
``x_anc(root) = p`` and ``u_anc(root) = q`` (problem SMPC, initial conditions).

Derivation used here.

1. ``x`` enters only linearly, so with the costate
   ``lambda_n = a_n + A' sum_{c in child(n)} lambda_c`` one has
   ``sum_n a_n'x_n = sum_n lambda_n'(B u_n + Gd d_n) + const``.
2. What remains is a tree DP in ``u`` with node cost
   ``p_n (u_n - u_anc)'W_u(u_n - u_anc) + e_n'u_n``, where
   ``e_n = p_n c_n + b_n + B'lambda_n``, over the affine set
   ``u_n in ubar_n + range(Z)`` (``Z`` a basis of ker E, ``ubar_n`` a
   particular solution of ``E u = -Ed d_n``).
3. Value functions ``V_n(v) = v'P_n v + 2 r_n'v + const`` of the parent's
   input give, per node,

       Q_n = p_n W_u + sum_c P_c,   M_n = Z'Q_n Z,   F_n = Z M_n^{-1} Z'
       K_n = p_n F_n W_u,           Gamma_n = I - F_n Q_n
       k_n = Gamma_n ubar_n - F_n (e_n / 2 + sum_c r_c)
       P_n = p_n W_u (I - K_n),     r_n = -p_n W_u k_n

   and the forward pass ``u_n = K_n u_anc + k_n``, then the dynamics.

:class:`NodeFactors` runs step 3 literally, node by node.
:class:`StageFactors` uses the fact that when the children's probabilities
add up to the parent's and ``W_u``, ``E`` do not depend on the node, every
factor scales with ``p_n`` (``F_n = Fbar_s / p_n``, ``K_n = Kbar_s``,
``P_n = p_n Pbar_s``); the two are checked against each other by a test, and
both against a dense KKT solve (:func:`dual_gradient_kkt`).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from .tree import TreeIndex


def null_basis(E: np.ndarray) -> np.ndarray:
    """Orthonormal basis ``Z`` of ker E (nu x m)."""
    return scipy.linalg.null_space(E)


def particular_inputs(net, demand: np.ndarray) -> np.ndarray:
    """``ubar_n`` with ``E ubar_n = -Ed d_n`` (minimum-norm solution), one row
    per node; eq. Phi_1 of Sec. 4.1."""
    rhs = -(demand @ net.Ed.T)  # (K, ns)
    sol, *_ = np.linalg.lstsq(net.E, rhs.T, rcond=None)
    return sol.T.copy()


def stage_linear_costs(problem) -> np.ndarray:
    """``c_n = W_alpha (alpha0 + pi_n c_E)`` for every node (Sec. 3.1, economic
    cost, with the price vector of node n equal to ``pi_n c_E``)."""
    w = problem.weights
    return w.W_alpha * (w.alpha0[None, :] + problem.data.price[:, None] * w.c_energy[None, :])


def costate(tidx: TreeIndex, net, a: np.ndarray) -> np.ndarray:
    """``lambda_n = a_n + A' sum_{c in child(n)} lambda_c`` from the leaves up."""
    lam = np.zeros_like(a)
    for s in range(tidx.N - 1, -1, -1):
        nodes = tidx.nodes(s)
        acc = np.zeros((tidx.K, a.shape[1]))
        if s + 1 < tidx.N:
            ch = tidx.nodes(s + 1)
            np.add.at(acc, tidx.anc[ch], lam[ch])
        lam[nodes] = a[nodes] + acc[nodes] @ net.A  # rows: (A' v)' = v' A
    return lam


class NodeFactors:
    """Per-node DP factors ``F_n, K_n, Gamma_n`` (step 3 above, node by node)."""

    def __init__(self, net, W_u: np.ndarray, tree):
        tidx = tree if isinstance(tree, TreeIndex) else TreeIndex(tree)
        self.tidx = tidx
        Z = null_basis(net.E)
        nu = net.nu
        K = tidx.K
        self.F = np.zeros((K, nu, nu))
        self.Kg = np.zeros((K, nu, nu))
        self.G = np.zeros((K, nu, nu))
        P = np.zeros((K, nu, nu))
        I = np.eye(nu)
        for s in range(tidx.N - 1, -1, -1):
            for n in tidx.nodes(s):
                pn = tidx.prob[n]
                Q = pn * W_u + sum((P[c] for c in tidx.children[n]), np.zeros((nu, nu)))
                M = Z.T @ Q @ Z
                F = Z @ np.linalg.solve(M, Z.T)
                Kn = pn * F @ W_u
                self.F[n] = F
                self.Kg[n] = Kn
                self.G[n] = I - F @ Q
                P[n] = pn * W_u @ (I - Kn)

    def mul(self, which: str, s: int, v: np.ndarray) -> np.ndarray:
        """``M_n v_n`` for the nodes of stage s (``which`` in F, K, G)."""
        nodes = self.tidx.nodes(s)
        M = {"F": self.F, "K": self.Kg, "G": self.G}[which][nodes]
        return np.einsum("nij,nj->ni", M, v)


class StageFactors:
    """Probability-scaled per-stage factors: ``F_n = Fbar_s / p_n``,
    ``K_n = Kbar_s``, ``Gamma_n = Gammabar_s``; recursion
    ``Pbar_N = 0``, ``Qbar_s = W_u + Pbar_{s+1}``, ``Fbar_s = Z (Z'Qbar_s Z)^{-1} Z'``,
    ``Kbar_s = Fbar_s W_u``, ``Gammabar_s = I - Fbar_s Qbar_s``,
    ``Pbar_s = W_u - W_u Fbar_s W_u``."""

    def __init__(self, net, W_u: np.ndarray, tree):
        tidx = tree if isinstance(tree, TreeIndex) else TreeIndex(tree)
        self.tidx = tidx
        Z = null_basis(net.E)
        nu = net.nu
        N = tidx.N
        I = np.eye(nu)
        self.Fbar = np.zeros((N, nu, nu))
        self.Kbar = np.zeros((N, nu, nu))
        self.Gbar = np.zeros((N, nu, nu))
        self.Pbar = np.zeros((N + 1, nu, nu))
        for s in range(N - 1, -1, -1):
            Q = W_u + self.Pbar[s + 1]
            F = Z @ np.linalg.solve(Z.T @ Q @ Z, Z.T)
            self.Fbar[s] = F
            self.Kbar[s] = F @ W_u
            self.Gbar[s] = I - F @ Q
            P = W_u - W_u @ F @ W_u
            self.Pbar[s] = 0.5 * (P + P.T)

    def mul(self, which: str, s: int, v: np.ndarray) -> np.ndarray:
        nodes = self.tidx.nodes(s)
        if which == "F":
            return (v @ self.Fbar[s].T) / self.tidx.prob[nodes][:, None]
        M = {"K": self.Kbar, "G": self.Gbar}[which][s]
        return v @ M.T


def split_dual(w: np.ndarray, nx: int, nu: int):
    """Blocks ``(w1, w2, w3)`` of a dual vector stored node by node as
    ``(y1 in R^nx, y2 in R^nx, y3 in R^nu)`` (operator H, Sec. 4.1)."""
    return w[:, :nx], w[:, nx:2 * nx], w[:, 2 * nx:2 * nx + nu]


def dual_gradient(problem, w: np.ndarray, factors, ubar: np.ndarray | None = None,
                  cost_lin: np.ndarray | None = None):
    """``(u_hat, x_hat) = argmin f + <w, H .>`` by the tree DP.

    ``w`` has shape (K, 2 nx + nu).  ``factors`` is a :class:`NodeFactors` or
    :class:`StageFactors` built for this network, ``W_u`` and tree.
    """
    net, wts, data = problem.net, problem.weights, problem.data
    tidx = factors.tidx
    nx, nu = net.nx, net.nu
    K, N = tidx.K, tidx.N
    prob = tidx.prob
    if ubar is None:
        ubar = particular_inputs(net, data.demand)
    if cost_lin is None:
        cost_lin = stage_linear_costs(problem)
    w1, w2, w3 = split_dual(w, nx, nu)
    lam = costate(tidx, net, w1 + w2)
    e = prob[:, None] * cost_lin + w3 + lam @ net.B  # B' lambda_n as a row

    k = np.zeros((K, nu))
    r = np.zeros((K, nu))
    for s in range(N - 1, -1, -1):
        nodes = tidx.nodes(s)
        rsum = np.zeros((K, nu))
        if s + 1 < N:
            ch = tidx.nodes(s + 1)
            np.add.at(rsum, tidx.anc[ch], r[ch])
        k[nodes] = factors.mul("G", s, ubar[nodes]) - factors.mul(
            "F", s, 0.5 * e[nodes] + rsum[nodes])
        r[nodes] = -prob[nodes][:, None] * (k[nodes] @ wts.W_u.T)

    u = np.zeros((K, nu))
    x = np.zeros((K, nx))
    gd = data.demand @ net.Gd.T
    for s in range(N):
        nodes = tidx.nodes(s)
        if s == 0:
            upar = problem.q[None, :].repeat(len(nodes), 0)
            xpar = problem.p[None, :].repeat(len(nodes), 0)
        else:
            upar = u[tidx.anc[nodes]]
            xpar = x[tidx.anc[nodes]]
        u[nodes] = factors.mul("K", s, upar) + k[nodes]
        x[nodes] = xpar @ net.A.T + u[nodes] @ net.B.T + gd[nodes]
    return u, x


def dual_gradient_kkt(problem, w: np.ndarray):
    """Same minimiser from one dense equality-constrained QP (tiny trees).

    Unknowns ``z = (u_0..u_{K-1}, x_0..x_{K-1})``; the KKT system
    ``[Q C'; C 0] [z; mu] = [-h; rhs]`` is solved with ``numpy.linalg.solve``.
    """
    net, wts, data, tree = problem.net, problem.weights, problem.data, problem.tree
    tidx = TreeIndex(tree)
    nx, nu, ns = net.nx, net.nu, net.ns
    K = tidx.K
    prob = tidx.prob
    nz = K * (nu + nx)

    def ui(n):
        return slice(n * nu, (n + 1) * nu)

    def xi(n):
        return slice(K * nu + n * nx, K * nu + (n + 1) * nx)

    w1, w2, w3 = split_dual(w, nx, nu)
    c = stage_linear_costs(problem)
    Q = np.zeros((nz, nz))
    h = np.zeros(nz)
    Wu = wts.W_u
    for n in range(K):
        pn = prob[n]
        a = tidx.anc[n]
        # p_n (u_n - u_a)' W_u (u_n - u_a): Hessian 2 p_n [W -W; -W W]
        Q[ui(n), ui(n)] += 2 * pn * Wu
        if a >= 0:
            Q[ui(a), ui(a)] += 2 * pn * Wu
            Q[ui(n), ui(a)] -= 2 * pn * Wu
            Q[ui(a), ui(n)] -= 2 * pn * Wu
        else:
            h[ui(n)] += -2 * pn * Wu @ problem.q
        h[ui(n)] += pn * c[n] + w3[n]
        h[xi(n)] += w1[n] + w2[n]

    rows = []
    rhs = []
    for n in range(K):
        a = tidx.anc[n]
        C = np.zeros((nx, nz))
        C[:, xi(n)] = np.eye(nx)
        C[:, ui(n)] = -net.B
        r = net.Gd @ data.demand[n]
        if a >= 0:
            C[:, xi(a)] = -net.A
        else:
            r = r + net.A @ problem.p
        rows.append(C)
        rhs.append(r)
        Cm = np.zeros((ns, nz))
        Cm[:, ui(n)] = net.E
        rows.append(Cm)
        rhs.append(-net.Ed @ data.demand[n])
    C = np.vstack(rows)
    rhs = np.concatenate(rhs)
    nc = C.shape[0]
    KKT = np.zeros((nz + nc, nz + nc))
    KKT[:nz, :nz] = Q
    KKT[:nz, nz:] = C.T
    KKT[nz:, :nz] = C
    sol = np.linalg.solve(KKT, np.concatenate([-h, rhs]))
    z = sol[:nz]
    u = z[:K * nu].reshape(K, nu)
    x = z[K * nu:].reshape(K, nx)
    return u, x
