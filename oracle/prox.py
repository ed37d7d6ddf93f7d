"""Proximal operators of ``g`` and of its conjugate ``g*``.

TEST INFRASTRUCTURE (CPU oracle).

``g`` (Sec. 4.1, eq. g) is a separable sum over nodes of
``W_x dist(y1 | [xmin, xmax]) + W_s dist(y2 | [xs, inf)) + delta(y3 | U)``.
The prox of ``tau dist(. | C)`` follows the piecewise formula of Sec. 4.3
(prox of a distance function), with the prox parameter ``tau`` written in
its second branch condition and in the step, where the printed formula has
it only in the condition:

    prox(z) = z + tau (P_C z - z) / dist(z | C)   if dist(z | C) > tau
            = P_C z                               otherwise.

``prox_{gamma g*}`` follows from the Moreau decomposition (Sec. 4.2):
``prox_{gamma g*}(v) = v - gamma prox_{g/gamma}(v / gamma)``.
"""

from __future__ import annotations

import numpy as np


def proj_box(z: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Euclidean projection on ``{lo <= z <= hi}`` (elementwise clip)."""
    return np.minimum(np.maximum(z, lo), hi)


def proj_lower(z: np.ndarray, lo: np.ndarray) -> np.ndarray:
    """Projection on ``{z >= lo}``."""
    return np.maximum(z, lo)


def prox_dist(z: np.ndarray, tau: float, proj) -> np.ndarray:
    """Prox of ``tau * dist(. | C)`` applied to every row of ``z``;
    ``proj`` projects rows on ``C``."""
    pz = proj(z)
    d = np.linalg.norm(z - pz, axis=-1, keepdims=True)
    far = d > tau
    safe_d = np.where(far, d, 1.0)
    return np.where(far, z + tau * (pz - z) / safe_d, pz)


def prox_g(z: np.ndarray, lam: float, net, weights) -> np.ndarray:
    """``prox_{lam g}(z)`` for a dual-shaped array ``z`` (K, 2nx+nu)."""
    nx, nu = net.nx, net.nu
    out = np.empty_like(z)
    out[:, :nx] = prox_dist(z[:, :nx], lam * weights.W_x,
                            lambda v: proj_box(v, net.xmin, net.xmax))
    out[:, nx:2 * nx] = prox_dist(z[:, nx:2 * nx], lam * weights.W_s,
                                  lambda v: proj_lower(v, net.xs))
    out[:, 2 * nx:2 * nx + nu] = proj_box(z[:, 2 * nx:2 * nx + nu], net.umin, net.umax)
    return out


def prox_gconj(v: np.ndarray, gamma: float, net, weights):
    """``prox_{gamma g*}(v)`` by Moreau; also returns ``t = prox_{g/gamma}(v/gamma)``."""
    t = prox_g(v / gamma, 1.0 / gamma, net, weights)
    return v - gamma * t, t
