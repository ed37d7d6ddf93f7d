"""Seeded sample paths of prediction errors for scenario-tree construction
(Sec. 2.3: the errors of the demand and price forecasts, zero at stage 0;
Sec. 6.2: Monte-Carlo paths of a fitted time-series model).

Only input generation.  Each path has, per stage, nd log-errors of the
demands and one relative error of the price, each an AR(1) process started at
zero: e_t = rho e_{t-1} + s sqrt(1 - rho^2) eta_t (rho 0.8, s 0.1 for the
demands; rho 0.7, s 0.2 for the price), so that errors persist across stages
as the paper's scenario trees assume.  A node with error e carries the demand
forecast times exp(e_d) and the price forecast times (1 + e_p).
"""

from __future__ import annotations

import numpy as np


def make_error_paths(M: int, H: int, nd: int, seed: int, rho_d: float = 0.8, s_d: float = 0.1,
                     rho_p: float = 0.7, s_p: float = 0.2) -> np.ndarray:
    """(M, H, nd + 1) error paths; stage 0 is zero."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 200]))
    out = np.zeros((M, H, nd + 1))
    for t in range(1, H):
        eta = rng.standard_normal((M, nd + 1))
        out[:, t, :nd] = rho_d * out[:, t - 1, :nd] + s_d * np.sqrt(1 - rho_d ** 2) * eta[:, :nd]
        out[:, t, nd] = rho_p * out[:, t - 1, nd] + s_p * np.sqrt(1 - rho_p ** 2) * eta[:, nd]
    return out
