"""Seeded inputs of a closed-loop receding-horizon simulation (Sec. 6.3).

Only input generation: the observed demand and price at every sampling
instant, and, for every instant k, the forecast scenario tree's node data
(Sec. 2.3: the forecast plus a prediction error per node, zero error at the
root, which therefore carries the demand and price observed at k).  The
demand profile is the daily sinusoid of :func:`dwn_synth.generate.make_node_data`
with lognormal errors (sigma 0.1); the price is the day-ahead sinusoid with
20 % multiplicative errors.  Observations use the same error model as the
forecast's nodes, so the tree describes the uncertainty the plant meets.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .problem import Network, ScenarioTree


def _stages(tree: ScenarioTree) -> np.ndarray:
    return np.repeat(np.arange(tree.N), tree.nodes_per_stage)


@dataclass
class LoopInputs:
    """Demand profile parameters and the observed series of one simulation."""
    dbar: np.ndarray       # (nd,) mean demand
    phi: np.ndarray        # (nd,) phase (hours)
    demand: np.ndarray     # (H, nd) observed demand at each instant
    price: np.ndarray      # (H,) observed price at each instant
    seed: int
    demand_model: str
    price_model: str

    def profile(self, hours: np.ndarray) -> np.ndarray:
        return self.dbar[None, :] * (1.0 + 0.3 * np.sin(
            2 * math.pi * (hours[:, None] + self.phi[None, :]) / 24.0))

    def price_base(self, hours: np.ndarray) -> np.ndarray:
        if self.price_model == "dayahead":
            return 0.1 * (1.0 + 0.5 * np.sin(2 * math.pi * (hours - 8.0) / 24.0))
        return np.full(hours.shape, 0.125)

    def _demand_at(self, hours, noise):
        prof = self.profile(hours)
        if self.demand_model == "lognormal":
            return prof * np.exp(noise)
        return np.maximum(prof + noise, 0.0)

    def _price_at(self, hours, noise):
        if self.price_model == "dayahead":
            return np.maximum(self.price_base(hours) * (1.0 + 0.2 * noise), 0.005)
        return self.price_base(hours) * (1.0 + 0.4 * np.clip(noise, -1.5, 1.5) / 1.5)

    def tree_data(self, net: Network, tree: ScenarioTree, k: int):
        """Node data of the tree solved at instant k: (demand (K, nd), price (K))."""
        rng = np.random.default_rng(np.random.SeedSequence([self.seed, 101, k]))
        hours = k + _stages(tree).astype(np.float64)
        dn = rng.normal(0.0, 0.1, size=(tree.K, net.nd))
        pn = rng.normal(size=tree.K)
        demand = self._demand_at(hours, dn)
        price = self._price_at(hours, pn)
        demand[0] = self.demand[k]
        price[0] = self.price[k]
        return np.ascontiguousarray(demand), np.ascontiguousarray(price)


def make_loop_inputs(net: Network, H: int, seed: int, demand_model: str = "lognormal",
                     price_model: str = "dayahead") -> LoopInputs:
    """Observed demand and price at instants 0..H-1 (seeded)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 100]))
    dbar = rng.uniform(0.4, 1.2, size=net.nd)
    phi = rng.uniform(0.0, 24.0, size=net.nd)
    inp = LoopInputs(dbar=dbar, phi=phi, demand=np.zeros((H, net.nd)), price=np.zeros(H),
                     seed=seed, demand_model=demand_model, price_model=price_model)
    hours = np.arange(H, dtype=np.float64)
    inp.demand = inp._demand_at(hours, rng.normal(0.0, 0.1, size=(H, net.nd)))
    inp.price = inp._price_at(hours, rng.normal(size=H))
    return inp
