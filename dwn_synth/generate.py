"""Seeded generators for networks, scenario trees and node data.

The paper's own workload (the Barcelona network with EXAA day-ahead prices,
Sec. 6) is not available, so these generators produce synthetic instances
with its dimensions (63 tanks, 114 flows of which 75 pumps and 39 valves,
88 demand sectors, 17 mixing nodes), its horizon (24 hourly stages) and a
range of scenario counts.

Construction rules (all seeded, ``numpy.random.Generator``):

* every tank gets one source->tank pump, so every tank can be refilled;
* every mixing node gets one tank->mixing valve and one demand, plus the
  extra source->mixing pumps; the inputs of different mixing nodes are
  disjoint, so ``E`` has full row rank;
* the remaining valves link random pairs of tanks, the remaining demands
  are drawn from random tanks;
* ``A = I`` (tanks integrate their net inflow over one sampling period).

Nothing here computes any part of the solver.
"""

from __future__ import annotations

import math

import numpy as np

from .problem import Network, NodeData, Problem, ScenarioTree, Weights

# ---------------------------------------------------------------------------
# Workload configurations.  Each names its sizes and seed; sub-streams of the
# seed feed the network, the tree and the node data separately.
# ---------------------------------------------------------------------------
CONFIGS = {
    # Small network, horizon 6, binary branching at stages 1-2 (4 scenarios).
    "small": dict(nx=4, nu=6, nd=3, ns=2, n_pumps=4, N=6, b1=2, S=4, seed=1001,
                  demand_model="sinusoid", price_model="uniform"),
    # Barcelona-sized network, 24 hourly stages, 4 then x2 up to 128 scenarios.
    "dwn128": dict(nx=63, nu=114, nd=88, ns=17, n_pumps=75, N=24, b1=4, S=128,
                   seed=1002, demand_model="lognormal", price_model="dayahead"),
    # 64 uneven trees, scenario counts drawn from {16,...,256}.
    "batch64": dict(nx=63, nu=114, nd=88, ns=17, n_pumps=75, N=24, b1=4,
                    S_choices=(16, 32, 64, 128, 256), n_trees=64, seed=1003,
                    demand_model="lognormal", price_model="dayahead"),
    # Receding-horizon requests with trees of 32..512 scenarios.
    "serve": dict(nx=63, nu=114, nd=88, ns=17, n_pumps=75, N=24, b1=4,
                  S_choices=(32, 64, 128, 256, 512), rate_hz=200.0, seed=1004,
                  demand_model="lognormal", price_model="dayahead"),
    # One large tree with 2048 scenarios.
    "dwn2048": dict(nx=63, nu=114, nd=88, ns=17, n_pumps=75, N=24, b1=4, S=2048,
                    seed=1005, demand_model="lognormal", price_model="dayahead"),
}


def _streams(seed: int, n: int = 3):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------
def make_network(rng: np.random.Generator, nx: int, nu: int, nd: int, ns: int,
                 n_pumps: int) -> Network:
    """Random flow network with the stated dimensions (see module doc)."""
    n_src_row = n_pumps - nx
    n_tank_tank = nu - n_pumps - ns
    if n_src_row < 0 or n_tank_tank < 0 or nd < ns:
        raise ValueError("inconsistent network dimensions")
    if n_tank_tank > 0 and nx < 2:
        raise ValueError("tank->tank valves need at least two tanks")

    cols = []  # (kind, a, b): kind in src_tank, tank_row, src_row, tank_tank
    for t in range(nx):
        cols.append(("src_tank", t, -1))
    feed = rng.choice(nx, size=ns, replace=ns > nx)  # distinct feeding tanks
    for r in range(ns):
        cols.append(("tank_row", int(feed[r]), r))
    for _ in range(n_src_row):
        cols.append(("src_row", -1, int(rng.integers(ns))))
    for _ in range(n_tank_tank):
        a, b = rng.choice(nx, size=2, replace=False)
        cols.append(("tank_tank", int(a), int(b)))
    perm = rng.permutation(nu)
    cols = [cols[i] for i in perm]

    B = np.zeros((nx, nu))
    E = np.zeros((ns, nu))
    is_pump = np.zeros(nu, dtype=bool)
    for i, (kind, a, b) in enumerate(cols):
        if kind == "src_tank":
            B[a, i] = 1.0
            is_pump[i] = True
        elif kind == "tank_row":
            B[a, i] = -1.0
            E[b, i] = 1.0
        elif kind == "src_row":
            E[b, i] = 1.0
            is_pump[i] = True
        else:
            B[a, i] = -1.0
            B[b, i] = 1.0

    Gd = np.zeros((nx, nd))
    Ed = np.zeros((ns, nd))
    dem_sites = [("row", r) for r in range(ns)]
    # Tank demands go round-robin over a random order of the tanks that do
    # not feed a mixing node (then over all tanks), so that no tank carries
    # more load than its source pump can refill.
    free = [t for t in rng.permutation(nx) if t not in set(int(f) for f in feed)]
    order = free if free else list(rng.permutation(nx))
    dem_sites += [("tank", int(order[i % len(order)])) for i in range(nd - ns)]
    dperm = rng.permutation(nd)
    dem_sites = [dem_sites[i] for i in dperm]
    for k, (kind, idx) in enumerate(dem_sites):
        if kind == "row":
            Ed[idx, k] = -1.0
        else:
            Gd[idx, k] = -1.0

    return Network(
        A=np.eye(nx), B=B, Gd=Gd, E=E, Ed=Ed,
        xmin=np.zeros(nx), xmax=np.full(nx, 10.0), xs=np.full(nx, 2.0),
        umin=np.zeros(nu), umax=np.full(nu, 5.0), is_pump=is_pump,
        kind=tuple(c[0] for c in cols),
    )


def steady_input(net: Network, d: np.ndarray) -> np.ndarray:
    """A feasible input that keeps the tanks level under demand ``d``: each
    mixing node's demand is split evenly over its inflows, tank->tank valves
    are closed, and every source pump refills its tank's outflow (clipped to
    the pump's range).  Used as the previous input ``q`` of a first solve."""
    u = np.zeros(net.nu)
    row_dem = -(net.Ed @ d)
    for r in range(net.ns):
        ins = np.nonzero(net.E[r] > 0)[0]
        u[ins] = row_dem[r] / len(ins)
    out = -(net.Gd @ d)
    for i, k in enumerate(net.kind):
        if k == "tank_row":
            out[int(np.argmin(net.B[:, i]))] += u[i]
    for i, k in enumerate(net.kind):
        if k == "src_tank":
            t = int(np.argmax(net.B[:, i]))
            u[i] = out[t]
    return np.minimum(np.maximum(u, net.umin), net.umax)


# ---------------------------------------------------------------------------
# Scenario trees
# ---------------------------------------------------------------------------
def nodes_per_stage_for(N: int, b1: int, S: int) -> np.ndarray:
    """Stage widths: one root, ``b1`` nodes at stage 1, then doubling until
    ``S`` scenarios, then constant."""
    mu = [1]
    for s in range(1, N):
        m = min(b1, S) if s == 1 else min(2 * mu[-1], S)
        mu.append(max(m, mu[-1]))
    return np.asarray(mu, dtype=np.int64)


def _tree_from_child_counts(rng, N, counts_per_stage):
    """Build breadth-first ``anc`` and ``prob`` from per-node child counts.

    ``counts_per_stage[s]`` lists the number of children of every node of
    stage ``s`` (s = 0..N-2).  Conditional branch probabilities are drawn
    proportional to U[0.5, 1.5] so that the tree is not uniform.
    """
    anc = [-1]
    prob = [1.0]
    mu = [1]
    first = 0
    for s in range(N - 1):
        counts = counts_per_stage[s]
        assert len(counts) == mu[-1]
        for i, c in enumerate(counts):
            parent = first + i
            wts = rng.uniform(0.5, 1.5, size=c)
            wts = wts / wts.sum()
            for k in range(c):
                anc.append(parent)
                prob.append(prob[parent] * wts[k])
        first += mu[-1]
        mu.append(int(sum(counts)))
    return ScenarioTree(N=N, nodes_per_stage=np.asarray(mu, dtype=np.int64),
                        anc=np.asarray(anc, dtype=np.int64),
                        prob=np.asarray(prob, dtype=np.float64))


def make_tree(rng: np.random.Generator, N: int, b1: int, S: int) -> ScenarioTree:
    """Regular tree with the widths of :func:`nodes_per_stage_for`; when a
    stage grows by a non-integer factor the extra children go to the first
    nodes of the stage."""
    mu = nodes_per_stage_for(N, b1, S)
    counts_per_stage = []
    for s in range(N - 1):
        base, extra = divmod(int(mu[s + 1]), int(mu[s]))
        counts_per_stage.append([base + (1 if i < extra else 0) for i in range(mu[s])])
    return _tree_from_child_counts(rng, N, counts_per_stage)


def make_irregular_tree(rng: np.random.Generator, N: int, max_children: int = 3,
                        max_width: int = 64) -> ScenarioTree:
    """Tree whose non-leaf nodes have a random number of children
    (1..max_children), every leaf at stage N-1, stage width capped."""
    counts_per_stage = []
    width = 1
    for s in range(N - 1):
        counts = [int(rng.integers(1, max_children + 1)) for _ in range(width)]
        while sum(counts) > max_width:
            j = int(np.argmax(counts))
            counts[j] -= 1
        counts_per_stage.append(counts)
        width = sum(counts)
    return _tree_from_child_counts(rng, N, counts_per_stage)


def _stages_of(tree: ScenarioTree) -> np.ndarray:
    return np.repeat(np.arange(tree.N), tree.nodes_per_stage)


# ---------------------------------------------------------------------------
# Node data (demands and prices)
# ---------------------------------------------------------------------------
def make_node_data(rng: np.random.Generator, net: Network, tree: ScenarioTree,
                   demand_model: str = "lognormal", price_model: str = "dayahead",
                   hour0: int = 0) -> NodeData:
    """Per-node demand and price.

    The forecast follows a daily sinusoidal profile; every node other than
    the root adds its own prediction error (the root's error is zero, as at
    stage 0 of the paper's tree).

    * ``sinusoid`` demand: ``dbar_k (1 + 0.3 sin(2 pi (h+phi_k)/24)) + N(0, 0.1)``,
      clipped at 0, with ``dbar_k ~ U[0.4, 1.2]``;
    * ``lognormal`` demand: the same profile times ``exp(N(0, 0.1^2))``;
    * ``uniform`` price: ``U[0.05, 0.2]`` at every node;
    * ``dayahead`` price: ``0.1 (1 + 0.5 sin(2 pi (h-8)/24))`` times
      ``(1 + 0.2 N(0,1))``, clipped at 0.005.
    """
    K, nd = tree.K, net.nd
    st = _stages_of(tree)
    hours = hour0 + st
    dbar = rng.uniform(0.4, 1.2, size=nd)
    phi = rng.uniform(0.0, 24.0, size=nd)
    profile = dbar[None, :] * (1.0 + 0.3 * np.sin(2 * math.pi * (hours[:, None] + phi[None, :]) / 24.0))
    if demand_model == "sinusoid":
        noise = rng.normal(0.0, 0.1, size=(K, nd))
        noise[0] = 0.0
        demand = np.maximum(profile + noise, 0.0)
    elif demand_model == "lognormal":
        noise = rng.normal(0.0, 0.1, size=(K, nd))
        noise[0] = 0.0
        demand = profile * np.exp(noise)
    else:
        raise ValueError(demand_model)

    if price_model == "uniform":
        price = rng.uniform(0.05, 0.2, size=K)
    elif price_model == "dayahead":
        base = 0.1 * (1.0 + 0.5 * np.sin(2 * math.pi * (hours - 8.0) / 24.0))
        mult = 1.0 + 0.2 * rng.normal(size=K)
        mult[0] = 1.0
        price = np.maximum(base * mult, 0.005)
    else:
        raise ValueError(price_model)
    return NodeData(demand=np.ascontiguousarray(demand), price=np.ascontiguousarray(price))


def make_weights(rng: np.random.Generator, net: Network) -> Weights:
    """Scale-free analogues of the paper's weights: ``W_alpha = 1``,
    ``W_u = 100 I``, ``W_s = 10``, ``W_x = 100``; production cost ``alpha0`` on
    the inputs fed from a source (U[0.01, 0.05]), energy cost on pumps only.

    ``W_u`` sets the curvature of the dual (its Lipschitz constant scales as
    ``1/W_u``); with ``W_u = I`` the Barcelona-sized instance needs far more
    than 10^5 iterations to reach a residual of 1e-4, with ``100 I`` it
    converges in the 10^4 range."""
    nu = net.nu
    from_source = net.is_pump  # every pump in these networks draws from a source
    alpha0 = np.where(from_source, rng.uniform(0.01, 0.05, size=nu), 0.0)
    return Weights(W_alpha=1.0, W_u=100.0 * np.eye(nu), W_s=10.0, W_x=100.0,
                   alpha0=alpha0, c_energy=net.is_pump.astype(np.float64))


def dense_input_weight(nu: int, seed: int = 5, base: float = 100.0, coupling: float = 5.0,
                       rank: int = 8) -> np.ndarray:
    """A dense symmetric positive definite ``W_u = base I + coupling M M' / rank``
    (``M`` seeded standard normal, ``nu x rank``): the smoothing cost couples
    the inputs, so no stage factor reduces to a projector (the general path)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    M = rng.standard_normal((nu, rank))
    W = base * np.eye(nu) + coupling * (M @ M.T) / rank
    return 0.5 * (W + W.T)


def make_problem(nx, nu, nd, ns, n_pumps, N, b1, S, seed, demand_model="lognormal",
                 price_model="dayahead", hour0=0, name="") -> Problem:
    """Full instance from one seed (three sub-streams: network, tree, data)."""
    rn, rt, rd = _streams(seed)
    net = make_network(rn, nx, nu, nd, ns, n_pumps)
    w = make_weights(rn, net)
    tree = make_tree(rt, N, b1, S)
    data = make_node_data(rd, net, tree, demand_model, price_model, hour0)
    return Problem(net=net, tree=tree, data=data, weights=w,
                   p=np.full(nx, 5.0), q=steady_input(net, data.demand[0]), name=name,
                   meta=dict(seed=seed, S=S, N=N, b1=b1))


def config_problem(name: str, index: int = 0) -> Problem:
    """Instance of a named configuration.  For the multi-tree configurations
    (``batch64``, ``serve``) ``index`` selects the tree; all trees of one
    configuration share the network and weights."""
    c = CONFIGS[name]
    if "S" in c:
        return make_problem(c["nx"], c["nu"], c["nd"], c["ns"], c["n_pumps"], c["N"],
                            c["b1"], c["S"], c["seed"], c["demand_model"],
                            c["price_model"], name=name)
    rn, rt, rd = _streams(c["seed"])
    net = make_network(rn, c["nx"], c["nu"], c["nd"], c["ns"], c["n_pumps"])
    w = make_weights(rn, net)
    # per-tree streams: scenario count, tree and data of tree ``index``
    rs_i = np.random.default_rng(np.random.SeedSequence([c["seed"], 3, index]))
    S = int(rs_i.choice(np.asarray(c["S_choices"])))
    rt_i = np.random.default_rng(np.random.SeedSequence([c["seed"], 7, index]))
    rd_i = np.random.default_rng(np.random.SeedSequence([c["seed"], 11, index]))
    tree = make_tree(rt_i, c["N"], c["b1"], S)
    data = make_node_data(rd_i, net, tree, c["demand_model"], c["price_model"],
                          hour0=int(index % 24))
    return Problem(net=net, tree=tree, data=data, weights=w, p=np.full(c["nx"], 5.0),
                   q=steady_input(net, data.demand[0]), name=f"{name}[{index}]",
                   meta=dict(seed=c["seed"], S=S, N=c["N"], b1=c["b1"], index=index))
