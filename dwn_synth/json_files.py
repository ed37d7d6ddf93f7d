"""Write a generated instance as the JSON files of the library's front-end
(Sec. 5.1: network, scenario tree, forecaster, controller configuration,
plant state).  Only serialisation: no arithmetic of the method.

The tree file can hold the node values themselves, or the prediction errors
of Sec. 2.2 (eq. prediction-error) with a forecaster file holding the nominal
forecast per stage; :func:`split_forecast` makes that split (forecast = the
stage's first node value, error = value - forecast), and the node data the
library then builds is ``forecast[stage] + error``, which
:func:`node_data_from_split` returns for comparisons.
"""

from __future__ import annotations

import json
import os

import numpy as np


def _rows(a):
    a = np.asarray(a, dtype=np.float64)
    return [[float(v) for v in r] for r in a.reshape(a.shape[0], -1)] if a.size else []


def _vec(a):
    return [float(v) for v in np.asarray(a, dtype=np.float64).ravel()]


def _dump(obj, path):
    with open(path, "w") as f:
        json.dump(obj, f, indent=1, allow_nan=False)
    return path


def write_network(net, path, name="network"):
    return _dump({"name": name, "nx": int(net.nx), "nu": int(net.nu), "nd": int(net.nd),
                  "ns": int(net.ns), "A": _rows(net.A), "B": _rows(net.B), "Gd": _rows(net.Gd),
                  "E": _rows(net.E), "Ed": _rows(net.Ed), "xmin": _vec(net.xmin),
                  "xmax": _vec(net.xmax), "xs": _vec(net.xs), "umin": _vec(net.umin),
                  "umax": _vec(net.umax)}, path)


def _stages(tree):
    return np.repeat(np.arange(len(tree.nodes_per_stage)), tree.nodes_per_stage)


def split_forecast(tree, demand, price):
    """(forecast demand [N, nd], forecast price [N], demand errors [K, nd],
    price errors [K]) with value = forecast[stage] + error up to rounding."""
    st = _stages(tree)
    first = np.concatenate([[0], np.cumsum(tree.nodes_per_stage)[:-1]])
    fd, fp = np.asarray(demand)[first], np.asarray(price)[first]
    return fd, fp, np.asarray(demand) - fd[st], np.asarray(price) - fp[st]


def node_data_from_split(tree, fd, fp, ed, ep):
    st = _stages(tree)
    return fd[st] + ed, fp[st] + ep


def write_tree(tree, path, demand=None, price=None, demand_error=None, price_error=None,
               children=False, name="scenario tree"):
    obj = {"name": name, "N": int(len(tree.nodes_per_stage)),
           "nodes_per_stage": [int(v) for v in tree.nodes_per_stage],
           "ancestor": [int(v) for v in tree.anc], "probability": _vec(tree.prob)}
    if children:
        K = int(np.sum(tree.nodes_per_stage))
        ch = [[] for _ in range(K)]
        for n in range(1, K):
            ch[int(tree.anc[n])].append(n)
        obj["children"] = ch
    if demand is not None:
        obj["demand"], obj["price"] = _rows(demand), _vec(price)
    else:
        obj["demand_error"], obj["price_error"] = _rows(demand_error), _vec(price_error)
    return _dump(obj, path)


def write_forecaster(fd, fp, path):
    return _dump({"name": "forecaster", "demand": _rows(fd), "price": _vec(fp)}, path)


def write_config(weights, path, tol, max_iter, **extra):
    w = weights
    obj = {"W_alpha": float(w.W_alpha), "W_s": float(w.W_s), "W_x": float(w.W_x),
           "alpha0": _vec(w.alpha0), "c_energy": _vec(w.c_energy), "W_u": _rows(w.W_u),
           "tol": float(tol), "max_iter": int(max_iter)}
    obj.update(extra)
    return _dump(obj, path)


def write_state(x, u_prev, path, k=0):
    return _dump({"k": int(k), "x": _vec(x), "u_prev": _vec(u_prev)}, path)


def write_instance(P, folder, tol=1e-4, max_iter=10000, errors=True, **config):
    """All five input files of an instance under ``folder``; returns their
    paths (forecaster None when the tree holds node values)."""
    os.makedirs(folder, exist_ok=True)
    j = lambda n: os.path.join(folder, n)  # noqa: E731
    paths = {"network": write_network(P.net, j("network.json")),
             "config": write_config(P.weights, j("controllerconfig.json"), tol, max_iter, **config),
             "state": write_state(P.p, P.q, j("state.json")), "forecaster": None}
    if errors:
        fd, fp, ed, ep = split_forecast(P.tree, P.data.demand, P.data.price)
        paths["tree"] = write_tree(P.tree, j("scenarioTree.json"), demand_error=ed, price_error=ep)
        paths["forecaster"] = write_forecaster(fd, fp, j("forecaster.json"))
    else:
        paths["tree"] = write_tree(P.tree, j("scenarioTree.json"), demand=P.data.demand,
                                   price=P.data.price)
    return paths
