"""Seeded synthetic workloads for the scenario-tree stochastic MPC of a
drinking-water network (Sopasakis et al., arXiv 1904.10548).

This package only *generates inputs*: network matrices, scenario trees,
node demands and prices, weights and the initial condition.  It holds none
of the solver's arithmetic, so both the CPU oracle and the GPU library's
tests can draw their inputs from it without sharing any computation.

Data containers follow the paper's notation:

* network (Sec. 2, eqs. dynamics / input-disturbance-coupling):
  ``x+ = A x + B u + Gd d`` and ``E u + Ed d = 0``, boxes
  ``xmin <= x <= xmax`` (soft), safety level ``xs`` (soft) and
  ``umin <= u <= umax`` (hard);
* scenario tree (Sec. 2.3): stages ``0..N-1``, ``mu_j`` nodes per stage,
  breadth-first node numbering with contiguous children, ancestor index and
  node probability ``p``;
* per-node demand ``d`` and electricity price (Sec. 2.2/2.3);
* weights ``W_alpha, W_u, W_s, W_x`` (Sec. 3.1).
"""

from .problem import Network, ScenarioTree, NodeData, Weights, Problem
from .generate import (
    make_network,
    make_tree,
    make_irregular_tree,
    make_node_data,
    make_weights,
    make_problem,
    nodes_per_stage_for,
    CONFIGS,
    config_problem,
    dense_input_weight,
)
from .closed_loop import LoopInputs, make_loop_inputs
from .scenarios import make_error_paths
from . import json_files

__all__ = [
    "Network",
    "ScenarioTree",
    "NodeData",
    "Weights",
    "Problem",
    "make_network",
    "make_tree",
    "make_irregular_tree",
    "make_node_data",
    "make_weights",
    "make_problem",
    "nodes_per_stage_for",
    "CONFIGS",
    "dense_input_weight",
    "config_problem",
    "LoopInputs",
    "make_loop_inputs",
    "make_error_paths",
]
