"""Marshalling of a generated instance into the tapg binding (no arithmetic)."""

import numpy as np

from paper_1904_10548_amd import tapg


def net_arrays(P):
    n = P.net
    return dict(A=n.A, B=n.B, Gd=n.Gd, E=n.E, Ed=n.Ed, xmin=n.xmin, xmax=n.xmax, xs=n.xs,
                umin=n.umin, umax=n.umax)


def weight_args(P):
    w = P.weights
    return dict(W_alpha=w.W_alpha, W_s=w.W_s, W_x=w.W_x, alpha0=w.alpha0,
                c_energy=w.c_energy, W_u=w.W_u)


def make_solver(P, **cfg):
    return tapg.Solver(net_arrays(P), weight_args(P), P.tree.N, **cfg)


def add_tree(S, P):
    t = P.tree
    return S.add_tree(t.nodes_per_stage, t.anc, t.prob, P.data.demand, P.data.price)
