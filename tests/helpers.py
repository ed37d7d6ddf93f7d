"""Small instances shared by the tests (built from the seeded generators)."""

import numpy as np

import dwn_synth as ds
from dwn_synth.generate import make_network, make_node_data, make_tree, make_weights, \
    make_irregular_tree, steady_input


def tiny_problem(N=3, b1=2, S=2, seed=7, p_level=5.0, price_scale=1.0, irregular=False,
                 max_children=3, max_width=64, wu=1.0):
    """Small-network instance (nx=4, nu=6, nd=3, ns=2) on a short tree, with
    ``W_u = wu I``."""
    ss = np.random.SeedSequence(seed)
    rn, rt, rd = [np.random.default_rng(s) for s in ss.spawn(3)]
    net = make_network(rn, 4, 6, 3, 2, 4)
    w = make_weights(rn, net)
    w.W_u = wu * np.eye(net.nu)
    if irregular:
        tree = make_irregular_tree(rt, N, max_children, max_width)
    else:
        tree = make_tree(rt, N, b1, S)
    data = make_node_data(rd, net, tree, "sinusoid", "uniform")
    data.price = data.price * price_scale
    return ds.Problem(net=net, tree=tree, data=data, weights=w,
                      p=np.full(4, p_level), q=steady_input(net, data.demand[0]),
                      name=f"tiny{seed}")
