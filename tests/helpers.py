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


def tiny_batch(shapes, N=5, seed=11, wu=1.0):
    """Several instances on one small network and weight set: ``shapes`` is a
    list of ``(b1, S)`` (regular tree) or ``("irregular", max_children,
    max_width)``; every tree gets its own data and initial state."""
    ss = np.random.SeedSequence(seed)
    rn, *rest = [np.random.default_rng(s) for s in ss.spawn(1 + 3 * len(shapes))]
    net = make_network(rn, 4, 6, 3, 2, 4)
    w = make_weights(rn, net)
    w.W_u = wu * np.eye(net.nu)
    out = []
    for k, shape in enumerate(shapes):
        rt, rd, rp = rest[3 * k:3 * k + 3]
        if shape[0] == "irregular":
            tree = make_irregular_tree(rt, N, shape[1], shape[2])
        else:
            tree = make_tree(rt, N, shape[0], shape[1])
        data = make_node_data(rd, net, tree, "sinusoid", "uniform")
        p = rp.uniform(3.0, 7.0, size=net.nx)
        out.append(ds.Problem(net=net, tree=tree, data=data, weights=w, p=p,
                              q=steady_input(net, data.demand[0]), name=f"batch{seed}[{k}]"))
    return out
