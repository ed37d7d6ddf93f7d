"""The C-ABI library: it loads, exports every declared symbol, and rejects
invalid networks and trees on the host (no GPU needed for these calls)."""

import ctypes
import os
import re

import numpy as np
import pytest

import dwn_synth as ds
from paper_1904_10548_amd import tapg

from helpers import tiny_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tapg.h")).read()
    return sorted(set(re.findall(r"\b(tapg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = tapg.lib()
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(tapg.EXPORTED)
    assert "gfx950" in tapg.tapg_version()


def _net_args(P):
    n = P.net
    return [n.A, n.B, n.Gd, n.E, n.Ed, n.xmin, n.xmax, n.xs, n.umin, n.umax]


def test_network_create_and_validation():
    P = ds.config_problem("small")
    h = tapg.tapg_network_create(*_net_args(P))
    tapg.tapg_network_destroy(h)
    # rank-deficient E
    bad = _net_args(P)
    bad[3] = np.vstack([P.net.E[0], P.net.E[0]])
    with pytest.raises(tapg.TapgError) as e:
        tapg.tapg_network_create(*bad)
    assert e.value.status == tapg.TAPG_ENUMERIC
    # umin > umax
    bad = _net_args(P)
    bad[8] = P.net.umax + 1.0
    with pytest.raises(tapg.TapgError) as e:
        tapg.tapg_network_create(*bad)
    assert e.value.status == tapg.TAPG_EINVAL
    # non-finite
    bad = _net_args(P)
    bad[0] = P.net.A.copy()
    bad[0][0, 0] = np.nan
    with pytest.raises(tapg.TapgError):
        tapg.tapg_network_create(*bad)


def _tree_args(P):
    t = P.tree
    return [t.nodes_per_stage.copy(), t.anc.copy(), t.prob.copy(), P.data.demand.copy(),
            P.data.price.copy()]


def test_tree_create_valid_and_irregular():
    for P in [ds.config_problem("small"), tiny_problem(N=5, irregular=True, seed=3),
              ds.config_problem("dwn128")]:
        h = tapg.tapg_tree_create(*_tree_args(P))
        assert tapg.tapg_tree_num_nodes(h) == P.tree.K
        tapg.tapg_tree_set_data(h, P.data.demand * 1.1, P.data.price)
        tapg.tapg_tree_destroy(h)


@pytest.mark.parametrize("case", ["prob_sum", "root_prob", "not_bfs", "leaf_early", "anc_range",
                                  "mu0", "neg_prob"])
def test_tree_validation_errors(case):
    P = ds.config_problem("small")
    mu, anc, prob, dem, price = _tree_args(P)
    if case == "prob_sum":
        prob[5] *= 1.01
    elif case == "root_prob":
        prob[0] = 0.9
    elif case == "not_bfs":
        # stage 2 nodes 3..6 have parents 1,1,2,2; swap to make them non-contiguous
        anc[3], anc[5] = anc[5], anc[3]
    elif case == "leaf_early":
        # the last stage-4 node loses its child: give it to the previous node
        anc[-1] = anc[-2]
        prob[-1] = prob[-1]
    elif case == "anc_range":
        anc[4] = 99
    elif case == "mu0":
        mu = mu.copy()
        mu[0], mu[1] = 2, mu[1] - 1
    elif case == "neg_prob":
        prob[7] = -prob[7]
    with pytest.raises(tapg.TapgError) as e:
        tapg.tapg_tree_create(mu, anc, prob, dem, price)
    assert e.value.status in (tapg.TAPG_EINVAL, tapg.TAPG_EDIM)
    assert tapg.tapg_last_error() != ""


def test_null_handles_are_errors():
    L = tapg.lib()
    assert L.tapg_factor_step(None, 4) == tapg.TAPG_EINVAL
    assert L.tapg_tree_num_nodes(None) == -1
    r = tapg.TapgResult()
    assert L.tapg_residuals(None, None, ctypes.byref(r)) == tapg.TAPG_EINVAL
    # destroy functions accept NULL
    L.tapg_tree_destroy(None)
    L.tapg_network_destroy(None)
    L.tapg_solver_destroy(None)


@pytest.mark.parametrize("name", ["small", "dwn128", "dwn2048"])
@pytest.mark.parametrize("precision", [tapg.TAPG_FP64, tapg.TAPG_FP32])
def test_schedule_plan_covers_stages(name, precision):
    """The planner's levels cover stages 0..N-1 in order, every workgroup
    holds at most 4 nodes per stage, and the groups of a level cover its
    first stage."""
    P = ds.config_problem(name)
    h = tapg.tapg_tree_create(*_tree_args(P))
    try:
        plan = tapg.tapg_plan_schedule(h, precision)
    finally:
        tapg.tapg_tree_destroy(h)
    cap = 4
    assert plan[0][0] == 0 and plan[-1][1] == P.tree.N - 1
    for a, b in zip(plan, plan[1:]):
        assert b[0] == a[1] + 1
    for s0, s1, g, nwg, wmax in plan:
        assert wmax <= cap
        assert nwg == -(-int(P.tree.nodes_per_stage[s0]) // g)


def test_schedule_override_and_rejection():
    P = ds.config_problem("dwn128")
    h = tapg.tapg_tree_create(*_tree_args(P))
    try:
        plan = tapg.tapg_plan_schedule(h, tapg.TAPG_FP64, "0:1,2:2,4:1")
        assert [p[:3] for p in plan] == [(0, 1, 1), (2, 3, 2), (4, 23, 1)]
        assert max(p[4] for p in plan) == 4
        with pytest.raises(tapg.TapgError):
            tapg.tapg_plan_schedule(h, tapg.TAPG_FP64, "1:1,4:1")  # must start at stage 0
        # one workgroup from stage 2 (8 nodes) down to stage 5 would hold 8
        # nodes of stage 5: beyond the limit of 4 in either precision
        plan = tapg.tapg_plan_schedule(h, tapg.TAPG_FP32, "0:1,2:1,5:1")
        assert max(p[4] for p in plan) == 4
        for prec in (tapg.TAPG_FP64, tapg.TAPG_FP32):
            with pytest.raises(tapg.TapgError):
                tapg.tapg_plan_schedule(h, prec, "0:1,2:1,6:1")
    finally:
        tapg.tapg_tree_destroy(h)


def test_server_argument_errors_on_host():
    """Server entry points validate their arguments before touching a device."""
    import ctypes
    L = tapg.lib()
    out = ctypes.c_void_p()
    assert L.tapg_server_create(None, 1 << 30, 8, ctypes.byref(out)) == tapg.TAPG_EINVAL
    assert L.tapg_server_poll(None, 1, 0, None, None, None) == tapg.TAPG_EINVAL
    assert L.tapg_server_stats(None, None, None, None, None) == tapg.TAPG_EINVAL
    t = ctypes.c_longlong(0)
    assert L.tapg_server_submit(None, None, None, None, 0, ctypes.byref(t)) == tapg.TAPG_EINVAL
    L.tapg_server_destroy(None)  # no-op
    assert L.tapg_server_timing(None, None, None, None) == tapg.TAPG_EINVAL


def test_sweep_form_argument_errors_on_host():
    """tapg_sweep_form rejects missing handles and empty batches before any
    device work."""
    import ctypes
    L = tapg.lib()
    f, nl = ctypes.c_int(-1), ctypes.c_int(-1)
    assert L.tapg_sweep_form(None, 1, None, ctypes.byref(f), ctypes.byref(nl)) == tapg.TAPG_EINVAL
    assert f.value == -1 and nl.value == -1
    buf = ctypes.create_string_buffer(64)
    assert L.tapg_schedule_spec(None, 1, None, buf, 64) == tapg.TAPG_EINVAL
    assert buf.value == b""
    us = ctypes.c_double(-1.0)
    assert L.tapg_event_pair_overhead(None, ctypes.byref(us)) == tapg.TAPG_EINVAL
    assert us.value == -1.0
    assert tapg.FORM_NAMES == {0: "stages", 1: "segment", 2: "projector", 3: "scan"}
