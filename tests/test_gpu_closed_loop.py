"""GPU: the closed-loop receding-horizon simulation (Sec. 6.3) through
tapg_closed_loop against the oracle's loop on the same seeded inputs: the
state and input trajectories element by element (FP64, 1e-9 of their scale)
at a fixed iteration count per step, and the economic and safety indices."""

import os
import sys

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O
from paper_1904_10548_amd import tapg

from gpu_helpers import add_tree, make_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_schedule():
    for k in ("TAPG_LEVELS", "TAPG_PROJ", "TAPG_CHAIN", "TAPG_SCAN", "TAPG_FWD_GROUP"):
        os.environ.pop(k, None)
    os.environ["TAPG_USE_GRAPH"] = "1"
    os.environ["TAPG_SEGMENTS"] = "1"
    yield


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _run(P, inp, H, gamma, iters, tol=0.0, warm=True, check_every=50):
    with make_solver(P, gamma=gamma, tol=tol, max_iter=iters, check_every=check_every) as S:
        t = add_tree(S, P)
        return tapg.tapg_closed_loop(S.h, t, H, P.p, P.q,
                                     lambda k: inp.tree_data(P.net, P.tree, k), P.tree.K,
                                     P.net.nd, warm_start=warm)


@pytest.mark.parametrize("name,H,iters,warm", [("small", 24, 200, True), ("small", 10, 150, False),
                                               ("dwn128", 3, 30, True)])
def test_closed_loop_matches_oracle_fixed_iterations(name, H, iters, warm):
    P = ds.config_problem(name)
    f = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, f, 60))
    model = ("sinusoid", "uniform") if name == "small" else ("lognormal", "dayahead")
    inp = ds.make_loop_inputs(P.net, H + P.tree.N, seed=11, demand_model=model[0],
                              price_model=model[1])
    say("closed loop", name, H, iters, warm)
    xt, ut, tau, its, st = _run(P, inp, H, gamma, iters, warm=warm)
    ref = O.closed_loop(P, inp, H, gamma, f, iters, warm_start=warm)
    say("KPI_E", st.kpi_E, ref.kpi_E, "KPI_S", st.kpi_S, ref.kpi_S, "KPI_tau ms", st.kpi_tau_ms)
    assert np.all(its == iters) and st.iters == H * iters
    assert np.abs(xt - ref.x).max() <= 1e-9 * max(1.0, np.abs(ref.x).max())
    assert np.abs(ut - ref.u).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())
    assert abs(st.kpi_E - ref.kpi_E) <= 1e-9 * max(1.0, abs(ref.kpi_E))
    assert abs(st.kpi_S - ref.kpi_S) <= 1e-9 * max(1.0, abs(ref.kpi_S))
    assert st.max_viol_eq <= 1e-9
    assert np.all(tau > 0) and st.kpi_tau_ms == pytest.approx(tau.max())


def test_closed_loop_to_tolerance_warm_starts():
    """Steps solved to a tolerance: each step stops within one iteration of the
    oracle's, warm starts cut the iterations of later steps, and the
    trajectories agree to the accuracy the tolerance leaves."""
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / O.lipschitz_dense(P, nf)
    H, tol = 24, 1e-5
    inp = ds.make_loop_inputs(P.net, H + P.tree.N, seed=3, demand_model="sinusoid",
                              price_model="uniform")
    xt, ut, tau, its, st = _run(P, inp, H, gamma, 50000, tol=tol, check_every=1)
    ref = O.closed_loop(P, inp, H, gamma, nf, 50000, tol=tol)
    say("iters", its.tolist(), ref.iters.tolist())
    assert st.steps_converged == H
    assert np.abs(its - ref.iters).max() <= 1
    assert np.abs(ut - ref.u).max() <= 1e-3
    assert its[1:].mean() < its[0]
