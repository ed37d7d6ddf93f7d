"""GPU: batched solves (several trees swept together as one forest) against
the FP64 oracle per tree and against single-tree solves of the same trees.

Bars as for single trees (FP64): iterates to 1e-9 of their scale, cost to 1e-6
relative; against a single-tree GPU solve the same arithmetic runs per node,
so iteration counts are equal and iterates agree to 1e-12.
"""

import os
import sys

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O
from paper_1904_10548_amd import tapg

from gpu_helpers import add_tree, make_solver
from helpers import tiny_batch

pytestmark = pytest.mark.gpu

SHAPES = [(2, 4), (3, 3), ("irregular", 3, 20), (1, 1), (2, 8)]


@pytest.fixture(autouse=True)
def _default_schedule():
    for k in ("TAPG_LEVELS", "TAPG_PROJ", "TAPG_CHAIN", "TAPG_SCAN", "TAPG_FWD_GROUP", "TAPG_TOP"):
        os.environ.pop(k, None)
    os.environ["TAPG_USE_GRAPH"] = "1"
    os.environ["TAPG_SEGMENTS"] = "1"
    yield


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _gamma_for(batch):
    """One step size valid for every tree of the batch (0.9 / max L)."""
    Ls = []
    for P in batch:
        Ls.append(O.lipschitz_power(P, O.StageFactors(P.net, P.weights.W_u, P.tree), 300))
    return 0.9 / max(Ls)


def _force(scan=None, fwd_group=None, top=None, levels="0:1,2:1,3:1"):
    """Schedule switches; light upper levels come with a plan of three levels
    (the default plan of a small forest may have one)."""
    for k, v in (("TAPG_SCAN", scan), ("TAPG_FWD_GROUP", fwd_group), ("TAPG_TOP", top),
                 ("TAPG_LEVELS", levels if top else None)):
        if v:
            os.environ[k] = v


@pytest.mark.parametrize("scan,fwd_group,top", [("0", None, None), (None, None, None),
                                                ("1", "1", None), ("1", None, "1"),
                                                ("1", "1", "1")])
def test_batch_fixed_iterations_matches_oracle_per_tree(scan, fwd_group, top):
    """Every tree of a forest against its own oracle run: the segment form,
    the default (scan) form, the scan form's forward launch on one leaf per
    workgroup, and the scan form with light upper levels (every tree's upper
    levels inside the bottom level's backward launch)."""
    _force(scan, fwd_group, top)
    batch = tiny_batch(SHAPES)
    gamma = _gamma_for(batch)
    iters = 300
    say("batch fixed", [P.tree.K for P in batch], "iters", iters, "scan", scan, "fwd", fwd_group,
        "top", top)
    with make_solver(batch[0], gamma=gamma, tol=0.0, max_iter=iters, check_every=64) as S:
        trees = [add_tree(S, P) for P in batch]
        st, u0s, res = S.batch_solve(trees, [P.p for P in batch], [P.q for P in batch])
        out = [(S.primal(t), S.dual(t), tapg.tapg_residual_history(S.h, t, iters)) for t in trees]
        form = tapg.tapg_sweep_form(S.h, trees)
    assert st == tapg.TAPG_OK
    if top:  # one backward launch per iteration
        assert form[0] == "scan" and form[1] == 1
    for P, r, u0, ((u, x), y, hist) in zip(batch, res, u0s, out):
        ref = O.apg(P, gamma, O.StageFactors(P.net, P.weights.W_u, P.tree), iters)
        assert r.iters == iters
        su, sx, sy = (max(1.0, np.abs(v).max()) for v in (ref.u, ref.x, ref.y))
        assert np.abs(u - ref.u).max() <= 1e-9 * su
        assert np.abs(x - ref.x).max() <= 1e-9 * sx
        assert np.abs(y - ref.y).max() <= 1e-9 * sy
        assert np.abs(u0 - ref.u[0]).max() <= 1e-9 * su
        J = O.primal_cost(P, ref.u, ref.x)
        assert abs(r.cost - J) <= 1e-6 * max(1.0, abs(J))
        vb, ve = O.violations(P, ref.u, ref.x)
        assert abs(r.viol_box - vb) <= 1e-6 and r.viol_eq <= 1e-9
        assert np.allclose(hist, ref.res_hist, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("precision", [tapg.TAPG_FP64, tapg.TAPG_FP32])
@pytest.mark.parametrize("check_every,scan,top", [(50, "0", None), (7, None, None), (7, "1", "1")])
def test_batch_equals_single_tree_solves_to_tolerance(precision, check_every, scan, top):
    """Auto step size per tree and a tolerance: every tree stops at the same
    iteration as its own tapg_solve, with the same iterate; trees stop at
    different iterations inside the batch (and inside runs of odd length),
    also with light upper levels (scan form), where a stopped tree's upper
    workgroups take no part in the launches that follow."""
    _force(scan=scan, top=top)
    batch = tiny_batch(SHAPES, seed=23)
    # FP32 sweeps: a tolerance above their floor (the FP64 residual of an FP32
    # dual cannot resolve steps below the dual's rounding over gamma)
    tol = 1e-6 if precision == tapg.TAPG_FP64 else 1e-3
    kw = dict(gamma=0.0, tol=tol, max_iter=20000, check_every=check_every, precision=precision)
    say("batch vs single", [P.tree.K for P in batch], "prec", precision)
    with make_solver(batch[0], **kw) as S:
        trees = [add_tree(S, P) for P in batch]
        st, u0s, res = S.batch_solve(trees, [P.p for P in batch], [P.q for P in batch])
        got = [S.primal(t) for t in trees]
    with make_solver(batch[0], **kw) as S:
        single = []
        for P in batch:
            t = add_tree(S, P)
            st1, u01, r1 = S.solve(t, P.p, P.q)
            single.append((r1, S.primal(t), u01))
    assert st == tapg.TAPG_OK
    assert len({r.iters for r in res}) > 1  # the trees stop at different iterations
    tol = 1e-12 if precision == tapg.TAPG_FP64 else 1e-5
    for r, (u, x), u0, (r1, (u1, x1), u01) in zip(res, got, u0s, single):
        assert r.converged and r1.converged
        assert r.iters == r1.iters
        assert abs(r.gamma - r1.gamma) <= 1e-15 * r1.gamma
        assert np.abs(u - u1).max() <= tol * max(1.0, np.abs(u1).max())
        assert np.abs(x - x1).max() <= tol * max(1.0, np.abs(x1).max())
        assert np.abs(u0 - u01).max() <= tol * max(1.0, np.abs(u01).max())
        assert abs(r.cost - r1.cost) <= 1e-9 * max(1.0, abs(r1.cost))


def test_batch_warm_start_and_resolve():
    """A second batch solve warm-starts the chosen trees from their last dual:
    the same iterations as a warm single-tree solve; cold trees repeat their
    first solve exactly."""
    batch = tiny_batch(SHAPES[:3], seed=5)
    kw = dict(gamma=0.0, tol=1e-6, max_iter=20000, check_every=50)
    with make_solver(batch[0], **kw) as S:
        trees = [add_tree(S, P) for P in batch]
        ps, qs = [P.p for P in batch], [P.q for P in batch]
        _, _, r0 = S.batch_solve(trees, ps, qs)
        ps2 = [p + 0.1 for p in ps]
        _, _, r1 = S.batch_solve(trees, ps2, qs, warm_start=[1, 0, 1])
    with make_solver(batch[0], **kw) as S:
        single = []
        for P, p2 in zip(batch, ps2):
            t = add_tree(S, P)
            S.solve(t, P.p, P.q)
            single.append(S.solve(t, p2, P.q, warm_start=True)[2])
    assert r1[1].iters != 0
    for k in (0, 2):
        assert r1[k].iters == single[k].iters
        assert abs(r1[k].cost - single[k].cost) <= 1e-9 * max(1.0, abs(single[k].cost))


@pytest.mark.parametrize("scan,fwd_group,top", [("0", None, None), ("1", "2", None),
                                                ("1", "2", "1")])
def test_batch_of_full_size_trees_fp32(scan, fwd_group, top):
    """Three Barcelona-sized trees of the 64-tree configuration, FP32 sweeps
    (the segment form, the scan form with its forward launch on pairs of
    leaves, and that with light upper levels): each tree's cost after a fixed
    number of iterations within 1e-4 of the FP64 oracle's."""
    _force(scan, fwd_group, top, levels="0:1,2:1,5:2,7:4")
    batch = [ds.config_problem("batch64", i) for i in range(3)]
    iters = 30
    gamma = 0.0
    say("batch64 x3", [P.tree.K for P in batch])
    with make_solver(batch[0], gamma=gamma, tol=0.0, max_iter=iters, check_every=iters,
                     precision=tapg.TAPG_FP32) as S:
        trees = [add_tree(S, P) for P in batch]
        st, u0s, res = S.batch_solve(trees, [P.p for P in batch], [P.q for P in batch])
    for P, r in zip(batch, res):
        ref = O.apg(P, r.gamma, O.StageFactors(P.net, P.weights.W_u, P.tree), iters)
        J = O.primal_cost(P, ref.u, ref.x)
        assert r.iters == iters
        assert abs(r.cost - J) <= 1e-4 * max(1.0, abs(J))


def test_batch_argument_errors():
    batch = tiny_batch(SHAPES[:2])
    with make_solver(batch[0], gamma=1e-3, tol=0.0, max_iter=5) as S:
        trees = [add_tree(S, P) for P in batch]
        with pytest.raises(tapg.TapgError):
            S.batch_solve([trees[0], trees[0]], [batch[0].p] * 2, [batch[0].q] * 2)
        with pytest.raises(tapg.TapgError):
            S.batch_solve([], [], [])


def test_autotuned_schedule_keeps_parity():
    """The autotuner times the candidate schedules of a batch's forest and of a
    single tree; solves under the chosen schedules still match the oracle."""
    batch = tiny_batch(SHAPES, seed=13)
    gamma = _gamma_for(batch)
    iters = 200
    with make_solver(batch[0], gamma=gamma, tol=0.0, max_iter=iters, check_every=50) as S:
        trees = [add_tree(S, P) for P in batch]
        ms_b, nc_b = tapg.tapg_autotune(S.h, trees, 10)
        ms_1, nc_1 = tapg.tapg_autotune(S.h, trees[2:3], 10)
        form_b = tapg.tapg_sweep_form(S.h, trees)
        form_1 = tapg.tapg_sweep_form(S.h, trees[2:3])
        spec_1 = tapg.tapg_schedule_spec(S.h, trees[2:3])
        say("autotune", ms_b, nc_b, form_b, ms_1, nc_1, form_1, spec_1)
        env = dict(kv.split("=") for kv in spec_1.split())
        assert env["TAPG_SCAN"] == ("1" if form_1[0] == "scan" else "0")
        # one backward launch per level, or one in all with light upper levels
        n_lev = len(env["TAPG_LEVELS"].split(","))
        assert form_1[1] == (1 if env.get("TAPG_TOP") == "1" else n_lev)
        st, u0s, res = S.batch_solve(trees, [P.p for P in batch], [P.q for P in batch])
        u, x = S.primal(trees[2])
        assert tapg.tapg_sweep_form(S.h, trees) == form_b  # the solve keeps the tuned form
    assert nc_b >= 1 and nc_1 >= 1 and ms_b > 0 and ms_1 > 0
    # both sweep forms are candidates where the scan form applies (A = I, W_u = w I)
    assert form_b[0] in ("scan", "projector") and form_1[0] in ("scan", "projector")
    # every schedule candidate in both forms, three further groupings of the
    # scan form's forward launch, then (scan form chosen) the plans again with
    # light upper levels (those where they apply)
    assert nc_b >= 2 + 3 and nc_1 >= 2 + 3
    assert form_b[1] >= 1
    for P, r in zip(batch, res):
        ref = O.apg(P, gamma, O.StageFactors(P.net, P.weights.W_u, P.tree), iters)
        J = O.primal_cost(P, ref.u, ref.x)
        assert r.iters == iters and abs(r.cost - J) <= 1e-6 * max(1.0, abs(J))
    ref = O.apg(batch[2], gamma, O.StageFactors(batch[2].net, batch[2].weights.W_u, batch[2].tree), iters)
    assert np.abs(u - ref.u).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())


def test_schedule_spec_reproduces_the_tuned_solve():
    """The environment settings that tapg_schedule_spec reports force the tuned
    schedule on a fresh solver: the same form and launches, and the same
    iterate bit for bit."""
    P = tiny_batch(SHAPES, seed=13)[4]
    gamma = _gamma_for([P])
    iters = 120
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=40) as S:
        t = add_tree(S, P)
        tapg.tapg_autotune(S.h, [t], 10)
        spec = tapg.tapg_schedule_spec(S.h, [t])
        form = tapg.tapg_sweep_form(S.h, [t])
        S.solve(t, P.p, P.q)
        u1, x1 = S.primal(t)
    say("spec", spec, form)
    env = dict(kv.split("=") for kv in spec.split())
    os.environ.update(env)
    try:
        with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=40) as S:
            t = add_tree(S, P)
            S.solve(t, P.p, P.q)
            assert tapg.tapg_sweep_form(S.h, [t]) == form
            assert tapg.tapg_schedule_spec(S.h, [t]) == spec
            u2, x2 = S.primal(t)
    finally:
        for k in env:
            os.environ.pop(k, None)
    assert np.array_equal(u1, u2) and np.array_equal(x1, x2)


def test_kernel_timing_and_event_pair_overhead():
    """Timed solves count every backward and forward launch of the iterations
    that did work, and the event-pair dispatch cost is a few microseconds."""
    P = tiny_batch(SHAPES, seed=13)[4]
    gamma = _gamma_for([P])
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=45, check_every=20) as S:
        t = add_tree(S, P)
        tapg.tapg_kernel_timing(S.h, True)
        st, u0, r = S.solve(t, P.p, P.q)
        kt = tapg.tapg_kernel_times(S.h)
        tapg.tapg_kernel_timing(S.h, False)
        form, nbwd = tapg.tapg_sweep_form(S.h, [t])
        us = tapg.tapg_event_pair_overhead(S.h)
    say("kernel times", kt, form, nbwd, us)
    assert r.iters == 45
    # the scan form's forward sweep is one launch; the segment form's one per level
    assert kt["bwd"][1] == 45 * nbwd and kt["fwd"][1] == 45 * (1 if form == "scan" else nbwd)
    assert kt["end"][1] == 3  # one per run of iterations (20, 20, 5 of 20)
    assert all(v[0] > 0 for k, v in kt.items() if k != "chain")
    assert 0.0 < us < 50.0


def test_autotune_longer_than_max_iter():
    """Timing runs longer than the solver's max_iter (their residual history
    needs more room than a solve's): the solve afterwards still matches the
    oracle with its own history."""
    P = tiny_batch(SHAPES, seed=13)[4]
    gamma = _gamma_for([P])
    iters = 12
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=iters) as S:
        t = add_tree(S, P)
        ms, nc = tapg.tapg_autotune(S.h, [t], 40)
        st, u0, r = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
        hist = tapg.tapg_residual_history(S.h, t, iters)
    ref = O.apg(P, gamma, O.StageFactors(P.net, P.weights.W_u, P.tree), iters)
    assert ms > 0 and nc >= 1 and r.iters == iters
    assert np.abs(u - ref.u).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())
    assert np.allclose(hist, ref.res_hist, rtol=1e-7, atol=1e-12)
