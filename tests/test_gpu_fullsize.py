"""GPU parity at the sizes the measurements are quoted at.

* The 128-scenario tree (K = 2,429) solved to tolerance 1e-4 under the
  benchmark's schedule and under a schedule tuned in the test, against the
  oracle's full solve stored in ``tests/golden/dwn128_tol1e-4.json`` (written
  by ``tests/golden/make_dwn128_golden.py`` from ``oracle/`` alone): the same
  stopping iteration within one, cost and root input within 1e-6 relative.
* Full-size trees of the 64-tree batch in one FP64 forest, element by element
  against the oracle, and the whole 64-tree forest against each tree solved
  alone.
* Served requests on the full-size network at a fixed iteration count against
  the oracle, and served to a tolerance alone and in a mix.

Bars (FP64): iterates to 1e-9 of their scale, cost to 1e-6 relative.
"""

import json
import os
import sys
import time

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O
from paper_1904_10548_amd import tapg

from gpu_helpers import add_tree, make_solver

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dwn128_tol1e-4.json")
# The schedule the benchmark's autotuner chose for this tree (scan form, four
# levels, the three upper ones light, inside the bottom level's backward
# launch; forward launch on groups of one leaf).
BENCH_SPEC = {"TAPG_SCAN": "1", "TAPG_LEVELS": "0:1,1:1,4:1,6:1", "TAPG_FWD_GROUP": "1",
              "TAPG_TOP": "1"}
ENV_KEYS = ("TAPG_LEVELS", "TAPG_PROJ", "TAPG_CHAIN", "TAPG_SCAN", "TAPG_FWD_GROUP",
            "TAPG_TOP", "TAPG_TEST_SERVER_SETUP_FAIL")


@pytest.fixture(autouse=True)
def _default_schedule():
    for k in ENV_KEYS:
        os.environ.pop(k, None)
    os.environ["TAPG_USE_GRAPH"] = "1"
    os.environ["TAPG_SEGMENTS"] = "1"
    yield
    for k in ENV_KEYS:
        os.environ.pop(k, None)


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/dwn128_tol1e-4.json has not been written yet "
                    "(tests/golden/make_dwn128_golden.py)")
    with open(GOLDEN) as f:
        return json.load(f)


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max()))


@pytest.mark.parametrize("schedule", ["bench", "autotuned"])
def test_dwn128_solve_to_tolerance_matches_oracle(schedule):
    """The headline solve (FP64, tolerance 1e-4, ~10^5 iterations) against the
    oracle's own full solve at the same step size."""
    g = _golden()
    P = ds.config_problem("dwn128")
    if schedule == "bench":
        os.environ.update(BENCH_SPEC)
    say("dwn128 to tol", g["tol"], "oracle iters", g["iters"], "schedule", schedule)
    with make_solver(P, gamma=g["gamma"], tol=g["tol"], max_iter=400_000,
                     check_every=100) as S:
        t = add_tree(S, P)
        if schedule == "autotuned":
            tapg.tapg_autotune(S.h, [t], 100)
        st, u0, res = S.solve(t, P.p, P.q)
        spec = tapg.tapg_schedule_spec(S.h, [t])
        u, x = S.primal(t)
        hist = tapg.tapg_residual_history(S.h, t, res.iters)
    nodes = np.asarray(g["sample_nodes"])
    h_or = np.asarray(g["res_every_1000"])
    n = min(len(h_or), len(hist) // 1000)
    h_gpu = np.asarray([hist[1000 * k + 999] for k in range(n)])
    dev = np.abs(h_gpu - h_or[:n]) / h_or[:n]
    say("schedule", spec, "iters", res.iters, "cost", repr(res.cost), "oracle", g["cost"],
        "u_root rel", _rel(u0, g["u_root"]), "max rel residual deviation", float(dev.max()),
        "at", int(dev.argmax()))
    assert st == tapg.TAPG_OK and res.converged
    assert abs(res.iters - g["iters"]) <= 1
    assert abs(res.cost - g["cost"]) <= 1e-6 * max(1.0, abs(g["cost"]))
    assert _rel(u0, g["u_root"]) <= 1e-6
    assert _rel(u[nodes], g["u_sample"]) <= 1e-6
    assert _rel(x[nodes], g["x_sample"]) <= 1e-6
    assert abs(res.viol_box - g["viol_box"]) <= 1e-6 and res.viol_eq <= 1e-9
    # the residual history follows the oracle's (the two sides round
    # differently, so the deviation may grow slowly over 10^5 iterations)
    assert dev[:20].max() <= 1e-6
    assert dev.max() <= 1e-3


@pytest.mark.parametrize("iters", [1000, 20000])
def test_dwn128_fixed_iteration_snapshots(iters):
    """The same solve stopped at fixed iteration counts on the way."""
    g = _golden()
    snap = g["snapshots"][str(iters)]
    P = ds.config_problem("dwn128")
    os.environ.update(BENCH_SPEC)
    say("dwn128 snapshot", iters)
    with make_solver(P, gamma=g["gamma"], tol=0.0, max_iter=iters, check_every=100) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
    say("cost", repr(res.cost), "oracle", snap["cost"], "u_root rel", _rel(u0, snap["u_root"]))
    assert res.iters == iters
    assert abs(res.cost - snap["cost"]) <= 1e-6 * max(1.0, abs(snap["cost"]))
    assert _rel(u0, snap["u_root"]) <= 1e-6
    assert abs(res.viol_box - snap["viol_box"]) <= 1e-6


def _batch64(indices):
    return [ds.config_problem("batch64", i) for i in indices]


@pytest.mark.parametrize("scan", ["0", "1"])
def test_batch64_trees_in_one_fp64_forest_match_oracle(scan):
    """Five full-size trees of the 64-tree configuration (K = 349 to 4,605)
    in one FP64 forest, in the segment form with projector factors and in the
    scan form: every tree's u, x and y element by element against its own
    oracle run."""
    os.environ["TAPG_SCAN"] = scan
    batch = _batch64([0, 1, 4, 5, 8])
    iters = 30
    say("batch64 x5 fp64", [P.tree.K for P in batch], "scan", scan)
    with make_solver(batch[0], gamma=0.0, tol=0.0, max_iter=iters, check_every=iters) as S:
        trees = [add_tree(S, P) for P in batch]
        st, u0s, res = S.batch_solve(trees, [P.p for P in batch], [P.q for P in batch])
        form = tapg.tapg_sweep_form(S.h, trees)
        out = [(S.primal(t), S.dual(t)) for t in trees]
    say("form", form)
    assert st == tapg.TAPG_OK
    assert form[0] == ("scan" if scan == "1" else "projector")
    assert len({P.tree.K for P in batch}) > 1
    for P, r, u0, ((u, x), y) in zip(batch, res, u0s, out):
        ref = O.apg(P, r.gamma, O.StageFactors(P.net, P.weights.W_u, P.tree), iters)
        assert r.iters == iters
        su, sx, sy = (max(1.0, np.abs(v).max()) for v in (ref.u, ref.x, ref.y))
        assert np.abs(u - ref.u).max() <= 1e-9 * su
        assert np.abs(x - ref.x).max() <= 1e-9 * sx
        assert np.abs(y - ref.y).max() <= 1e-9 * sy
        assert np.abs(u0 - ref.u[0]).max() <= 1e-9 * su
        J = O.primal_cost(P, ref.u, ref.x)
        assert abs(r.cost - J) <= 1e-6 * max(1.0, abs(J))


def test_dense_input_weight_at_full_size_matches_oracle():
    """A dense W_u (100 I plus a seeded rank-8 coupling): no stage factor is a
    projector, so the sweeps hold the dense 114 x 114 factor blocks (one per
    stage) in registers, in the segment form.  Three full-size trees of the
    64-tree configuration in one FP64 forest and the 128-scenario tree alone,
    element by element against the oracle after 30 iterations."""
    batch = _batch64([0, 1, 4])
    single = ds.config_problem("dwn128")
    W = ds.dense_input_weight(single.net.nu)
    for P in batch + [single]:
        P.weights.W_u = W
    iters = 30
    for group in (batch, [single]):
        say("dense W_u", [P.tree.K for P in group])
        with make_solver(group[0], gamma=0.0, tol=0.0, max_iter=iters, check_every=iters) as S:
            trees = [add_tree(S, P) for P in group]
            st, u0s, res = S.batch_solve(trees, [P.p for P in group], [P.q for P in group])
            form = tapg.tapg_sweep_form(S.h, trees)
            nb = tapg.tapg_factor_blocks(S.h, group[0].tree.N)
            out = [S.primal(t) for t in trees]
        say("form", form, "factor blocks", nb)
        assert st == tapg.TAPG_OK and form[0] == "segment"
        for P, r, (u, x) in zip(group, res, out):
            ref = O.apg(P, r.gamma, O.StageFactors(P.net, P.weights.W_u, P.tree), iters)
            su, sx = (max(1.0, np.abs(v).max()) for v in (ref.u, ref.x))
            assert r.iters == iters
            assert np.abs(u - ref.u).max() <= 1e-9 * su
            assert np.abs(x - ref.x).max() <= 1e-9 * sx
            J = O.primal_cost(P, ref.u, ref.x)
            assert abs(r.cost - J) <= 1e-6 * max(1.0, abs(J))


def test_batch64_whole_forest_equals_each_tree_alone():
    """All 64 trees (132,448 nodes) in one FP64 forest: each tree's iterate
    after a fixed number of iterations equals the tree solved alone."""
    batch = _batch64(range(64))
    iters = 20
    say("batch64 all", sum(P.tree.K for P in batch))
    with make_solver(batch[0], gamma=0.0, tol=0.0, max_iter=iters, check_every=iters) as S:
        trees = [add_tree(S, P) for P in batch]
        st, u0s, res = S.batch_solve(trees, [P.p for P in batch], [P.q for P in batch])
        got = [(S.primal(t), S.dual(t)) for t in trees]
        for t in trees:
            tapg.tapg_solver_forget(S.h, t)
        alone = []
        for t, P in zip(trees, batch):
            _, u01, r1 = S.solve(t, P.p, P.q)
            alone.append((r1, S.primal(t), S.dual(t), u01))
            tapg.tapg_solver_forget(S.h, t)
    assert st == tapg.TAPG_OK
    for r, u0, ((u, x), y), (r1, (u1, x1), y1, u01) in zip(res, u0s, got, alone):
        assert r.iters == r1.iters == iters
        assert abs(r.gamma - r1.gamma) <= 1e-15 * r1.gamma
        for a, b in ((u, u1), (x, x1), (y, y1), (u0, u01)):
            assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())
        assert abs(r.cost - r1.cost) <= 1e-10 * max(1.0, abs(r1.cost))


def _serve(S, trees, problems, sessions, gap_s=0.0, budget=1 << 36, max_batch=64, wait_ms=-1,
           ps=None):
    srv = tapg.tapg_server_create(S.h, budget, max_batch)
    try:
        tk = []
        for k, (t, P, s) in enumerate(zip(trees, problems, sessions)):
            p = P.p if ps is None else ps[k]
            tk.append(tapg.tapg_server_submit(srv, t, p, P.q, session=s))
            if gap_s:
                time.sleep(gap_s)
        out = [tapg.tapg_server_poll(srv, x, S.nu, wait_ms) for x in tk]
        stats = tapg.tapg_server_stats(srv)
    finally:
        tapg.tapg_server_destroy(srv)
    return out, stats


def test_served_full_size_requests_match_oracle_at_fixed_iterations():
    """Barcelona-sized requests of 32 to 512 scenarios served together (some
    arriving while others iterate), FP64, at a fixed iteration count: each
    ticket's cost and root input against its own oracle run."""
    probs = [ds.config_problem("serve", i) for i in range(5)]
    iters = 40
    say("served vs oracle", [P.tree.K for P in probs])
    with make_solver(probs[0], gamma=0.0, tol=0.0, max_iter=iters, check_every=10) as S:
        trees = [add_tree(S, P) for P in probs]
        out, stats = _serve(S, trees, probs, range(len(probs)), gap_s=0.002)
    say("forests formed", stats["batches"])
    for P, (st, u0, r, lat) in zip(probs, out):
        assert st == tapg.TAPG_OK and r.iters == iters
        ref = O.apg(P, r.gamma, O.StageFactors(P.net, P.weights.W_u, P.tree), iters)
        J = O.primal_cost(P, ref.u, ref.x)
        assert abs(r.cost - J) <= 1e-6 * max(1.0, abs(J))
        assert np.abs(u0 - ref.u[0]).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())


def test_served_full_size_same_result_alone_and_in_the_mix():
    """Barcelona-sized requests to the paper's tolerance (5e-2), FP64: each
    result is the same served in a mix (requests arriving while others
    iterate) as solved alone."""
    probs = [ds.config_problem("serve", i) for i in range(4)]
    kw = dict(gamma=0.0, tol=5e-2, max_iter=100_000, check_every=25)
    say("served mix", [P.tree.K for P in probs])
    with make_solver(probs[0], **kw) as S:
        trees = [add_tree(S, P) for P in probs]
        out, stats = _serve(S, trees, probs, range(len(probs)), gap_s=0.02)
    with make_solver(probs[0], **kw) as S:
        alone = []
        for P in probs:
            t = add_tree(S, P)
            _, u0, r = S.solve(t, P.p, P.q)
            alone.append((u0, r))
    say("forests", stats["batches"], "iters", [o[2].iters for o in out])
    assert stats["batches"] >= 2
    for (st, u0, r, lat), (u0a, ra) in zip(out, alone):
        assert st == tapg.TAPG_OK and r.converged
        assert r.iters == ra.iters
        assert np.abs(u0 - u0a).max() <= 1e-12 * max(1.0, np.abs(u0a).max())
        assert abs(r.cost - ra.cost) <= 1e-9 * max(1.0, abs(ra.cost))


FIXED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fixed_iterations.json")


def _fixed(name):
    if not os.path.exists(FIXED):
        pytest.skip("tests/golden/fixed_iterations.json has not been written yet "
                    "(tests/golden/make_fixed_golden.py)")
    with open(FIXED) as f:
        return json.load(f)[name]


@pytest.mark.parametrize("name", ["dwn128", "dwn2048"])
@pytest.mark.parametrize("precision", [tapg.TAPG_FP64, tapg.TAPG_FP32])
def test_fixed_iterations_fp64_and_fp32_against_oracle(name, precision):
    """The 2,429-node tree after 3,000 iterations and the 30,717-node tree after
    500 (residuals 1.6 and 28), at the oracle's step size: FP64
    sweeps to the FP64 bar; FP32 sweeps (FP64 factors, prox and residual) with
    their cost error against the FP64 oracle at the same iteration."""
    g = _fixed(name)
    P = ds.config_problem(name)
    nodes = np.asarray(g["sample_nodes"])
    say(name, "fixed", g["iters"], "precision", precision)
    with make_solver(P, gamma=g["gamma"], tol=0.0, max_iter=g["iters"], check_every=100,
                     precision=precision) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
    rel = abs(res.cost - g["cost"]) / max(1.0, abs(g["cost"]))
    du = _rel(u0, g["u_root"])
    say("cost", repr(res.cost), "oracle", g["cost"], "rel", rel, "u_root rel", du,
        "residual", res.primal_res, "oracle", g["final_res"])
    assert res.iters == g["iters"]
    if precision == tapg.TAPG_FP64:
        assert rel <= 1e-6 and du <= 1e-6
        assert _rel(u[nodes], g["u_sample"]) <= 1e-9 * 1e3
        assert _rel(x[nodes], g["x_sample"]) <= 1e-9 * 1e3
        assert abs(res.primal_res - g["final_res"]) <= 1e-6 * g["final_res"]
    else:
        # measured: 6.9e-4 after 3,000 iterations of the 2,429-node tree (the
        # FP32 and FP64 trajectories drift apart over the iterations), within
        # 1e-4 after 500 of the 30,717-node tree
        assert rel <= (1e-3 if name == "dwn128" else 1e-4)
        assert du <= 1e-2
