"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Bars (FP64): primal iterates and duals agree elementwise to 1e-9 of their
scale, cost to 1e-6 relative and constraint violations to 1e-6 (the stated
accuracy of the method's FP64 implementation); rounding-order differences
between the two sides are ~1e-13 here, so the bars leave margin without
hiding a wrong term.  FP32 sweeps: cost within 1e-4 relative of the FP64
oracle.
"""

import functools
import os
import sys

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O
from paper_1904_10548_amd import tapg

from gpu_helpers import add_tree, make_solver
from helpers import tiny_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_schedule():
    _schedule_env()
    yield
    _schedule_env()


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _oracle_run(P, gamma, iters, tol=None, factors=None):
    f = factors or O.StageFactors(P.net, P.weights.W_u, P.tree)
    return O.apg(P, gamma, f, iters, tol=tol)


def _schedule_env(graph=True, segments=True, levels=None, proj=True, chain=False, scan=True,
                  fwd_group=0):
    os.environ["TAPG_USE_GRAPH"] = "1" if graph else "0"
    os.environ["TAPG_SEGMENTS"] = "1" if segments else "0"
    os.environ["TAPG_PROJ"] = "1" if proj else "0"
    os.environ["TAPG_CHAIN"] = "1" if chain else "0"
    os.environ["TAPG_SCAN"] = "1" if scan else "0"
    if fwd_group:
        os.environ["TAPG_FWD_GROUP"] = str(fwd_group)
    else:
        os.environ.pop("TAPG_FWD_GROUP", None)
    if levels:
        os.environ["TAPG_LEVELS"] = levels
    else:
        os.environ.pop("TAPG_LEVELS", None)


def _compare_fixed(P, gamma, iters, precision=tapg.TAPG_FP64, check_every=50, graph=True,
                   segments=True, levels=None, proj=True, chain=False, scan=True, fwd_group=0):
    _schedule_env(graph, segments, levels, proj, chain, scan, fwd_group)
    say(P.name, "K", P.tree.K, "iters", iters, "prec", precision, "graph", graph,
        "segments", segments, "levels", levels, "proj", proj, "chain", chain, "scan", scan,
        "fwd_group", fwd_group)
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=check_every,
                     precision=precision) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
        y = S.dual(t)
        hist = tapg.tapg_residual_history(S.h, t, iters)
    ref = _oracle_run(P, gamma, iters)
    return st, u0, res, u, x, y, hist, ref


def _assert_fp64_parity(P, res, u, x, y, hist, ref, iters):
    assert res.iters == iters
    su = max(1.0, np.abs(ref.u).max())
    sx = max(1.0, np.abs(ref.x).max())
    sy = max(1.0, np.abs(ref.y).max())
    assert np.abs(u - ref.u).max() <= 1e-9 * su
    assert np.abs(x - ref.x).max() <= 1e-9 * sx
    assert np.abs(y - ref.y).max() <= 1e-9 * sy
    J = O.primal_cost(P, ref.u, ref.x)
    vb, ve = O.violations(P, ref.u, ref.x)
    assert abs(res.cost - J) <= 1e-6 * max(1.0, abs(J))
    assert abs(res.viol_box - vb) <= 1e-6
    assert res.viol_eq <= 1e-9 and ve <= 1e-9
    rh = np.asarray(ref.res_hist)
    assert np.allclose(hist, rh, rtol=1e-7, atol=1e-12)
    assert abs(res.primal_res - rh[-1]) <= 1e-7 * rh[-1] + 1e-12


@pytest.mark.parametrize("graph,segments,chain,scan", [(True, True, False, True),
                                                      (False, True, False, True),
                                                      (True, True, True, False),
                                                      (True, True, False, False),
                                                      (True, False, False, False)])
def test_small_500_iterations_fp64(graph, segments, chain, scan):
    """The small configuration at exactly 500 iterations (no early stop):
    scan-form and segment-form level launches with and without graphs, the
    persistent iteration, per-stage kernels."""
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / O.lipschitz_dense(P, nf)
    st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 500, graph=graph,
                                                     segments=segments, chain=chain, scan=scan)
    assert st == tapg.TAPG_OK
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 500)
    assert np.abs(u0 - ref.u[0]).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())


@pytest.mark.parametrize("scan,fwd_group", [(True, 0), (True, 1), (True, 4), (False, 0)])
def test_wide_ragged_tree_scan_and_segment_fp64(scan, fwd_group):
    """Irregular branching up to 40 children per node: the scan form (children
    of a workgroup's last stage in the level below, ragged node ranges; the
    forward launch on the bottom level's workgroups or on groups of 1 or 4
    leaves, each walking its ancestors) and the segment form."""
    P = tiny_problem(N=7, irregular=True, seed=12, max_children=40, max_width=3000)
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 0.9 / O.lipschitz_power(P, sf, 200)
    st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 80, scan=scan, fwd_group=fwd_group)
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 80)


@pytest.mark.parametrize("segments", [True, False])
def test_irregular_tree_general_A_Wu_fp64(segments):
    """Irregular branching, non-identity A and dense W_u (generic paths)."""
    P = tiny_problem(N=6, irregular=True, seed=31, max_children=3, max_width=40)
    rng = np.random.default_rng(2)
    P.net.A = np.eye(4) + 0.05 * rng.standard_normal((4, 4))
    G = rng.standard_normal((6, 6))
    P.weights.W_u = G @ G.T + 3 * np.eye(6)
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 0.9 / O.lipschitz_power(P, sf, 300)
    st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 300, segments=segments)
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 300)


def test_wide_ragged_tree_fp64_and_fp32():
    """Stages wide enough for multi-node tiles, with ragged last tiles."""
    P = tiny_problem(N=5, irregular=True, seed=8, max_children=40, max_width=2500)
    widths = P.tree.nodes_per_stage
    assert widths.max() >= 1024 and any(w % 8 for w in widths)
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 0.9 / O.lipschitz_power(P, sf, 200)
    st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 60)
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 60)
    st, u0, r32, u, x, y, hist, ref = _compare_fixed(P, gamma, 60, precision=tapg.TAPG_FP32)
    J = O.primal_cost(P, ref.u, ref.x)
    assert abs(r32.cost - J) <= 1e-4 * max(1.0, abs(J))


@pytest.mark.parametrize("levels,fp32,proj,chain,scan,fwd_group",
                         [(None, False, True, False, True, 1),
                          (None, True, True, False, True, 2),
                          (None, False, True, False, True, 0),
                          (None, False, True, True, False, 0),
                          (None, False, True, False, False, 0),
                          (None, False, False, False, False, 0),
                          ("0:1,2:2,4:1", False, True, False, True, 0),
                          ("0:1,2:2,4:1", False, True, True, False, 0),
                          ("0:1,2:1,4:1,6:2,15:4", False, True, False, True, 0),
                          ("0:1,2:1,4:1,6:2,15:4", False, True, False, True, 1),
                          ("0:1,2:1,4:1,6:1", False, True, False, True, 0),
                          ("0:1,2:1,4:1,6:1", False, True, False, False, 0),
                          ("0:1,1:1,3:2,5:2", True, True, False, True, 0),
                          ("0:1,1:1,3:2,5:2", True, True, True, False, 0),
                          ("0:1,1:1,3:2,5:2", True, False, False, False, 0)])
def test_dwn128_fixed_iterations(levels, fp32, proj, chain, scan, fwd_group):
    """Full-size network and tree (K = 2429): 40 iterations, every element;
    planned schedule and forced multi-level / grouped schedules, in scan form,
    segment form and as one persistent launch."""
    P = ds.config_problem("dwn128")
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, sf, 60))
    if fp32:  # FP32 sweeps on a five-level schedule with groups of two
        st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 40, check_every=40,
                                                         precision=tapg.TAPG_FP32, levels=levels,
                                                         proj=proj, chain=chain, scan=scan,
                                                         fwd_group=fwd_group)
        J = O.primal_cost(P, ref.u, ref.x)
        assert abs(res.cost - J) <= 1e-4 * max(1.0, abs(J))
        return
    st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 40, check_every=40, levels=levels,
                                                     proj=proj, chain=chain, scan=scan,
                                                     fwd_group=fwd_group)
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 40)


@functools.lru_cache(maxsize=1)
def _dwn2048_reference():
    """The oracle's 30 iterations on the 2,048-scenario tree (computed once)."""
    P = ds.config_problem("dwn2048")
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, sf, 40))
    iters = 30
    return P, gamma, iters, O.apg(P, gamma, sf, iters)


@pytest.mark.parametrize("precision,scan", [(tapg.TAPG_FP64, True), (tapg.TAPG_FP64, False),
                                            (tapg.TAPG_FP32, True), (tapg.TAPG_FP32, False)])
def test_dwn2048_against_oracle(precision, scan):
    """The 2,048-scenario tree (K = 30,717), 30 iterations, in the scan form and
    in the segment form with projector factors (the autotuner's choices for this
    tree in FP32 and FP64): in FP64 u, x and y element by element against the
    oracle's, cost within 1e-6; with FP32 sweeps (FP64 factors and residuals)
    cost and root input within 1e-4 of the FP64 oracle's."""
    P, gamma, iters, ref = _dwn2048_reference()
    _schedule_env(scan=scan)
    say("dwn2048", P.tree.K, "prec", precision, "scan", scan)
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=iters,
                     precision=precision) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        form = tapg.tapg_sweep_form(S.h, [t])
        if precision == tapg.TAPG_FP64:
            u, x = S.primal(t)
            y = S.dual(t)
            hist = tapg.tapg_residual_history(S.h, t, iters)
    assert form[0] == ("scan" if scan else "projector")
    J = O.primal_cost(P, ref.u, ref.x)
    rel = abs(res.cost - J) / max(1.0, abs(J))
    du = np.abs(u0 - ref.u[0]).max() / max(1.0, np.abs(ref.u[0]).max())
    say("dwn2048 cost", res.cost, "oracle", J, "rel", rel, "root du", du)
    if precision == tapg.TAPG_FP64:
        _assert_fp64_parity(P, res, u, x, y, hist, ref, iters)
        return
    assert res.iters == iters and rel <= 1e-4 and du <= 1e-3


def test_small_converged_matches_oracle_iteration_count():
    """Run to a tolerance: same stopping iteration and result as the oracle."""
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / O.lipschitz_dense(P, nf)
    tol = 1e-5
    ref = _oracle_run(P, gamma, 20000, tol=tol, factors=nf)
    say("small converged", ref.iters)
    with make_solver(P, gamma=gamma, tol=tol, max_iter=20000, check_every=64) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
    assert st == tapg.TAPG_OK and res.converged
    assert abs(res.iters - ref.iters) <= 1
    J = O.primal_cost(P, ref.u, ref.x)
    assert abs(res.cost - J) <= 1e-6 * max(1.0, abs(J))
    if res.iters == ref.iters:
        assert np.abs(u - ref.u).max() <= 1e-8


@pytest.mark.parametrize("scan,graph,check_every", [(True, True, 7), (False, True, 7),
                                                    (True, False, 5), (True, True, 1)])
def test_odd_chunks_and_stop_inside_a_chunk(scan, graph, check_every):
    """Iterations in runs of odd length: the level launches end each iteration
    in the next one's first backward launch (two control blocks used in turn)
    and a run with one small launch.  103 fixed iterations (the last run cut
    by max_iter) match the oracle element by element with the whole residual
    history, and a run to a tolerance stops at the oracle's iteration."""
    P = tiny_problem(N=7, irregular=True, seed=12, max_children=40, max_width=3000)
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 0.9 / O.lipschitz_power(P, sf, 200)
    st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 103, check_every=check_every,
                                                     graph=graph, scan=scan)
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 103)
    P = tiny_problem(N=6, irregular=True, seed=5, max_children=4, max_width=60)
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 0.9 / O.lipschitz_power(P, sf, 200)
    tol = 1e-3
    ref2 = _oracle_run(P, gamma, 5000, tol=tol, factors=sf)
    assert ref2.converged  # 1,516 iterations
    with make_solver(P, gamma=gamma, tol=tol, max_iter=5000, check_every=check_every) as S:
        t = add_tree(S, P)
        st, u0, r2 = S.solve(t, P.p, P.q)
        h2 = tapg.tapg_residual_history(S.h, t, r2.iters)
    say("stop", r2.iters, "oracle", ref2.iters)
    assert st == tapg.TAPG_OK and r2.converged and r2.iters == ref2.iters
    assert np.allclose(h2, np.asarray(ref2.res_hist), rtol=1e-7, atol=1e-12)


def test_factor_step_matches_oracle_stage_factors():
    P = ds.config_problem("dwn128")
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    with make_solver(P, gamma=1e-3, tol=0.0, max_iter=1) as S:
        for s in [0, 11, 23]:
            F, Kb, G = tapg.tapg_get_factors(S.h, s, P.net.nu)
            assert np.abs(F - sf.Fbar[s]).max() <= 1e-11 * np.abs(sf.Fbar[s]).max()
            assert np.abs(Kb - sf.Kbar[s]).max() <= 1e-11 * max(1.0, np.abs(sf.Kbar[s]).max())
            assert np.abs(G - sf.Gbar[s]).max() <= 1e-11 * max(1.0, np.abs(sf.Gbar[s]).max())


def test_factor_blocks_shared_when_equal():
    """Stages whose factors agree to rounding share one block: one block for
    W_u = w I (Fbar_s = Pi / w at every stage); with a dense W_u every stage's
    block equals its own factor to 16 ulp."""
    P = ds.config_problem("dwn128")
    with make_solver(P, gamma=1e-3, tol=0.0, max_iter=1) as S:
        fid, nb = tapg.tapg_factor_blocks(S.h, P.tree.N)
    assert nb == 1 and np.all(fid == P.tree.N - 1)
    Pg = tiny_problem(N=9, b1=3, S=8, seed=5)
    rng = np.random.default_rng(7)
    M = rng.standard_normal((Pg.net.nu, Pg.net.nu))
    Pg.weights.W_u = M @ M.T + Pg.net.nu * np.eye(Pg.net.nu)
    sf = O.StageFactors(Pg.net, Pg.weights.W_u, Pg.tree)
    with make_solver(Pg, gamma=1e-3, tol=0.0, max_iter=1) as S:
        fid, nb = tapg.tapg_factor_blocks(S.h, Pg.tree.N)
    N = Pg.tree.N
    assert fid[N - 1] == N - 1 and 1 <= nb <= N
    assert len(set(fid.tolist())) == nb
    for s in range(N):
        assert s <= fid[s] and fid[fid[s]] == fid[s]
        F, R = sf.Fbar[s], sf.Fbar[fid[s]]
        assert np.abs(F - R).max() <= 16 * 2.3e-16 * np.abs(R).max() + 1e-15


def test_power_iteration_lipschitz():
    """Device power iteration approaches the largest eigenvalue from below."""
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    L = O.lipschitz_dense(P, nf)
    with make_solver(P, gamma=1e-3, tol=0.0, max_iter=1) as S:
        t = add_tree(S, P)
        Lg = tapg.tapg_estimate_lipschitz(S.h, t, 400)
    assert Lg <= L * (1 + 1e-10)
    assert Lg >= L * (1 - 1e-6)


def test_auto_gamma_and_warm_start():
    """gamma = 0 selects 1/(1.02 L); a warm-started re-solve of the same data
    needs fewer iterations and returns the same answer within the tolerance;
    get/set dual round-trips."""
    P = ds.config_problem("small")
    with make_solver(P, gamma=0.0, tol=1e-4, max_iter=20000, check_every=50) as S:
        t = add_tree(S, P)
        st, u0, r1 = S.solve(t, P.p, P.q)
        nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
        L = O.lipschitz_dense(P, nf)
        assert abs(r1.gamma - 1.0 / (1.02 * L)) <= 1e-6 * r1.gamma
        y1 = S.dual(t)
        st, u0b, r2 = S.solve(t, P.p, P.q, warm_start=True)
        assert r2.iters < r1.iters
        assert abs(r2.cost - r1.cost) <= 1e-3 * max(1.0, abs(r1.cost))
        tapg.tapg_set_dual(S.h, t, y1)
        np.testing.assert_array_equal(S.dual(t), y1)


def test_deterministic_repeat():
    P = ds.config_problem("dwn128")
    out = []
    with make_solver(P, gamma=1e-7, tol=0.0, max_iter=30, check_every=30) as S:
        t = add_tree(S, P)
        for _ in range(2):
            S.solve(t, P.p, P.q)
            u, x = S.primal(t)
            out.append((u, x, S.dual(t)))
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)


def test_edge_cases_single_node_and_chain():
    """N = 1 (root only) and a single scenario chain."""
    for P in [tiny_problem(N=1, b1=1, S=1, seed=2), tiny_problem(N=7, b1=1, S=1, seed=2)]:
        sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
        gamma = 1.0 / (1.02 * O.lipschitz_power(P, sf, 200))
        st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 120)
        _assert_fp64_parity(P, res, u, x, y, hist, ref, 120)


def test_interior_problem_stops_after_one_iteration():
    P = tiny_problem(N=4, b1=2, S=4, seed=9)
    d0 = P.data.demand[0]
    P.data.demand[:] = d0
    P.data.price[:] = 0.0
    P.weights.alpha0[:] = 0.0
    from dwn_synth.generate import steady_input
    P.q = steady_input(P.net, d0) + 0.3 * np.array([k == "src_tank" for k in P.net.kind])
    with make_solver(P, gamma=1e-2, tol=1e-9, max_iter=100, check_every=10) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
    u_k, x_k = O.dual_gradient_kkt(P, np.zeros((P.tree.K, 14)))
    assert res.iters == 1 and res.converged and res.primal_res <= 1e-12
    assert np.abs(u - u_k).max() <= 1e-10


def test_fp32_sweeps_small_cost_error():
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / O.lipschitz_dense(P, nf)
    st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 500, precision=tapg.TAPG_FP32)
    J = O.primal_cost(P, ref.u, ref.x)
    assert abs(res.cost - J) <= 1e-4 * max(1.0, abs(J))
    assert res.viol_eq <= 1e-4


def test_forward_groupings_bit_identical():
    """The scan form's forward launch on the bottom level's workgroups or on
    groups of 1, 2 or 4 leaves computes every node in the same order (shared
    ancestors are recomputed, not re-associated): the iterates agree bit for
    bit."""
    P = ds.config_problem("dwn128")
    gamma = 1e-6
    out = {}
    for fg in (0, 1, 2, 4):
        _schedule_env(scan=True, fwd_group=fg)
        say("dwn128 fwd group", fg)
        with make_solver(P, gamma=gamma, tol=0.0, max_iter=30, check_every=30) as S:
            t = add_tree(S, P)
            st, u0, res = S.solve(t, P.p, P.q)
            u, x = S.primal(t)
            out[fg] = (u, x, S.dual(t), res.primal_res)
    os.environ.pop("TAPG_FWD_GROUP", None)
    for fg in (1, 2, 4):
        for a, b in zip(out[0], out[fg]):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_max_iter_before_tolerance_is_enotconv():
    """A tolerance the iteration cannot reach within max_iter: TAPG_ENOTCONV,
    with the iterate of the last iteration (the same as a fixed-count run), for
    a single tree and in a batch."""
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / O.lipschitz_dense(P, nf)
    iters = 57
    ref = _oracle_run(P, gamma, iters, factors=nf)
    with make_solver(P, gamma=gamma, tol=1e-14, max_iter=iters, check_every=10) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
        stb, u0b, rb = S.batch_solve([t], [P.p], [P.q])
    assert st == tapg.TAPG_ENOTCONV and stb == tapg.TAPG_ENOTCONV
    assert res.iters == iters and not res.converged and res.primal_res > 1e-14
    assert rb[0].iters == iters and not rb[0].converged
    assert np.abs(u - ref.u).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())
    assert np.abs(u0b - u0).max() <= 1e-12 * max(1.0, np.abs(u0).max())


def test_diverging_step_size_is_enumeric():
    """A step size 100 times 1/L makes the dual iterates grow until they are
    no longer finite (the oracle's run with this step size does so at
    iteration 373; every kernel still completes): the solve returns
    TAPG_ENUMERIC, a single tree and a batch alike, and the solver stays
    usable."""
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    L = O.lipschitz_dense(P, nf)
    with np.errstate(all="ignore"):
        ref = _oracle_run(P, 100.0 / L, 3000, tol=1e-300, factors=nf)
    bad = np.flatnonzero(~np.isfinite(np.asarray(ref.res_hist)))
    assert bad.size and bad[0] < 1000
    with make_solver(P, gamma=100.0 / L, tol=1e-6, max_iter=3000, check_every=50) as S:
        t = add_tree(S, P)
        with pytest.raises(tapg.TapgError) as e:
            S.solve(t, P.p, P.q)
        assert e.value.status == tapg.TAPG_ENUMERIC
        with pytest.raises(tapg.TapgError) as e:
            S.batch_solve([t], [P.p], [P.q])
        assert e.value.status == tapg.TAPG_ENUMERIC
        r = tapg.tapg_residuals(S.h, t)
        assert r.iters <= bad[0] + 2 and not r.converged
        assert np.isnan(r.dual_gap)  # a diverged dual has no gap
    with make_solver(P, gamma=1.0 / L, tol=1e-6, max_iter=20000, check_every=50) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        assert st == tapg.TAPG_OK and res.converged


def test_forward_group_out_of_range_is_rejected():
    """The scan form's forward launch holds at most 4 leaves per workgroup:
    other groupings are refused with TAPG_EINVAL instead of being run."""
    P = ds.config_problem("dwn128")
    for fg in ("3", "5", "8"):
        _schedule_env(scan=True)
        os.environ["TAPG_FWD_GROUP"] = fg
        with make_solver(P, gamma=1e-6, tol=0.0, max_iter=2, check_every=2) as S:
            t = add_tree(S, P)
            with pytest.raises(tapg.TapgError) as e:
                S.solve(t, P.p, P.q)
            assert e.value.status == tapg.TAPG_EINVAL
    os.environ.pop("TAPG_FWD_GROUP", None)


@pytest.mark.parametrize("scan", [True, False])
def test_fp32_sweeps_residual_is_fp64(scan):
    """With FP32 sweeps the prox and the stop test run in FP64 on the widened
    FP32 inputs: one iteration from a dual of size ~1 (given with
    tapg_set_dual, FP32-representable) on the 2,429-node tree, whose step size
    (~1.4e-6) would amplify an FP32 dual update's rounding (ulp(1)/gamma ~ 0.04)
    into the residual, gives the oracle's FP64 residual to 1e-4."""
    P = ds.config_problem("dwn128")
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, sf, 60))
    rng = np.random.default_rng(5)
    nx, nu, K = P.net.nx, P.net.nu, P.tree.K
    y1 = rng.standard_normal((K, nx))
    y1 *= np.minimum(1.0, 0.9 * P.weights.W_x / np.linalg.norm(y1, axis=1))[:, None]
    y2 = -np.abs(rng.standard_normal((K, nx)))
    y2 *= np.minimum(1.0, 0.9 * P.weights.W_s / np.linalg.norm(y2, axis=1))[:, None]
    y3 = rng.standard_normal((K, nu))
    y = np.concatenate([y1, y2, y3], axis=1).astype(np.float32).astype(np.float64)
    _schedule_env(scan=scan)
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=1, check_every=1,
                     precision=tapg.TAPG_FP32) as S:
        t = add_tree(S, P)
        S.solve(t, P.p, P.q)
        tapg.tapg_set_dual(S.h, t, y)
        st, u0, res = S.solve(t, P.p, P.q, warm_start=True)
    ref = O.apg(P, gamma, sf, 1, y0=y)
    say("fp32 residual", res.primal_res, "oracle", ref.res_hist[0], "gamma", gamma)
    assert res.iters == 1
    assert abs(res.primal_res - ref.res_hist[0]) <= 1e-4 * max(1.0, ref.res_hist[0])


@pytest.mark.parametrize("levels", [None, "0:1,2:1,4:1,6:1", "0:1,2:2,4:1", "0:1,1:1,3:2,5:2",
                                    "0:1,2:1,4:1,6:2,15:4"])
@pytest.mark.parametrize("fp32", [False, True])
def test_light_upper_levels_dwn128(levels, fp32):
    """Light upper levels (TAPG_TOP=1): the levels above the bottom one sum
    local parts that the bottom level's launch computed for their nodes; the
    same iterates as the oracle, element by element (FP64), or its cost to
    1e-4 (FP32), on several level sets."""
    P = ds.config_problem("dwn128")
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, sf, 60))
    os.environ["TAPG_TOP"] = "1"
    try:
        prec = tapg.TAPG_FP32 if fp32 else tapg.TAPG_FP64
        st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 40, check_every=13,
                                                         precision=prec, levels=levels)
    finally:
        os.environ.pop("TAPG_TOP", None)
    if fp32:
        J = O.primal_cost(P, ref.u, ref.x)
        assert abs(res.cost - J) <= 1e-4 * max(1.0, abs(J))
        return
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 40)


@pytest.mark.parametrize("seed,fwd_group", [(12, 0), (12, 1), (5, 0), (5, 1)])
def test_light_upper_levels_irregular(seed, fwd_group):
    """Light upper levels on irregular trees (up to 40 children per node,
    ragged node ranges), with the forward launch on the bottom level's
    workgroups or on single leaves."""
    P = tiny_problem(N=7, irregular=True, seed=seed, max_children=40, max_width=3000)
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 0.9 / O.lipschitz_power(P, sf, 200)
    os.environ["TAPG_TOP"] = "1"
    try:
        st, u0, res, u, x, y, hist, ref = _compare_fixed(P, gamma, 80, check_every=9,
                                                         fwd_group=fwd_group)
    finally:
        os.environ.pop("TAPG_TOP", None)
    _assert_fp64_parity(P, res, u, x, y, hist, ref, 80)



def test_light_upper_levels_power_iteration():
    """The power iteration (the linear part of the dual gradient, no data)
    also runs on light upper levels: the same Lipschitz estimate as with the
    full kernels, from the same start and number of steps."""
    P = ds.config_problem("dwn128")
    out = {}
    for top in ("0", "1"):
        _schedule_env(scan=True, levels="0:1,2:1,4:1,6:1")
        os.environ["TAPG_TOP"] = top
        try:
            with make_solver(P, gamma=1e-6, tol=0.0, max_iter=1) as S:
                t = add_tree(S, P)
                out[top] = tapg.tapg_estimate_lipschitz(S.h, t, 60)
        finally:
            os.environ.pop("TAPG_TOP", None)
    say("power", out)
    assert abs(out["1"] - out["0"]) <= 1e-9 * out["0"]
