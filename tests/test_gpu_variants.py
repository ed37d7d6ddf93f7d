"""GPU: the duality gap on the boundary and the variants of the iteration
(Sec. 4.2-4.3) against the FP64 oracle.

* tapg_residuals' duality gap and dual objective of the returned dual, and of
  any dual set with tapg_set_dual, against ``oracle.split_gap``;
* the stop test on the gap (with the residual), at the oracle's iteration;
* theta = 2/(nu+2) and beta = 0 element by element;
* the averaged primal element by element.

Bars (FP64): iterates to 1e-9 of their scale; the gap and the dual objective
to 1e-9 of the size of their terms (both are sums of O(K) terms that cancel).
"""

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

ENV_KEYS = ("TAPG_LEVELS", "TAPG_PROJ", "TAPG_CHAIN", "TAPG_SCAN", "TAPG_FWD_GROUP")


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


def _scale_of_gap(P, y, gamma, f):
    """Size of the terms whose sum is the gap: |f(x')|, |<y, Hx'>|, |g*(y)|."""
    u, x = O.dual_gradient(P, y, f)
    hx = np.concatenate([x, x, u], axis=1)
    return max(1.0, abs(O.objective.smooth_cost(P, u)), float(np.sum(np.abs(y * hx))),
               abs(O.g_conj(P, y)))


@pytest.mark.parametrize("name,iters,scan", [("small", 37, True), ("small", 400, False),
                                            ("dwn128", 40, True), ("dwn128", 40, False)])
def test_dual_gap_of_the_returned_dual_matches_oracle(name, iters, scan):
    P = ds.config_problem(name)
    f = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, f, 60))
    os.environ["TAPG_SCAN"] = "1" if scan else "0"
    say("gap", name, iters, "scan", scan)
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=iters) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        r = tapg.tapg_residuals(S.h, t)
    ref = O.apg(P, gamma, f, iters)
    G, F = O.split_gap(P, ref.y, gamma, f)
    sc = _scale_of_gap(P, ref.y, gamma, f)
    say("G", r.dual_gap, G, "F", r.dual_obj, F, "scale", sc)
    assert np.isnan(res.dual_gap)  # the solve itself did not evaluate it
    assert abs(r.dual_gap - G) <= 1e-9 * sc
    assert abs(r.dual_obj - F) <= 1e-9 * sc
    assert r.iters == iters and abs(r.cost - res.cost) == 0.0


def test_dual_gap_of_a_set_dual_matches_oracle():
    """Any dual point given with tapg_set_dual: random points of dom g* on an
    irregular tree with a general A and a dense W_u (the evaluation uses the
    per-stage kernels and the dense factors)."""
    P = tiny_problem(N=6, irregular=True, seed=31, max_children=3, max_width=40)
    rng = np.random.default_rng(2)
    P.net.A = np.eye(4) + 0.05 * rng.standard_normal((4, 4))
    G0 = rng.standard_normal((6, 6))
    P.weights.W_u = G0 @ G0.T + 3 * np.eye(6)
    f = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 0.9 / O.lipschitz_power(P, f, 300)
    nx, K = P.net.nx, P.tree.K
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=5, check_every=5) as S:
        t = add_tree(S, P)
        S.solve(t, P.p, P.q)
        for k in range(4):
            y1 = rng.standard_normal((K, nx))
            y1 *= np.minimum(1.0, 0.9 * P.weights.W_x / np.linalg.norm(y1, axis=1))[:, None]
            y2 = -np.abs(rng.standard_normal((K, nx)))
            y2 *= np.minimum(1.0, 0.9 * P.weights.W_s / np.linalg.norm(y2, axis=1))[:, None]
            y3 = 10.0 ** (k - 2) * rng.standard_normal((K, P.net.nu))
            y = np.concatenate([y1, y2, y3], axis=1)
            tapg.tapg_set_dual(S.h, t, y)
            r = tapg.tapg_residuals(S.h, t)
            G, F = O.split_gap(P, y, gamma, f)
            sc = _scale_of_gap(P, y, gamma, f)
            say("set dual", k, r.dual_gap, G, r.dual_obj, F)
            assert abs(r.dual_gap - G) <= 1e-9 * sc
            assert abs(r.dual_obj - F) <= 1e-9 * sc


def test_dual_gap_fp32_sweeps():
    """FP32 sweeps: the gap is still evaluated in FP64, of the FP32 dual."""
    P = ds.config_problem("dwn128")
    f = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, f, 60))
    iters = 40
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=iters,
                     precision=tapg.TAPG_FP32) as S:
        t = add_tree(S, P)
        S.solve(t, P.p, P.q)
        y32 = S.dual(t)
        r = tapg.tapg_residuals(S.h, t)
    G, F = O.split_gap(P, y32, gamma, f)  # the oracle's gap of the GPU's own dual
    sc = _scale_of_gap(P, y32, gamma, f)
    say("fp32 gap", r.dual_gap, G, r.dual_obj, F)
    assert abs(r.dual_gap - G) <= 1e-9 * sc
    assert abs(r.dual_obj - F) <= 1e-9 * sc


@pytest.mark.parametrize("tol", [0.0, 1e-3])
def test_gap_stop_test_matches_oracle(tol):
    """gap_tol > 0: the solve stops at the first check (every 10 iterations)
    where |G| <= gap_tol (and the residual <= tol when tol > 0), at the
    oracle's iteration, returning that gap."""
    P = ds.config_problem("small")
    nf = O.NodeFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / O.lipschitz_dense(P, nf)
    check, gap_tol = 10, 1e-4
    seen = []

    def cb(nu, y_new, w, u, x):
        if (nu + 1) % check:
            return False
        res = float(np.max(np.abs(y_new - w))) / gamma
        G, F = O.split_gap(P, y_new, gamma, nf)
        seen.append((nu + 1, G, res))
        return abs(G) <= gap_tol and (tol <= 0 or res <= tol)

    ref = O.apg(P, gamma, nf, 20000, callback=cb)
    assert ref.converged
    margins = [abs(abs(G) - gap_tol) / gap_tol for _, G, _ in seen]
    assert min(margins) > 1e-6  # no check sits on the threshold
    with make_solver(P, gamma=gamma, tol=tol, max_iter=20000, check_every=check,
                     gap_tol=gap_tol) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
    say("gap stop", res.iters, ref.iters, res.dual_gap, seen[-1][1])
    assert st == tapg.TAPG_OK and res.converged
    assert res.iters == ref.iters
    assert abs(res.dual_gap - seen[-1][1]) <= 1e-9 * max(1.0, abs(res.dual_obj))
    assert np.abs(u - ref.u).max() <= 1e-9 * max(1.0, np.abs(ref.u).max())


@pytest.mark.parametrize("rule,name", [(tapg.TAPG_BETA_SIMPLE, "small"),
                                       (tapg.TAPG_BETA_ZERO, "small"),
                                       (tapg.TAPG_BETA_SIMPLE, "dwn128"),
                                       (tapg.TAPG_BETA_ZERO, "dwn128")])
@pytest.mark.parametrize("scan", [True, False])
def test_beta_rules_match_oracle(rule, name, scan):
    P = ds.config_problem(name)
    f = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, f, 60))
    iters = 300 if name == "small" else 40
    os.environ["TAPG_SCAN"] = "1" if scan else "0"
    rname = {tapg.TAPG_BETA_SIMPLE: "simple", tapg.TAPG_BETA_ZERO: "zero"}[rule]
    say("beta rule", rname, name, "scan", scan)
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=23,
                     beta_rule=rule) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
        y = S.dual(t)
        hist = tapg.tapg_residual_history(S.h, t, iters)
    ref = O.apg(P, gamma, f, iters, beta_rule=rname)
    for a, b in ((u, ref.u), (x, ref.x), (y, ref.y)):
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max())
    assert np.allclose(hist, ref.res_hist, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("rule,name,scan", [(tapg.TAPG_BETA_PAPER, "small", True),
                                            (tapg.TAPG_BETA_ZERO, "small", False),
                                            (tapg.TAPG_BETA_SIMPLE, "small", True),
                                            (tapg.TAPG_BETA_PAPER, "dwn128", True),
                                            (tapg.TAPG_BETA_PAPER, "dwn128", False)])
def test_averaged_primal_matches_oracle(rule, name, scan):
    P = ds.config_problem(name)
    f = O.StageFactors(P.net, P.weights.W_u, P.tree)
    gamma = 1.0 / (1.02 * O.lipschitz_power(P, f, 60))
    iters = 300 if name == "small" else 40
    os.environ["TAPG_SCAN"] = "1" if scan else "0"
    rname = {tapg.TAPG_BETA_PAPER: "paper", tapg.TAPG_BETA_SIMPLE: "simple",
             tapg.TAPG_BETA_ZERO: "zero"}[rule]
    say("averaged", rname, name, "scan", scan)
    with make_solver(P, gamma=gamma, tol=0.0, max_iter=iters, check_every=17,
                     beta_rule=rule, averaged_primal=True) as S:
        t = add_tree(S, P)
        st, u0, res = S.solve(t, P.p, P.q)
        u, x = S.primal(t)
        with pytest.raises(tapg.TapgError) as e:
            S.batch_solve([t], [P.p], [P.q])
        assert e.value.status == tapg.TAPG_EINVAL
    ref = O.apg(P, gamma, f, iters, beta_rule=rname, average=True)
    assert np.abs(u - ref.u_avg).max() <= 1e-9 * max(1.0, np.abs(ref.u_avg).max())
    assert np.abs(x - ref.x_avg).max() <= 1e-9 * max(1.0, np.abs(ref.x_avg).max())
    assert np.abs(u0 - ref.u_avg[0]).max() <= 1e-9 * max(1.0, np.abs(ref.u_avg).max())
    J = O.primal_cost(P, ref.u_avg, ref.x_avg)
    vb, ve = O.violations(P, ref.u_avg, ref.x_avg)
    assert abs(res.cost - J) <= 1e-6 * max(1.0, abs(J))
    assert abs(res.viol_box - vb) <= 1e-6 and res.viol_eq <= 1e-9
