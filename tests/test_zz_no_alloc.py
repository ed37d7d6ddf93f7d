"""GPU: the solve that allocates no device memory (tapg_solve_noalloc, every
buffer in the library's static scratch array) against tapg_solve on the same
trees: same iteration count, root input, primal and cost to the FP64 bar
(1e-9 of the scale; the two run differently associated sweeps).  Two calls in
a row, the second on a smaller tree, after a larger one left its contents in
the array."""

import os
import sys

import numpy as np
import pytest

import dwn_synth as ds
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


def _compare(S, t, P, tol_iters=0):
    K, nx, nu = P.tree.K, P.net.nx, P.net.nu
    st0, u00, r0 = S.solve(t, P.p, P.q)
    u_ref, x_ref = S.primal(t)
    st1, u01, u1, x1, r1 = tapg.tapg_solve_noalloc(S.h, t, P.p, P.q, K, nx, nu)
    say(P.name, "K", K, "iters", r0.iters, r1.iters, "cost", r0.cost, r1.cost)
    assert st1 == st0 and r1.converged == r0.converged
    # a run to a tolerance may stop one iteration apart (rounding order); a
    # fixed count is compared element by element
    assert abs(r1.iters - r0.iters) <= tol_iters
    if r1.iters != r0.iters:
        return
    su, sx = max(1.0, np.abs(u_ref).max()), max(1.0, np.abs(x_ref).max())
    assert np.abs(u01 - u00).max() <= 1e-9 * su
    assert np.abs(u1 - u_ref).max() <= 1e-9 * su
    assert np.abs(x1 - x_ref).max() <= 1e-9 * sx
    assert abs(r1.cost - r0.cost) <= 1e-9 * max(1.0, abs(r0.cost))
    assert abs(r1.viol_box - r0.viol_box) <= 1e-9 and r1.viol_eq <= 1e-9
    assert r1.gamma == r0.gamma and np.isnan(r1.dual_gap)


@pytest.mark.parametrize("tol,iters", [(0.0, 300), (1e-5, 20000)])
def test_noalloc_small_matches_tapg_solve(tol, iters):
    P = ds.config_problem("small")
    with make_solver(P, gamma=0.0, tol=tol, max_iter=iters, check_every=50) as S:
        t = add_tree(S, P)
        _compare(S, t, P, tol_iters=1 if tol > 0 else 0)


def test_noalloc_two_calls_second_smaller():
    """A 2,429-node tree, then a 349-node tree of the same network: the second
    call starts from what the first left in the scratch array."""
    big, small = ds.config_problem("batch64", 1), ds.config_problem("batch64", 5)
    assert big.tree.K == 2429 and small.tree.K == 349
    with make_solver(big, gamma=0.0, tol=0.0, max_iter=40, check_every=20) as S:
        tb, ts = add_tree(S, big), add_tree(S, small)
        nb = tapg.tapg_noalloc_bytes(S.h, tb)
        assert tapg.tapg_noalloc_bytes(S.h, ts) < nb <= tapg.NOALLOC_SCRATCH_BYTES
        _compare(S, tb, big)
        _compare(S, ts, small)


def test_noalloc_fp32_and_tolerance():
    P = ds.config_problem("batch64", 4)
    with make_solver(P, gamma=0.0, tol=5e-2, max_iter=100000, check_every=25,
                     precision=tapg.TAPG_FP32) as S:
        t = add_tree(S, P)
        st0, u00, r0 = S.solve(t, P.p, P.q)
        st1, u01, u1, x1, r1 = tapg.tapg_solve_noalloc(S.h, t, P.p, P.q, P.tree.K, P.net.nx,
                                                       P.net.nu)
    say("fp32", r0.iters, r1.iters, r0.cost, r1.cost)
    assert r1.converged and r0.converged
    # FP32 sweeps round differently in the two kernel forms: the stop may move
    assert abs(r1.iters - r0.iters) <= 0.02 * r0.iters + 25
    assert abs(r1.cost - r0.cost) <= 1e-3 * max(1.0, abs(r0.cost))


def test_noalloc_errors():
    """No step size without an estimate; a tree beyond the array's size is
    refused before anything runs; the averaged primal is refused."""
    P = ds.config_problem("small")
    with make_solver(P, gamma=0.0, tol=0.0, max_iter=10) as S:
        t = add_tree(S, P)
        with pytest.raises(tapg.TapgError) as e:
            tapg.tapg_solve_noalloc(S.h, t, P.p, P.q, P.tree.K, P.net.nx, P.net.nu)
        assert e.value.status == tapg.TAPG_EINVAL
        tapg.tapg_estimate_lipschitz(S.h, t, 100)
        st, *_ = tapg.tapg_solve_noalloc(S.h, t, P.p, P.q, P.tree.K, P.net.nx, P.net.nu)
        assert st == tapg.TAPG_OK
    with make_solver(P, gamma=1e-3, tol=0.0, max_iter=10, averaged_primal=True) as S:
        t = add_tree(S, P)
        with pytest.raises(tapg.TapgError) as e:
            tapg.tapg_solve_noalloc(S.h, t, P.p, P.q, P.tree.K, P.net.nx, P.net.nu)
        assert e.value.status == tapg.TAPG_EINVAL
    L = ds.config_problem("dwn2048")
    with make_solver(L, gamma=1e-6, tol=0.0, max_iter=10) as S:
        t = add_tree(S, L)
        assert tapg.tapg_noalloc_bytes(S.h, t) > tapg.NOALLOC_SCRATCH_BYTES
        with pytest.raises(tapg.TapgError) as e:
            tapg.tapg_solve_noalloc(S.h, t, L.p, L.q, L.tree.K, L.net.nx, L.net.nu)
        assert e.value.status == tapg.TAPG_ENOMEM
