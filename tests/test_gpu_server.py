"""GPU: the request server (worker thread, batched rounds, session warm
starts, HBM admission) against single-tree solves of the same requests."""

import os
import sys

import numpy as np
import pytest

from paper_1904_10548_amd import tapg

from gpu_helpers import add_tree, make_solver
from helpers import tiny_batch

pytestmark = pytest.mark.gpu

SHAPES = [(2, 4), (3, 3), ("irregular", 3, 20), (1, 1), (2, 8)]


@pytest.fixture(autouse=True)
def _default_schedule():
    os.environ.pop("TAPG_LEVELS", None)
    os.environ.pop("TAPG_PROJ", None)
    os.environ.pop("TAPG_CHAIN", None)
    os.environ.pop("TAPG_SCAN", None)
    os.environ.pop("TAPG_FWD_GROUP", None)
    os.environ["TAPG_USE_GRAPH"] = "1"
    os.environ["TAPG_SEGMENTS"] = "1"
    yield


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_server_matches_single_solves_with_session_warm_start():
    """Every tree is requested twice by its own session; the second request
    (new initial state) is warm started from the first, as a warm tapg_solve."""
    batch = tiny_batch(SHAPES, seed=31)
    kw = dict(gamma=0.0, tol=1e-6, max_iter=20000, check_every=50)
    nu = batch[0].net.nu
    p2 = [P.p + 0.2 for P in batch]
    say("server", [P.tree.K for P in batch])
    with make_solver(batch[0], **kw) as S:
        trees = [add_tree(S, P) for P in batch]
        srv = tapg.tapg_server_create(S.h, 1 << 34, 64)
        try:
            t1 = [tapg.tapg_server_submit(srv, t, P.p, P.q, session=k)
                  for k, (t, P) in enumerate(zip(trees, batch))]
            t2 = [tapg.tapg_server_submit(srv, t, p, P.q, session=k)
                  for k, (t, P, p) in enumerate(zip(trees, batch, p2))]
            with pytest.raises(tapg.TapgError):  # the server owns the solver
                S.solve(trees[0], batch[0].p, batch[0].q)
            first = [tapg.tapg_server_poll(srv, t, nu) for t in t1]
            second = [tapg.tapg_server_poll(srv, t, nu) for t in t2]
            stats = tapg.tapg_server_stats(srv)
        finally:
            tapg.tapg_server_destroy(srv)
        S.solve(trees[0], batch[0].p, batch[0].q)  # usable again
    assert stats["solved"] == 2 * len(batch) and stats["batches"] >= 2
    with make_solver(batch[0], **kw) as S:
        ref = []
        for P, p in zip(batch, p2):
            t = add_tree(S, P)
            _, u0a, ra = S.solve(t, P.p, P.q)
            _, u0b, rb = S.solve(t, p, P.q, warm_start=True)
            ref.append(((u0a, ra), (u0b, rb)))
    for (st1, u1, r1, l1), (st2, u2, r2, l2), ((u0a, ra), (u0b, rb)) in zip(first, second, ref):
        assert st1 == tapg.TAPG_OK and st2 == tapg.TAPG_OK
        assert l1 > 0 and l2 > 0
        assert r1.iters == ra.iters and r2.iters == rb.iters
        assert np.abs(u1 - u0a).max() <= 1e-12 * max(1.0, np.abs(u0a).max())
        assert np.abs(u2 - u0b).max() <= 1e-12 * max(1.0, np.abs(u0b).max())
        assert abs(r2.cost - rb.cost) <= 1e-9 * max(1.0, abs(rb.cost))


def test_server_continuous_admission_same_result_alone_and_in_the_mix():
    """Requests arrive while others are being iterated: they join the running
    set between chunks (the forest is re-formed, every running tree keeping
    its exact state), and each result equals the tree solved alone."""
    import time
    batch = tiny_batch(SHAPES, seed=41)
    kw = dict(gamma=0.0, tol=1e-9, max_iter=200000, check_every=20)
    nu = batch[0].net.nu
    say("server continuous", [P.tree.K for P in batch])
    with make_solver(batch[0], **kw) as S:
        trees = [add_tree(S, P) for P in batch]
        srv = tapg.tapg_server_create(S.h, 1 << 34, 64)
        try:
            tickets = []
            for k, (t, P) in enumerate(zip(trees, batch)):
                tickets.append(tapg.tapg_server_submit(srv, t, P.p, P.q, session=k))
                time.sleep(0.01)
            out = [tapg.tapg_server_poll(srv, t, nu) for t in tickets]
            stats = tapg.tapg_server_stats(srv)
        finally:
            tapg.tapg_server_destroy(srv)
    with make_solver(batch[0], **kw) as S:
        alone = []
        for P in batch:
            t = add_tree(S, P)
            _, u0, r = S.solve(t, P.p, P.q)
            alone.append((u0, r))
    say("forests formed", stats["batches"], "iterations", [o[2].iters for o in out])
    assert stats["batches"] >= 2
    for (st, u0, r, lat), (u0a, ra) in zip(out, alone):
        assert st == tapg.TAPG_OK and r.converged
        assert r.iters == ra.iters
        assert np.abs(u0 - u0a).max() <= 1e-12 * max(1.0, np.abs(u0a).max())
        assert abs(r.cost - ra.cost) <= 1e-9 * max(1.0, abs(ra.cost))


def test_server_rejects_requests_over_the_budget():
    batch = tiny_batch(SHAPES[:2], seed=3)
    nu = batch[0].net.nu
    with make_solver(batch[0], gamma=1e-3, tol=0.0, max_iter=10) as S:
        trees = [add_tree(S, P) for P in batch]
        srv = tapg.tapg_server_create(S.h, 1024, 8)  # 1 KiB: nothing fits
        try:
            tk = [tapg.tapg_server_submit(srv, t, P.p, P.q) for t, P in zip(trees, batch)]
            out = [tapg.tapg_server_poll(srv, t, nu) for t in tk]
        finally:
            tapg.tapg_server_destroy(srv)
    assert all(o[0] == tapg.TAPG_ENOMEM for o in out)


def test_solver_forget_releases_and_resolves():
    batch = tiny_batch(SHAPES[:2], seed=9)
    with make_solver(batch[0], gamma=0.0, tol=1e-6, max_iter=20000) as S:
        t = add_tree(S, batch[0])
        _, u0a, ra = S.solve(t, batch[0].p, batch[0].q)
        tapg.tapg_solver_forget(S.h, t)
        with pytest.raises(tapg.TapgError):
            S.primal(t)  # nothing held for the tree any more
        _, u0b, rb = S.solve(t, batch[0].p, batch[0].q)
    assert ra.iters == rb.iters and np.array_equal(u0a, u0b)


def test_server_setup_failure_completes_every_ticket():
    """A failure while a set of requests is set up (forced from the host for
    one ticket) completes every request of that set with the error instead of
    leaving its tickets pending; later requests are served normally."""
    batch = tiny_batch(SHAPES, seed=43)
    nu = batch[0].net.nu
    os.environ["TAPG_TEST_SERVER_SETUP_FAIL"] = "2"
    try:
        with make_solver(batch[0], gamma=0.0, tol=1e-6, max_iter=20000, check_every=20) as S:
            trees = [add_tree(S, P) for P in batch]
            srv = tapg.tapg_server_create(S.h, 1 << 34, 64)
            try:
                tk = [tapg.tapg_server_submit(srv, t, P.p, P.q, session=k)
                      for k, (t, P) in enumerate(zip(trees, batch))]
                first = [tapg.tapg_server_poll(srv, x, nu, wait_ms=60000) for x in tk]
                tk2 = [tapg.tapg_server_submit(srv, t, P.p, P.q, session=k)
                       for k, (t, P) in enumerate(zip(trees, batch))]
                second = [tapg.tapg_server_poll(srv, x, nu, wait_ms=60000) for x in tk2]
            finally:
                tapg.tapg_server_destroy(srv)
    finally:
        os.environ.pop("TAPG_TEST_SERVER_SETUP_FAIL", None)
    say("setup failure", [o[0] for o in first], [o[0] for o in second])
    assert all(o[0] != tapg.TAPG_ESTATE for o in first)  # nothing left pending
    assert first[1][0] == tapg.TAPG_EDEVICE
    assert all(o[0] == tapg.TAPG_OK and o[2].converged for o in second)


def test_server_warm_start_only_from_the_sessions_own_dual():
    """Two sessions request the same tree in turn: the tree keeps one dual, so
    a session's second request is warm started only if no other session solved
    the tree in between; otherwise it runs cold, with the cold result."""
    batch = tiny_batch(SHAPES[:1], seed=47)
    P = batch[0]
    nu = P.net.nu
    kw = dict(gamma=0.0, tol=1e-6, max_iter=20000, check_every=10)
    pA, pB = P.p, P.p + 0.3
    with make_solver(P, **kw) as S:
        t = add_tree(S, P)
        srv = tapg.tapg_server_create(S.h, 1 << 34, 64)
        try:
            seq = []
            for p, sess in ((pA, 1), (pB, 2), (pA, 1), (pA, 1)):
                x = tapg.tapg_server_submit(srv, t, p, P.q, session=sess)
                seq.append(tapg.tapg_server_poll(srv, x, nu, wait_ms=60000))
        finally:
            tapg.tapg_server_destroy(srv)
    with make_solver(P, **kw) as S:
        t = add_tree(S, P)
        _, u_cold, r_cold = S.solve(t, pA, P.q)
        _, u_warm, r_warm = S.solve(t, pA, P.q, warm_start=True)
    assert all(o[0] == tapg.TAPG_OK for o in seq)
    # third request: session 2 wrote the tree's dual in between -> cold
    assert seq[2][2].iters == r_cold.iters
    assert np.abs(seq[2][1] - u_cold).max() <= 1e-12 * max(1.0, np.abs(u_cold).max())
    # fourth request: the session's own dual -> warm, as a warm tapg_solve
    assert seq[3][2].iters == r_warm.iters and r_warm.iters < r_cold.iters
