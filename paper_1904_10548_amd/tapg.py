"""ctypes binding of the tapg C ABI (``include/tapg.h``).

Functions carry the C names and only marshal arguments: numpy arrays become
float64/int32 pointers, status codes become :class:`TapgError`.  Every
computation runs inside ``libtapg.so`` (HIP kernels for gfx950 and the
library's host code); there is no Python or CPU fallback: if the library is
missing, :func:`lib` raises.

:class:`Solver` is a small owner object over the handles for tests and
benchmarks.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# TAPG_LIBRARY selects another build of the same library (e.g. an experiment).
LIB_PATH = os.environ.get("TAPG_LIBRARY") or os.path.join(_PKG, "libtapg.so")

TAPG_OK = 0
TAPG_ENOTCONV = 1
TAPG_EINVAL = -1
TAPG_EDIM = -2
TAPG_ENOMEM = -3
TAPG_EDEVICE = -4
TAPG_ESTATE = -5
TAPG_ENUMERIC = -6
TAPG_FP64 = 0
TAPG_FP32 = 1
TAPG_BETA_PAPER = 0
TAPG_BETA_SIMPLE = 1
TAPG_BETA_ZERO = 2

EXPORTED = [
    "tapg_network_create", "tapg_network_destroy", "tapg_tree_create", "tapg_tree_set_data",
    "tapg_tree_num_nodes", "tapg_tree_destroy", "tapg_solver_create", "tapg_solver_destroy",
    "tapg_factor_step", "tapg_get_factors", "tapg_factor_blocks", "tapg_solve", "tapg_batch_solve", "tapg_get_primal", "tapg_get_dual",
    "tapg_set_dual", "tapg_residual_history", "tapg_residuals", "tapg_estimate_lipschitz",
    "tapg_kernel_timing", "tapg_kernel_times", "tapg_plan_schedule", "tapg_autotune", "tapg_sweep_form",
    "tapg_schedule_spec", "tapg_event_pair_overhead",
    "tapg_solver_forget", "tapg_solve_noalloc", "tapg_noalloc_bytes", "tapg_closed_loop", "tapg_tree_build",
    "tapg_server_create", "tapg_server_submit", "tapg_server_poll", "tapg_server_stats", "tapg_server_timing",
    "tapg_server_destroy", "tapg_last_error", "tapg_version",
    "tapg_tree_dims", "tapg_network_dims", "tapg_network_from_json", "tapg_tree_from_json",
    "tapg_tree_data_from_json", "tapg_config_from_json", "tapg_state_from_json",
    "tapg_control_output_write",
]


class TapgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"tapg status {status}: {message}")
        self.status = status


class TapgConfig(ctypes.Structure):
    _fields_ = [
        ("W_alpha", ctypes.c_double),
        ("W_s", ctypes.c_double),
        ("W_x", ctypes.c_double),
        ("alpha0", ctypes.POINTER(ctypes.c_double)),
        ("c_energy", ctypes.POINTER(ctypes.c_double)),
        ("W_u", ctypes.POINTER(ctypes.c_double)),
        ("gamma", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("power_iters", ctypes.c_int),
        ("device", ctypes.c_int),
        ("hip_stream", ctypes.c_void_p),
        ("beta_rule", ctypes.c_int),
        ("averaged_primal", ctypes.c_int),
        ("gap_tol", ctypes.c_double),
    ]


class TapgResult(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("primal_res", ctypes.c_double),
        ("cost", ctypes.c_double),
        ("viol_box", ctypes.c_double),
        ("viol_eq", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("dual_gap", ctypes.c_double),
        ("dual_obj", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class TapgLoopStats(ctypes.Structure):
    _fields_ = [
        ("kpi_E", ctypes.c_double),
        ("kpi_S", ctypes.c_double),
        ("kpi_tau_ms", ctypes.c_double),
        ("mean_tau_ms", ctypes.c_double),
        ("max_viol_box", ctypes.c_double),
        ("max_viol_eq", ctypes.c_double),
        ("iters", ctypes.c_longlong),
        ("steps_converged", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


FORECAST_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))

_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib() -> ctypes.CDLL:
    """Load ``libtapg.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1904_10548_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "tapg_network_create": ([ctypes.c_int] * 4 + [_D] * 10 + [ctypes.POINTER(_P)], ctypes.c_int),
        "tapg_network_destroy": ([_P], None),
        "tapg_tree_create": ([ctypes.c_int, _I, _I, _D, ctypes.c_int, _D, _D, ctypes.POINTER(_P)],
                             ctypes.c_int),
        "tapg_tree_set_data": ([_P, _D, _D], ctypes.c_int),
        "tapg_tree_num_nodes": ([_P], ctypes.c_int),
        "tapg_tree_destroy": ([_P], None),
        "tapg_solver_create": ([_P, ctypes.POINTER(TapgConfig), ctypes.POINTER(_P)], ctypes.c_int),
        "tapg_solver_destroy": ([_P], None),
        "tapg_factor_step": ([_P, ctypes.c_int], ctypes.c_int),
        "tapg_get_factors": ([_P, ctypes.c_int, _D, _D, _D], ctypes.c_int),
        "tapg_factor_blocks": ([_P, _I, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "tapg_solver_forget": ([_P, _P], ctypes.c_int),
        "tapg_sweep_form": ([_P, ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "tapg_schedule_spec": ([_P, ctypes.c_int, ctypes.POINTER(_P), ctypes.c_char_p, ctypes.c_int],
                               ctypes.c_int),
        "tapg_event_pair_overhead": ([_P, _D], ctypes.c_int),
        "tapg_autotune": ([_P, ctypes.c_int, ctypes.POINTER(_P), ctypes.c_int, _D,
                           ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "tapg_server_create": ([_P, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_P)], ctypes.c_int),
        "tapg_server_submit": ([_P, _P, _D, _D, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)],
                               ctypes.c_int),
        "tapg_server_poll": ([_P, ctypes.c_longlong, ctypes.c_int, _D, ctypes.POINTER(TapgResult),
                             _D], ctypes.c_int),
        "tapg_server_stats": ([_P, ctypes.POINTER(ctypes.c_longlong),
                              ctypes.POINTER(ctypes.c_longlong), _D, ctypes.POINTER(ctypes.c_int)],
                             ctypes.c_int),
        "tapg_server_timing": ([_P, _D, _D, _D], ctypes.c_int),
        "tapg_server_destroy": ([_P], None),
        "tapg_solve": ([_P, _P, _D, _D, ctypes.c_int, _D, ctypes.POINTER(TapgResult)], ctypes.c_int),
        "tapg_solve_noalloc": ([_P, _P, _D, _D, _D, _D, _D, ctypes.POINTER(TapgResult)],
                               ctypes.c_int),
        "tapg_noalloc_bytes": ([_P, _P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "tapg_tree_build": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D, _I, ctypes.c_int,
                             ctypes.c_int, _I, _I, _D, _D, _I, _I], ctypes.c_int),
        "tapg_closed_loop": ([_P, _P, ctypes.c_int, _D, _D, FORECAST_FN, ctypes.c_void_p,
                              ctypes.c_int, _D, _D, _D, _I, ctypes.POINTER(TapgLoopStats)],
                             ctypes.c_int),
        "tapg_batch_solve": ([_P, ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_D),
                              ctypes.POINTER(_D), _I, ctypes.POINTER(_D),
                              ctypes.POINTER(TapgResult)], ctypes.c_int),
        "tapg_get_primal": ([_P, _P, _D, _D], ctypes.c_int),
        "tapg_get_dual": ([_P, _P, _D], ctypes.c_int),
        "tapg_set_dual": ([_P, _P, _D], ctypes.c_int),
        "tapg_residual_history": ([_P, _P, _D, ctypes.c_int, _I], ctypes.c_int),
        "tapg_residuals": ([_P, _P, ctypes.POINTER(TapgResult)], ctypes.c_int),
        "tapg_estimate_lipschitz": ([_P, _P, ctypes.c_int, _D], ctypes.c_int),
        "tapg_plan_schedule": ([_P, ctypes.c_int, ctypes.c_char_p, _I, ctypes.c_int, _I],
                               ctypes.c_int),
        "tapg_kernel_timing": ([_P, ctypes.c_int], ctypes.c_int),
        "tapg_kernel_times": ([_P, _D, ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
        "tapg_tree_dims": ([_P, _I, _I, _I], ctypes.c_int),
        "tapg_network_dims": ([_P, _I, _I, _I, _I], ctypes.c_int),
        "tapg_network_from_json": ([ctypes.c_char_p, ctypes.POINTER(_P)], ctypes.c_int),
        "tapg_tree_from_json": ([ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(_P)],
                                ctypes.c_int),
        "tapg_tree_data_from_json": ([ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int,
                                      ctypes.c_int, _D, _D], ctypes.c_int),
        "tapg_config_from_json": ([ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(TapgConfig), _D,
                                   _D, _D], ctypes.c_int),
        "tapg_state_from_json": ([ctypes.c_char_p, ctypes.c_int, ctypes.c_int, _D, _D],
                                 ctypes.c_int),
        "tapg_control_output_write": ([ctypes.c_char_p, ctypes.c_int, _D,
                                       ctypes.POINTER(TapgResult), ctypes.c_int], ctypes.c_int),
        "tapg_last_error": ([], ctypes.c_char_p),
        "tapg_version": ([], ctypes.c_char_p),
    }
    for name, (args, ret) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ret
    _lib = L
    return L


def _f64(a, n=None):
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and arr.size != n:
        raise ValueError(f"expected {n} values, got {arr.size}")
    return arr


def _ptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _check(status: int, allow=(TAPG_OK,)):
    if status not in allow:
        raise TapgError(status, lib().tapg_last_error().decode())
    return status


# --------------------------------------------------------------------------
# C-named functions
# --------------------------------------------------------------------------
def tapg_version() -> str:
    return lib().tapg_version().decode()


def tapg_last_error() -> str:
    return lib().tapg_last_error().decode()


def tapg_network_create(A, B, Gd, E, Ed, xmin, xmax, xs, umin, umax):
    A, B, Gd = _f64(A), _f64(B), _f64(Gd)
    nx, nu = B.shape
    nd = Gd.shape[1]
    E = _f64(E).reshape(-1, nu)
    ns = E.shape[0]
    Ed = _f64(Ed).reshape(ns, nd)
    arrs = [A, B, Gd, E, Ed, _f64(xmin, nx), _f64(xmax, nx), _f64(xs, nx), _f64(umin, nu),
            _f64(umax, nu)]
    out = _P()
    _check(lib().tapg_network_create(nx, nu, nd, ns, *[_ptr(a) for a in arrs], ctypes.byref(out)))
    return out


def tapg_network_destroy(h):
    lib().tapg_network_destroy(h)


def tapg_tree_create(nodes_per_stage, ancestor, prob, demand, price):
    mu = np.ascontiguousarray(nodes_per_stage, dtype=np.int32)
    anc = np.ascontiguousarray(ancestor, dtype=np.int32)
    K = int(mu.sum())
    if anc.size != K:
        raise ValueError("ancestor must have sum(nodes_per_stage) entries")
    demand = _f64(demand).reshape(K, -1)
    prob = _f64(prob, K)
    price = _f64(price, K)
    out = _P()
    _check(lib().tapg_tree_create(len(mu), mu.ctypes.data_as(_I), anc.ctypes.data_as(_I),
                                  _ptr(prob), demand.shape[1], _ptr(demand), _ptr(price),
                                  ctypes.byref(out)))
    return out


def tapg_tree_set_data(tree, demand, price):
    K = lib().tapg_tree_num_nodes(tree)
    demand = _f64(demand)
    if demand.size % max(K, 1):
        raise ValueError("demand must have K*nd values")
    _check(lib().tapg_tree_set_data(tree, _ptr(demand), _ptr(_f64(price, K))))


def tapg_tree_num_nodes(tree) -> int:
    return lib().tapg_tree_num_nodes(tree)


def tapg_tree_destroy(h):
    lib().tapg_tree_destroy(h)


def tapg_tree_dims(tree):
    """(N, K, nd) of a tree."""
    v = [ctypes.c_int(0) for _ in range(3)]
    _check(lib().tapg_tree_dims(tree, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def tapg_network_dims(net):
    """(nx, nu, nd, ns) of a network."""
    v = [ctypes.c_int(0) for _ in range(4)]
    _check(lib().tapg_network_dims(net, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def _path(p):
    return None if p is None else os.fsencode(p)


def tapg_network_from_json(path):
    out = _P()
    _check(lib().tapg_network_from_json(_path(path), ctypes.byref(out)))
    return out


def tapg_tree_from_json(tree_path, forecaster_path=None):
    out = _P()
    _check(lib().tapg_tree_from_json(_path(tree_path), _path(forecaster_path), ctypes.byref(out)))
    return out


def tapg_tree_data_from_json(tree_path, forecaster_path, K, nd):
    """(demand [K, nd], price [K]) as the tree built from these files holds."""
    dem, pr = np.zeros((K, nd)), np.zeros(K)
    _check(lib().tapg_tree_data_from_json(_path(tree_path), _path(forecaster_path), int(K),
                                          int(nd), _ptr(dem), _ptr(pr)))
    return dem, pr


def tapg_config_from_json(path, nu):
    """A :class:`TapgConfig` plus the arrays it points to (keep both alive)."""
    keep = [np.zeros(nu), np.zeros(nu), np.zeros(nu * nu)]
    cfg = TapgConfig()
    _check(lib().tapg_config_from_json(_path(path), int(nu), ctypes.byref(cfg), _ptr(keep[0]),
                                       _ptr(keep[1]), _ptr(keep[2])))
    return cfg, keep


def tapg_state_from_json(path, nx, nu):
    x, u = np.zeros(nx), np.zeros(nu)
    _check(lib().tapg_state_from_json(_path(path), int(nx), int(nu), _ptr(x), _ptr(u)))
    return x, u


def tapg_control_output_write(path, u0, result, status=TAPG_OK):
    u = _f64(u0)
    _check(lib().tapg_control_output_write(_path(path), u.size, _ptr(u), ctypes.byref(result),
                                           int(status)))


def make_config(nu, W_alpha, W_s, W_x, alpha0, c_energy, W_u, gamma=0.0, tol=1e-4,
                max_iter=10000, check_every=100, precision=TAPG_FP64, power_iters=100,
                device=0, stream=None, beta_rule=TAPG_BETA_PAPER, averaged_primal=False,
                gap_tol=0.0):
    """A :class:`TapgConfig` plus the arrays it points to (keep both alive)."""
    keep = [_f64(alpha0, nu), _f64(c_energy, nu), _f64(W_u, nu * nu)]
    cfg = TapgConfig(W_alpha, W_s, W_x, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]), gamma, tol,
                     max_iter, check_every, precision, power_iters, device,
                     ctypes.c_void_p(stream) if stream else None, int(beta_rule),
                     int(bool(averaged_primal)), float(gap_tol))
    return cfg, keep


def tapg_solver_create(net, cfg: TapgConfig):
    out = _P()
    _check(lib().tapg_solver_create(net, ctypes.byref(cfg), ctypes.byref(out)))
    return out


def tapg_solver_destroy(h):
    lib().tapg_solver_destroy(h)


def tapg_factor_step(solver, N: int):
    _check(lib().tapg_factor_step(solver, int(N)))


def tapg_get_factors(solver, stage: int, nu: int):
    F, Kb, G = (np.zeros((nu, nu)) for _ in range(3))
    _check(lib().tapg_get_factors(solver, stage, _ptr(F), _ptr(Kb), _ptr(G)))
    return F, Kb, G


def tapg_factor_blocks(solver, N: int):
    """``(fid, n_blocks)``: the factor block serving each stage and the count."""
    fid = np.zeros(N, dtype=np.int32)
    nb = ctypes.c_int(0)
    _check(lib().tapg_factor_blocks(solver, fid.ctypes.data_as(_I), N, ctypes.byref(nb)))
    return fid, nb.value


def tapg_solve(solver, tree, p, q, warm_start=False, nu=None):
    """Returns ``(status, u0, result)``; status is TAPG_OK or TAPG_ENOTCONV."""
    q = _f64(q)
    u0 = np.zeros(q.size if nu is None else nu)
    res = TapgResult()
    st = _check(lib().tapg_solve(solver, tree, _ptr(_f64(p)), _ptr(q), int(bool(warm_start)),
                                 _ptr(u0), ctypes.byref(res)), allow=(TAPG_OK, TAPG_ENOTCONV))
    return st, u0, res


NOALLOC_SCRATCH_BYTES = 64 << 20


def tapg_solve_noalloc(solver, tree, p, q, K, nx, nu):
    """Solve without device allocation; returns ``(status, u0, u, x, result)``."""
    u0 = np.zeros(nu)
    u = np.zeros((K, nu))
    x = np.zeros((K, nx))
    res = TapgResult()
    st = _check(lib().tapg_solve_noalloc(solver, tree, _ptr(_f64(p)), _ptr(_f64(q)), _ptr(u0),
                                         _ptr(u), _ptr(x), ctypes.byref(res)),
                allow=(TAPG_OK, TAPG_ENOTCONV))
    return st, u0, u, x, res


def tapg_noalloc_bytes(solver, tree) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tapg_noalloc_bytes(solver, tree, ctypes.byref(b)))
    return b.value


def tapg_tree_build(samples, branching, prob=None, device=0, cap=None):
    """Scenario tree from sample paths ``samples`` (M, H, d) with ``branching``
    (H,).  Returns a dict: nodes_per_stage, anc, prob, value (K, d), rep."""
    S = _f64(samples)
    M, H, d = S.shape
    br = np.ascontiguousarray(branching, dtype=np.int32)
    if br.size != H:
        raise ValueError("branching must have H entries")
    if cap is None:  # stage t has at most min(M, b_1 ... b_t) nodes
        cap, width = 1, 1
        for t in range(1, H):
            width = min(M, width * max(int(br[t]), 1))
            cap += width
    mu = np.zeros(H, dtype=np.int32)
    anc = np.zeros(cap, dtype=np.int32)
    pr = np.zeros(cap)
    val = np.zeros((cap, d))
    rep = np.zeros(cap, dtype=np.int32)
    K = ctypes.c_int(0)
    pp = None if prob is None else _f64(prob, M)
    _check(lib().tapg_tree_build(M, H, d, _ptr(S), _ptr(pp), br.ctypes.data_as(_I), int(device),
                                 int(cap), mu.ctypes.data_as(_I), anc.ctypes.data_as(_I), _ptr(pr),
                                 _ptr(val), rep.ctypes.data_as(_I), ctypes.byref(K)))
    k = K.value
    return {"nodes_per_stage": mu, "anc": anc[:k], "prob": pr[:k], "value": val[:k],
            "rep": rep[:k]}


def tapg_closed_loop(solver, tree, H_s, x0, u_prev, forecast, K, nd, warm_start=True):
    """Closed-loop simulation; ``forecast(k) -> (demand [K, nd], price [K])``
    supplies the tree's data at step k.  Returns ``(x_traj, u_traj, tau_ms,
    iters, stats)``."""
    x0, u_prev = _f64(x0), _f64(u_prev)
    nx, nu = x0.size, u_prev.size
    err = []

    def cb(ctx, k, dptr, pptr):
        try:
            d, p = forecast(k)
            d = _f64(d, K * nd)
            p = _f64(p, K)
            ctypes.memmove(dptr, d.ctypes.data, d.nbytes)
            ctypes.memmove(pptr, p.ctypes.data, p.nbytes)
            return 0
        except Exception as e:  # reported after the call
            err.append(e)
            return 1

    fn = FORECAST_FN(cb)
    xt = np.zeros((H_s + 1, nx))
    ut = np.zeros((H_s, nu))
    tau = np.zeros(H_s)
    its = np.zeros(H_s, dtype=np.int32)
    st = TapgLoopStats()
    status = lib().tapg_closed_loop(solver, tree, int(H_s), _ptr(x0), _ptr(u_prev), fn, None,
                                    int(bool(warm_start)), _ptr(xt), _ptr(ut), _ptr(tau),
                                    its.ctypes.data_as(_I), ctypes.byref(st))
    if err:
        raise err[0]
    _check(status)
    return xt, ut, tau, its, st


def tapg_batch_solve(solver, trees, ps, qs, warm_start=None, nu=None):
    """Solve ``trees`` together.  Returns ``(status, [u0], [result])``; status
    is TAPG_OK or TAPG_ENOTCONV (TAPG_ENUMERIC raises)."""
    n = len(trees)
    keep = [_f64(v) for v in ps] + [_f64(v) for v in qs]
    tarr = (_P * n)(*trees)
    parr = (_D * n)(*[_ptr(v) for v in keep[:n]])
    qarr = (_D * n)(*[_ptr(v) for v in keep[n:]])
    width = (keep[n].size if n else 0) if nu is None else nu
    u0 = [np.zeros(width) for _ in range(n)]
    uarr = (_D * n)(*[_ptr(v) for v in u0])
    warr = None
    if warm_start is not None:
        w = np.ascontiguousarray([int(bool(v)) for v in warm_start], dtype=np.int32)
        keep.append(w)
        warr = w.ctypes.data_as(_I)
    res = (TapgResult * n)()
    st = _check(lib().tapg_batch_solve(solver, n, tarr, parr, qarr, warr, uarr, res),
                allow=(TAPG_OK, TAPG_ENOTCONV))
    return st, u0, list(res)


def tapg_autotune(solver, trees, iters=20):
    """Time every candidate schedule of the tree / batch and keep the fastest;
    returns ``(ms_per_iteration, candidates)``."""
    n = len(trees)
    tarr = (_P * n)(*trees)
    ms = np.zeros(1)
    nc = ctypes.c_int(0)
    _check(lib().tapg_autotune(solver, n, tarr, int(iters), _ptr(ms), ctypes.byref(nc)))
    return float(ms[0]), nc.value


FORM_NAMES = {0: "stages", 1: "segment", 2: "projector", 3: "scan"}


def tapg_schedule_spec(solver, trees):
    """Schedule of a tree or batch after its last solve / autotune, as the
    environment settings that force it (e.g. "TAPG_SCAN=1 TAPG_LEVELS=0:1,5:1
    TAPG_FWD_GROUP=1")."""
    n = len(trees)
    tarr = (_P * n)(*trees)
    buf = ctypes.create_string_buffer(4096)
    _check(lib().tapg_schedule_spec(solver, n, tarr, buf, len(buf)))
    return buf.value.decode()


def tapg_sweep_form(solver, trees):
    """Sweep form of a tree or batch after its last solve / autotune:
    ``(form name, backward launches per iteration)``."""
    n = len(trees)
    tarr = (_P * n)(*trees)
    f, nl = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().tapg_sweep_form(solver, n, tarr, ctypes.byref(f), ctypes.byref(nl)))
    return FORM_NAMES.get(f.value, str(f.value)), nl.value


def tapg_solver_forget(solver, tree):
    _check(lib().tapg_solver_forget(solver, tree))


def tapg_server_create(solver, hbm_budget_bytes, max_batch=64):
    out = _P()
    _check(lib().tapg_server_create(solver, int(hbm_budget_bytes), int(max_batch),
                                    ctypes.byref(out)))
    return out


def tapg_server_submit(srv, tree, p, q, session=0):
    t = ctypes.c_longlong(0)
    _check(lib().tapg_server_submit(srv, tree, _ptr(_f64(p)), _ptr(_f64(q)), int(session),
                                    ctypes.byref(t)))
    return t.value


def tapg_server_poll(srv, ticket, nu, wait_ms=-1):
    """``(status, u0, result, latency_ms)``; status TAPG_ESTATE while pending,
    else the request's own status (an unknown ticket raises)."""
    u0 = np.zeros(nu)
    res = TapgResult()
    lat = np.zeros(1)
    st = lib().tapg_server_poll(srv, int(ticket), int(wait_ms), _ptr(u0), ctypes.byref(res),
                                _ptr(lat))
    if st == TAPG_EINVAL:
        _check(st)
    return st, u0, res, float(lat[0])


def tapg_server_stats(srv):
    b, s = ctypes.c_longlong(0), ctypes.c_longlong(0)
    busy = np.zeros(1)
    pend = ctypes.c_int(0)
    _check(lib().tapg_server_stats(srv, ctypes.byref(b), ctypes.byref(s), _ptr(busy),
                                   ctypes.byref(pend)))
    return {"batches": b.value, "solved": s.value, "busy_ms": float(busy[0]),
            "pending": pend.value}


def tapg_server_timing(srv):
    """Worker time in ms: forming forests, chunks of iterations, leaving forests."""
    t = np.zeros(3)
    _check(lib().tapg_server_timing(srv, _ptr(t[0:1]), _ptr(t[1:2]), _ptr(t[2:3])))
    return {"enter_ms": float(t[0]), "chunk_ms": float(t[1]), "leave_ms": float(t[2])}


def tapg_server_destroy(srv):
    lib().tapg_server_destroy(srv)


def tapg_get_primal(solver, tree, K, nx, nu):
    u = np.zeros((K, nu))
    x = np.zeros((K, nx))
    _check(lib().tapg_get_primal(solver, tree, _ptr(u), _ptr(x)))
    return u, x


def tapg_get_dual(solver, tree, K, m):
    y = np.zeros((K, m))
    _check(lib().tapg_get_dual(solver, tree, _ptr(y)))
    return y


def tapg_set_dual(solver, tree, y):
    _check(lib().tapg_set_dual(solver, tree, _ptr(_f64(y))))


def tapg_residual_history(solver, tree, n):
    h = np.zeros(max(n, 1))
    w = ctypes.c_int(0)
    _check(lib().tapg_residual_history(solver, tree, _ptr(h), n, ctypes.byref(w)))
    return h[:w.value]


def tapg_residuals(solver, tree) -> TapgResult:
    r = TapgResult()
    _check(lib().tapg_residuals(solver, tree, ctypes.byref(r)))
    return r


def tapg_estimate_lipschitz(solver, tree, iters=100) -> float:
    L = ctypes.c_double(0.0)
    _check(lib().tapg_estimate_lipschitz(solver, tree, int(iters), ctypes.byref(L)))
    return L.value


def tapg_plan_schedule(tree, precision=TAPG_FP64, levels=None):
    """List of (first stage, last stage, group, workgroups, widest stage)."""
    cap = 256
    out = np.zeros(5 * cap, dtype=np.int32)
    n = ctypes.c_int(0)
    _check(lib().tapg_plan_schedule(tree, precision, levels.encode() if levels else None,
                                    out.ctypes.data_as(_I), cap, ctypes.byref(n)))
    return [tuple(int(v) for v in out[5 * i:5 * i + 5]) for i in range(min(n.value, cap))]


def tapg_kernel_timing(solver, enable: bool):
    _check(lib().tapg_kernel_timing(solver, int(bool(enable))))


def tapg_event_pair_overhead(solver):
    """Microseconds that an event pair adds to each timed launch (median)."""
    us = np.zeros(1)
    _check(lib().tapg_event_pair_overhead(solver, _ptr(us)))
    return float(us[0])


def tapg_kernel_times(solver):
    """``{'bwd': (ms, launches), 'fwd': (...), 'end': (...), 'chain': (ms, iterations)}``
    of the last timed solve."""
    ms = np.zeros(4)
    n = (ctypes.c_longlong * 4)()
    _check(lib().tapg_kernel_times(solver, _ptr(ms), n))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(["bwd", "fwd", "end", "chain"])}


# --------------------------------------------------------------------------
# Owner object
# --------------------------------------------------------------------------
class Solver:
    """Network + solver handles for one set of weights; trees are added with
    :meth:`add_tree` and released with the solver."""

    def __init__(self, net_arrays: dict, weights: dict, N: int, **cfg_kw):
        self.nx = int(np.asarray(net_arrays["B"]).shape[0])
        self.nu = int(np.asarray(net_arrays["B"]).shape[1])
        self.net = tapg_network_create(**net_arrays)
        self.cfg, self._keep = make_config(self.nu, **weights, **cfg_kw)
        try:
            self.h = tapg_solver_create(self.net, self.cfg)
        except Exception:
            tapg_network_destroy(self.net)
            raise
        self.trees = []
        tapg_factor_step(self.h, N)

    def add_tree(self, nodes_per_stage, ancestor, prob, demand, price):
        t = tapg_tree_create(nodes_per_stage, ancestor, prob, demand, price)
        self.trees.append(t)
        return t

    def solve(self, tree, p, q, warm_start=False):
        return tapg_solve(self.h, tree, p, q, warm_start, nu=self.nu)

    def batch_solve(self, trees, ps, qs, warm_start=None):
        return tapg_batch_solve(self.h, trees, ps, qs, warm_start, nu=self.nu)

    def primal(self, tree):
        return tapg_get_primal(self.h, tree, tapg_tree_num_nodes(tree), self.nx, self.nu)

    def dual(self, tree):
        return tapg_get_dual(self.h, tree, tapg_tree_num_nodes(tree), 2 * self.nx + self.nu)

    def close(self):
        if getattr(self, "h", None):
            tapg_solver_destroy(self.h)
            self.h = None
        for t in self.trees:
            tapg_tree_destroy(t)
        self.trees = []
        if getattr(self, "net", None):
            tapg_network_destroy(self.net)
            self.net = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
