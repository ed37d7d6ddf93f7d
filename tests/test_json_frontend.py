"""The JSON front-end (Sec. 5.1: network, scenario tree, forecaster,
controller configuration and control output as JSON files) on the host: files
read back exactly, node data = forecast + error (eq. prediction-error), and
strict errors for malformed, misspelt, misshapen or inconsistent files.  No
GPU: these calls only parse and validate."""

import json
import math
import os

import numpy as np
import pytest

import dwn_synth as ds
from dwn_synth import json_files as jf
from paper_1904_10548_amd import tapg


@pytest.fixture
def small(tmp_path):
    P = ds.config_problem("small")
    return P, jf.write_instance(P, str(tmp_path), tol=1e-5, max_iter=777, check_every=13,
                                precision="fp32", beta_rule="simple", gap_tol=2.5e-3)


def _status(fn, *a):
    with pytest.raises(tapg.TapgError) as e:
        fn(*a)
    return e.value.status, str(e.value)


def test_network_and_tree_from_files(small):
    P, f = small
    net = tapg.tapg_network_from_json(f["network"])
    try:
        assert tapg.tapg_network_dims(net) == (P.net.nx, P.net.nu, P.net.nd, P.net.ns)
    finally:
        tapg.tapg_network_destroy(net)
    t = tapg.tapg_tree_from_json(f["tree"], f["forecaster"])
    try:
        K = int(np.sum(P.tree.nodes_per_stage))
        assert tapg.tapg_tree_dims(t) == (P.tree.N, K, P.net.nd)
        assert tapg.tapg_tree_num_nodes(t) == K
    finally:
        tapg.tapg_tree_destroy(t)


def test_node_data_is_forecast_plus_error_exactly(small):
    P, f = small
    K, nd = int(np.sum(P.tree.nodes_per_stage)), P.net.nd
    dem, pr = tapg.tapg_tree_data_from_json(f["tree"], f["forecaster"], K, nd)
    fd, fp, ed, ep = jf.split_forecast(P.tree, P.data.demand, P.data.price)
    want_d, want_p = jf.node_data_from_split(P.tree, fd, fp, ed, ep)
    assert np.array_equal(dem, want_d) and np.array_equal(pr, want_p)
    # and within rounding of the generated node data
    assert np.allclose(dem, P.data.demand, rtol=1e-14, atol=1e-12)
    # the root's error is zero: its data is the forecast of stage 0
    assert np.array_equal(dem[0], fd[0]) and pr[0] == fp[0]


def test_tree_of_node_values_reads_back_exactly(tmp_path):
    P = ds.config_problem("small")
    path = jf.write_tree(P.tree, str(tmp_path / "t.json"), demand=P.data.demand,
                         price=P.data.price, children=True)
    K, nd = int(np.sum(P.tree.nodes_per_stage)), P.net.nd
    dem, pr = tapg.tapg_tree_data_from_json(path, None, K, nd)
    assert np.array_equal(dem, P.data.demand) and np.array_equal(pr, P.data.price)
    # a forecaster for a tree of values is an error, and so is none for errors
    fc = jf.write_forecaster(P.data.demand[:P.tree.N], P.data.price[:P.tree.N],
                             str(tmp_path / "f.json"))
    st, msg = _status(tapg.tapg_tree_data_from_json, path, fc, K, nd)
    assert st == tapg.TAPG_EINVAL and "forecaster" in msg
    st, _ = _status(tapg.tapg_tree_data_from_json, path, None, K + 1, nd)
    assert st == tapg.TAPG_EDIM


def test_config_reads_every_field(small):
    P, f = small
    nu = P.net.nu
    cfg, keep = tapg.tapg_config_from_json(f["config"], nu)
    w = P.weights
    assert (cfg.W_alpha, cfg.W_s, cfg.W_x) == (w.W_alpha, w.W_s, w.W_x)
    assert np.array_equal(keep[0], w.alpha0) and np.array_equal(keep[1], w.c_energy)
    assert np.array_equal(keep[2].reshape(nu, nu), w.W_u)
    assert cfg.tol == 1e-5 and cfg.max_iter == 777 and cfg.check_every == 13
    assert cfg.precision == tapg.TAPG_FP32 and cfg.beta_rule == tapg.TAPG_BETA_SIMPLE
    assert cfg.gap_tol == 2.5e-3 and cfg.averaged_primal == 0
    assert cfg.gamma == 0.0 and cfg.power_iters == 100 and cfg.device == 0
    assert not cfg.hip_stream
    # the config's pointers are the caller's arrays
    assert cfg.alpha0[0] == keep[0][0] and cfg.W_u[nu * nu - 1] == keep[2][-1]


def test_config_scalar_W_u_means_a_multiple_of_the_identity(tmp_path):
    P = ds.config_problem("small")
    path = jf.write_config(P.weights, str(tmp_path / "c.json"), 1e-4, 10)
    obj = json.load(open(path))
    obj["W_u"] = 100.0
    json.dump(obj, open(path, "w"))
    cfg, keep = tapg.tapg_config_from_json(path, P.net.nu)
    assert np.array_equal(keep[2].reshape(P.net.nu, P.net.nu), 100.0 * np.eye(P.net.nu))


def test_state_reads_back(small):
    P, f = small
    x, u = tapg.tapg_state_from_json(f["state"], P.net.nx, P.net.nu)
    assert np.array_equal(x, P.p) and np.array_equal(u, P.q)
    st, _ = _status(tapg.tapg_state_from_json, f["state"], P.net.nx + 1, P.net.nu)
    assert st == tapg.TAPG_EDIM


def test_control_output_round_trip(tmp_path):
    r = tapg.TapgResult()
    r.iters, r.converged, r.primal_res, r.cost = 1234, 0, 3.3e-4, 657.9277121235365
    r.viol_box, r.viol_eq, r.gamma, r.solve_ms = 0.0, 1e-15, 1.4337926496058389e-06, 7.25
    r.dual_gap, r.dual_obj = math.nan, math.inf
    u = np.array([0.1, -2.5e-17, 1.0 / 3.0, 7e300])
    path = str(tmp_path / "controlOutput.json")
    tapg.tapg_control_output_write(path, u, r, tapg.TAPG_ENOTCONV)
    out = json.load(open(path))
    assert out["status"] == "not_converged" and out["iters"] == 1234 and out["converged"] is False
    assert out["u"] == list(u)  # 17 significant digits read back exactly
    assert out["cost"] == r.cost and out["gamma"] == r.gamma
    assert out["dual_gap"] is None and out["dual_obj"] is None
    assert not os.path.exists(path + ".tmp")


def _write(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


@pytest.mark.parametrize("text,where,what", [
    ('{"a": 1,}', "1:9", "key string"),
    ('{"a": [1, 2 3]}', "1:13", "',' or ']'"),
    ('{"a": 01}', "1:8", "',' or '}'"),
    ('{"a": 1.}', "1:9", "after '.'"),
    ('{"a": 1e}', "1:9", "exponent"),
    ('{"a": 1e999}', "1:12", "out of range"),
    ('{"a": "x\\q"}', "1:11", "escape"),
    ('{"a": "\\ud800"}', "1:14", "surrogate"),
    ('{"a": NaN}', "1:7", "unexpected character"),
    ('{"a": 1} x', "1:10", "after the top-level"),
    ('{"a": 1, "a": 2}', "1:13", "duplicate"),
    ('\n\n  {"a": tru}', "3:9", "unexpected character"),
    ('[' * 70 + ']' * 70, "1:66", "deeper than 64"),
    ('{"a": "unterminated', "1:20", "unterminated"),
])
def test_syntax_errors_name_line_and_column(tmp_path, text, where, what):
    p = _write(tmp_path, "bad.json", text)
    st, msg = _status(tapg.tapg_state_from_json, p, 1, 1)
    assert st == tapg.TAPG_EINVAL
    assert f"bad.json:{where}:" in msg and what in msg, msg


def test_valid_json_details_are_accepted(tmp_path):
    p = _write(tmp_path, "s.json",
               '{"name": "caf\\u00e9 \\ud83d\\ude00 \\"q\\" \\/", "description": "", '
               '"k": 0, "x": [-0, 1E+2, 2.5e-3, -1.0e1], "u_prev": [0.1]}')
    x, u = tapg.tapg_state_from_json(p, 4, 1)
    assert list(x) == [0.0, 100.0, 2.5e-3, -10.0] and list(u) == [0.1]
    assert math.copysign(1.0, x[0]) == -1.0


def test_strict_keys_types_and_shapes(small, tmp_path):
    P, f = small
    net = json.load(open(f["network"]))

    def net_status(mutate):
        obj = json.loads(json.dumps(net))
        mutate(obj)
        p = str(tmp_path / "n.json")
        json.dump(obj, open(p, "w"))
        return _status(tapg.tapg_network_from_json, p)

    st, msg = net_status(lambda o: o.update(Xmin=o["xmin"]))
    assert st == tapg.TAPG_EINVAL and 'unknown key "Xmin"' in msg
    st, msg = net_status(lambda o: o.pop("xs"))
    assert st == tapg.TAPG_EINVAL and 'missing key "xs"' in msg
    st, msg = net_status(lambda o: o.update(B=o["B"][:-1]))
    assert st == tapg.TAPG_EDIM and '"B"' in msg
    st, msg = net_status(lambda o: o["A"][1].append(0.0))
    assert st == tapg.TAPG_EDIM and "row 1" in msg
    st, msg = net_status(lambda o: o.update(nu=o["nu"] + 1))
    assert st == tapg.TAPG_EDIM and '"nu"' in msg
    st, msg = net_status(lambda o: o.update(umin="0"))
    assert st == tapg.TAPG_EINVAL and "expected an array" in msg
    # validation of the array entry point still applies: rank-deficient E
    st, msg = net_status(lambda o: o.update(E=[o["E"][0], o["E"][0]] + o["E"][2:]))
    assert st == tapg.TAPG_ENUMERIC and "n.json" in msg
    # umin > umax
    st, _ = net_status(lambda o: o.update(umin=[v + 1e9 for v in o["umax"]]))
    assert st == tapg.TAPG_EINVAL


def test_tree_file_errors(small, tmp_path):
    P, f = small
    tree = json.load(open(f["tree"]))

    def tree_status(mutate, fc=f["forecaster"]):
        obj = json.loads(json.dumps(tree))
        mutate(obj)
        p = str(tmp_path / "t.json")
        json.dump(obj, open(p, "w"))
        return _status(tapg.tapg_tree_from_json, p, fc)

    st, msg = tree_status(lambda o: o.update(N=o["N"] + 1))
    assert st == tapg.TAPG_EDIM
    st, msg = tree_status(lambda o: o.update(ancestor=o["ancestor"][:-1]))
    assert st == tapg.TAPG_EDIM and '"ancestor"' in msg
    st, msg = tree_status(lambda o: o.update(demand=o["demand_error"]))
    assert st == tapg.TAPG_EINVAL and "either" in msg
    # explicit children that disagree with the ancestors
    K = int(np.sum(P.tree.nodes_per_stage))
    ch = [[] for _ in range(K)]
    for n in range(1, K):
        ch[int(P.tree.anc[n])].append(n)
    ch[0] = ch[0][::-1]
    st, msg = tree_status(lambda o: o.update(children=ch))
    assert st == tapg.TAPG_EINVAL and "node 0" in msg
    # tree validation of the array entry point: probabilities that do not add up
    st, msg = tree_status(lambda o: o["probability"].__setitem__(-1, 0.5))
    assert st == tapg.TAPG_EINVAL
    # forecaster with the wrong number of stages
    fc = json.load(open(f["forecaster"]))
    fc["price"] = fc["price"][:-1]
    p = str(tmp_path / "f.json")
    json.dump(fc, open(p, "w"))
    st, msg = _status(tapg.tapg_tree_from_json, f["tree"], p)
    assert st == tapg.TAPG_EDIM and "f.json" in msg
    st, msg = _status(tapg.tapg_tree_from_json, str(tmp_path / "missing.json"), None)
    assert st == tapg.TAPG_EINVAL and "cannot open" in msg


def test_config_errors(small, tmp_path):
    P, f = small
    cfg = json.load(open(f["config"]))
    for key, val, code, text in [("precision", "fp16", tapg.TAPG_EINVAL, "fp64"),
                                 ("beta_rule", "nesterov", tapg.TAPG_EINVAL, "paper"),
                                 ("max_iter", 10.5, tapg.TAPG_EINVAL, "integer"),
                                 ("averaged_primal", 1, tapg.TAPG_EINVAL, "true or false"),
                                 ("W_u", [[1.0]], tapg.TAPG_EDIM, '"W_u"'),
                                 ("tolerance", 1e-4, tapg.TAPG_EINVAL, "unknown key")]:
        obj = dict(cfg)
        obj[key] = val
        p = str(tmp_path / "c.json")
        json.dump(obj, open(p, "w"))
        st, msg = _status(tapg.tapg_config_from_json, p, P.net.nu)
        assert st == code and text in msg, (key, msg)


def test_cli_rejects_bad_usage():
    import subprocess
    cli = os.path.join(os.path.dirname(tapg.LIB_PATH), "tapg_control")
    assert os.path.exists(cli), "build the library first (it builds tapg_control too)"
    r = subprocess.run([cli, "--network"], capture_output=True, text=True)
    assert r.returncode == 1 and "usage" in r.stderr
    r = subprocess.run([cli, "--network", "/nonexistent.json", "--config", "c", "--tree", "t",
                        "--state", "s", "--output", "o"], capture_output=True, text=True)
    assert r.returncode == 1 and "cannot open /nonexistent.json" in r.stderr
