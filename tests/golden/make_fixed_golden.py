"""Write the oracle's iterates at fixed iteration counts for the FP32 accuracy
tests: the 128-scenario tree after 3,000 iterations and the 2,048-scenario
tree after 500, each at an explicit step size (1/(1.02 L), L by the oracle's
power iteration).  Stored: the step size, the cost, the violations, the root
input and the primal at a few sampled nodes.  Everything comes from
``oracle/`` on inputs from ``dwn_synth/``.  Run with
``python tests/golden/make_fixed_golden.py`` (about 10 minutes).
"""

from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import dwn_synth as ds  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fixed_iterations.json")
CASES = (("dwn128", 3000, (0, 1, 4, 17, 60, 250, 700, 1500, 2428)),
         ("dwn2048", 500, (0, 1, 4, 17, 60, 250, 700, 5000, 20000, 30716)))


def main() -> None:
    out = {"source": "oracle.apg on dwn_synth.config_problem(name); this script"}
    for name, iters, nodes in CASES:
        t0 = time.time()
        P = ds.config_problem(name)
        sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
        L = O.lipschitz_power(P, sf, 60)
        gamma = 1.0 / (1.02 * L)
        r = O.apg(P, gamma, sf, iters)
        vb, ve = O.violations(P, r.u, r.x)
        out[name] = dict(iters=iters, L=L, gamma=gamma, K=P.tree.K,
                         cost=O.primal_cost(P, r.u, r.x), viol_box=vb, viol_eq=ve,
                         final_res=r.res, u_root=r.u[0].tolist(), sample_nodes=list(nodes),
                         u_sample=[r.u[n].tolist() for n in nodes],
                         x_sample=[r.x[n].tolist() for n in nodes],
                         oracle_seconds=time.time() - t0)
        print(f"{name}: {iters} iterations, cost {out[name]['cost']!r}, "
              f"{time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
