"""Write the oracle's full solve of the 128-scenario tree to tolerance 1e-4.

Stored values for the GPU test that runs the same solve: the step size, the
stopping iteration, the residual every 1,000 iterations, and the result at the
stop (cost, violations, root input, the primal at a few sampled nodes), plus
the iterate at two fixed iteration counts on the way.  Everything here comes
from ``oracle/`` on inputs from ``dwn_synth/``; nothing from the GPU library.

The solve is the dual APG of Sec. 4.3 (eqs. apg:1-apg:2) with the stop test
``max |H x_hat(w) - t| <= tol`` read in Sec. 6's sense of a tolerance on the
dual iteration.  It takes the oracle about 1.5 hours (~112,000 iterations at
~50 ms each); run it with ``python tests/golden/make_dwn128_golden.py``.
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import dwn_synth as ds  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dwn128_tol1e-4.json")
TOL = 1e-4
MAX_ITER = 400_000
SNAPSHOTS = (1_000, 20_000)
SAMPLE_NODES = (0, 1, 4, 17, 60, 250, 700, 1500, 2428)


def main() -> None:
    P = ds.config_problem("dwn128")
    sf = O.StageFactors(P.net, P.weights.W_u, P.tree)
    L = O.lipschitz_power(P, sf, 200)
    gamma = 1.0 / (1.02 * L)
    print(f"L={L!r} gamma={gamma!r}", flush=True)
    snaps = {}
    t0 = time.time()

    def cb(nu, y_new, w, u, x):
        it = nu + 1
        if it in SNAPSHOTS:
            vb, ve = O.violations(P, u, x)
            snaps[str(it)] = dict(cost=O.primal_cost(P, u, x), viol_box=vb,
                                  u_root=u[0].tolist(), x_root=x[0].tolist())
        if it % 1000 == 0:
            print(f"iter {it} elapsed {time.time() - t0:.0f} s", flush=True)

    ref = O.apg(P, gamma, sf, MAX_ITER, tol=TOL, callback=cb)
    vb, ve = O.violations(P, ref.u, ref.x)
    hist = np.asarray(ref.res_hist)
    out = dict(
        source="oracle.apg on dwn_synth.config_problem('dwn128'); this script",
        workload="dwn128: nx=63, nu=114, nd=88, N=24, 128 scenarios, K=2429, W_u=100 I",
        tol=TOL, L=L, gamma=gamma, iters=ref.iters, converged=bool(ref.converged),
        final_res=ref.res, cost=O.primal_cost(P, ref.u, ref.x), viol_box=vb, viol_eq=ve,
        u_root=ref.u[0].tolist(),
        sample_nodes=list(SAMPLE_NODES),
        u_sample=[ref.u[n].tolist() for n in SAMPLE_NODES],
        x_sample=[ref.x[n].tolist() for n in SAMPLE_NODES],
        res_every_1000=[float(hist[k - 1]) for k in range(1000, len(hist) + 1, 1000)],
        snapshots=snaps,
        oracle_seconds=time.time() - t0,
    )
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}: iters={ref.iters} cost={out['cost']!r}", flush=True)


if __name__ == "__main__":
    main()
