"""FP64 CPU oracle for the dual APG solver of scenario-tree stochastic MPC.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, direct NumPy/SciPy
implementation of what the GPU library computes, written from the paper
(Sopasakis et al., arXiv 1904.10548, Sec. 4 "Numerical Algorithm") and from
the dynamic-programming derivation of the dual gradient stated in
:mod:`oracle.dual_gradient`.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

It shares no code with the GPU path.  Its inputs come from the seeded
generators in :mod:`dwn_synth`, which hold none of the solver's arithmetic.

Modules
-------
tree            children lists, stage ranges and scenario paths from ``anc``
dual_gradient   x_hat(w) = argmin f(x) + <w, Hx>: per-node DP, per-stage DP,
                dense KKT
prox            distance-function prox, box projection, Moreau decomposition
apg             the accelerated proximal gradient on the Fenchel dual
objective       primal cost, constraint violations, dual objective,
                duality gap of a dual point
stepsize        Lipschitz constant of the dual gradient (power iteration and
                the dense eigenvalue for tiny trees)
closed_loop     receding-horizon simulation with the paper's performance indices
tree_build      scenario tree from sampled error paths by forward selection

Every function is pinned by a ``-m "not gpu"`` test against an independent
fact (closed forms, brute force, a textbook solver); none is "parity
unpinned".
"""

from .tree import TreeIndex
from .dual_gradient import (
    NodeFactors,
    StageFactors,
    dual_gradient,
    dual_gradient_kkt,
    costate,
    null_basis,
    particular_inputs,
)
from .prox import prox_dist, proj_box, proj_lower, prox_g, prox_gconj
from .apg import APGResult, apg, theta_next, theta_of, beta_sequence
from .objective import primal_cost, violations, dual_objective, g_conj, g_value, \
    split_residual, split_gap
from .stepsize import lipschitz_power, lipschitz_dense, dual_hessian_dense
from .closed_loop import LoopResult, closed_loop
from .tree_build import BuiltTree, build_tree, forward_selection

__all__ = [
    "TreeIndex",
    "NodeFactors",
    "StageFactors",
    "dual_gradient",
    "dual_gradient_kkt",
    "costate",
    "null_basis",
    "particular_inputs",
    "prox_dist",
    "proj_box",
    "proj_lower",
    "prox_g",
    "prox_gconj",
    "APGResult",
    "apg",
    "theta_next",
    "theta_of",
    "beta_sequence",
    "primal_cost",
    "violations",
    "dual_objective",
    "g_conj",
    "split_residual",
    "split_gap",
    "g_value",
    "lipschitz_power",
    "lipschitz_dense",
    "dual_hessian_dense",
    "LoopResult",
    "closed_loop",
    "BuiltTree",
    "build_tree",
    "forward_selection",
]
