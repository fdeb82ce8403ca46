"""The single-workgroup cycle of the small pressure levels (p_small = 1) runs the
passes of the pass-by-pass cycle (p_small = 0) in the same order with the same
arithmetic: after two preconditioned FGMRES iterations the iterates agree to
rounding, and converged solves take the same number of iterations.  Cases cover
cubes whose small hierarchy starts at 16^3 with the coarsest dense matrix in
LDS (at 32^3 that is the second level, with its own smoothing counts), a wave-tank shape whose dense matrix (288^2) stays in global memory,
V-cycles, W-cycles at every level or on the finest two, pre- or post-smoothing
only, linear prolongation, FP64 and FP32 multigrid."""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_solve, rel

pytestmark = pytest.mark.gpu

CASES = [("headline_recipe_64cubed", lambda: W.config5(n_cells=64)),
         ("dam_break_64cubed", lambda: W.config3(scale=2)),
         ("wave_tank_256x24x24", lambda: W.config4(scale=4)),
         # the small-level kernel starts at the second level here, so its pass list
         # carries that level's own smoothing counts (p_nu_second)
         ("headline_recipe_32cubed", lambda: W.config5(n_cells=32))]
OPTS = [dict(), dict(p_wdepth=0), dict(p_gamma=1), dict(nu1=0, nu2=2, p_wdepth=0),
        dict(nu1=3, nu2=1, p_prolong=1)]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("opts", OPTS, ids=["default", "wcycle_all", "vcycle", "post_only", "lin_prolong"])
@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
def test_small_cycle_matches_pass_by_pass(name, maker, opts, precision):
    prob = maker()
    print("small cycle", name, prob.n, opts, "precision", precision, flush=True)
    a = gpu_solve(prob, tol=1e-30, max_iters=2, precision=precision, p_small=0, **opts)
    b = gpu_solve(prob, tol=1e-30, max_iters=2, precision=precision, p_small=1, **opts)
    assert a[3].small_level == -1 and b[3].small_level >= 1, (a[3].as_dict(), b[3].as_dict())
    assert a[3].iters == b[3].iters == 2
    bound = 1e-11 if precision == 0 else 1e-4
    errs = [rel(b[0][c], a[0][c]) for c in range(prob.dim)] + [rel(b[1], a[1])]
    print("  small level", b[3].small_level, "of", b[3].levels, "rel diff", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) <= bound


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
def test_small_cycle_same_iterations_to_tolerance(name, maker):
    prob = maker()
    a = gpu_solve(prob, p_small=0)
    b = gpu_solve(prob, p_small=1)
    assert a[2] == 0 and b[2] == 0
    assert a[3].iters == b[3].iters, (a[3].as_dict(), b[3].as_dict())
    assert rel(b[1] - b[1].mean(), a[1] - a[1].mean()) <= 1e-9
