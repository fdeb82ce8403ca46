"""GPU parity: the HIP path (through the C-ABI) against the oracle.

Operator: stokes_apply against the oracle's assembled matrix and its C stencil
loop, element by element.  Solve: the solution of the linear system against
the oracle's direct solves (2D, small 3D) and the oracle's FGMRES (larger 3D),
relative L2 <= 1e-9 per field (each velocity component, mean-free pressure) at
tol 1e-13.  Full size: the oracle's own operator evaluates the residual of
the GPU solution.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble as A
from oracle import direct as D
from tests.gpu_util import gpu_apply, gpu_solve, rel

pytestmark = pytest.mark.gpu


def _prob_random_coeffs(dim, n, h, seed, dt=1e-3):
    rng = np.random.default_rng(seed)
    rho = [rng.uniform(1.2, 1000.0, size=W.face_shape(n, a)) if a < dim else None for a in range(3)]
    mu = np.exp(rng.uniform(np.log(1.8e-5), np.log(1e-3), size=W.cell_shape(n)))
    rhs_u, _ = W.fourier_rhs(rng, dim, n, h)
    return W.Problem(name="rand", dim=dim, n=n, h=h, dt=dt, rho_faces=rho, mu=mu, rhs_u=rhs_u,
                     rhs_p=np.zeros(W.cell_shape(n)), tol=1e-10)


APPLY_CASES = [
    ("config1", lambda: W.config1()),
    ("config3_16", lambda: W.config3(scale=8)),
    ("config4_64x6x6", lambda: W.config4(scale=16)),
    ("rand2d_ragged", lambda: _prob_random_coeffs(2, (13, 7, 1), (0.1, 0.07, 0.1), 1, dt=1e-7)),
    ("rand3d_ragged", lambda: _prob_random_coeffs(3, (5, 9, 6), (0.2, 0.1, 0.15), 2, dt=1e-7)),
    ("rand3d_min", lambda: _prob_random_coeffs(3, (2, 2, 2), (0.5, 0.5, 0.5), 3, dt=1e-7)),
]


@pytest.mark.parametrize("name,maker", APPLY_CASES)
@pytest.mark.parametrize("theta,matvec_z", [(1.0, 1), (0.5, 1), (1.0, 0)])
def test_apply_matches_oracle_matrix(name, maker, theta, matvec_z):
    prob = maker()
    print("apply", name, prob.n, theta, matvec_z, flush=True)
    sys = A.assemble(A.OGrid(prob.dim, prob.n, prob.h), prob.rho_faces, prob.mu, prob.dt, theta)
    xu, xp = W.random_vector(prob, prob.dim, 77)
    yu, yp = gpu_apply(prob, xu, xp, theta, matvec_z=matvec_z)
    y_ref = sys.K @ sys.pack(xu, xp)
    y_gpu = sys.pack(yu, yp)
    scale = np.abs(y_ref).max()
    assert np.abs(y_gpu - y_ref).max() <= 1e-13 * scale
    # wall-normal entries are written as zero
    for c in range(prob.dim):
        sl = [slice(None)] * 3
        for end in (0, -1):
            sl[2 - c] = end
            assert np.all(yu[c][tuple(sl)] == 0.0)


def test_apply_full_size_against_stencil_loop(oracle_lib):
    """The headline 256^3 workload: GPU stokes_apply equals the C oracle loop everywhere."""
    prob = W.config5()
    print("apply full", prob.n, flush=True)
    xu, xp = W.random_vector(prob, 3, 5)
    yu, yp = gpu_apply(prob, xu, xp)
    ou, op = oracle_lib.apply_problem(prob, xu, xp)
    for c in range(3):
        assert np.abs(yu[c] - ou[c]).max() <= 1e-13 * np.abs(ou[c]).max()
    assert np.abs(yp - op).max() <= 1e-13 * np.abs(op).max()


def _converged_or_stagnated(st, stats):
    """Parity runs ask for tol 1e-13, at the floor of FP64 residual evaluation for
    the larger grids: accept a solve that stagnated (status NOT_CONVERGED) below
    1e-12; the field errors below are the gate."""
    assert st == 0 or (st == 1 and stats.rel_res_true <= 1e-12), (st, stats.as_dict())


def _check_solution(prob, xu, xp, ru, rp, tol=1e-9):
    errs = [rel(xu[c], ru[c]) for c in range(prob.dim)]
    errs.append(rel(xp - xp.mean(), rp - rp.mean()))
    print("  rel errors per field", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= tol, errs


@pytest.mark.parametrize("name,maker", [
    ("config1_64", lambda: W.config1()),
    ("config2_128", lambda: W.config2(scale=4)),
    ("config2_512", lambda: W.config2()),
    ("config1_ragged_48x40", lambda: W.make_problem("r", 2, (48, 40, 1), (1 / 48, 1 / 40, 1 / 48), 1e-4, 1e-10,
                                                    lambda X, Y, Z: Y - 0.5, [], 5)),
    ("config1_nocoarsen_33x17", lambda: W.make_problem("r", 2, (33, 17, 1), (1 / 33, 1 / 17, 1 / 33), 1e-4, 1e-10,
                                                       lambda X, Y, Z: Y - 0.37, [], 6)),
    ("config3_16", lambda: W.config3(scale=8)),
])
@pytest.mark.parametrize("precision", [0])
def test_solve_matches_direct(name, maker, precision):
    prob = maker()
    print("solve", name, prob.n, flush=True)
    sys = A.from_problem(prob)
    ru, rp = D.solve_problem(prob, sys)
    xu, xp, st, stats = gpu_solve(prob, tol=1e-13, precision=precision, max_iters=400)
    print("  status", st, "iters", stats.iters, "res", stats.rel_res_true, flush=True)
    _converged_or_stagnated(st, stats)
    _check_solution(prob, xu, xp, ru, rp)


# Oracle solutions at tol 1e-13, kept for the session: the FP64 parity test and the
# FP32-multigrid error statement of one workload share one oracle solve.
_ORACLE = {}


def _oracle_solution(oracle_lib, name, prob):
    if name not in _ORACLE:
        # restart 20 keeps the oracle's Krylov basis within host memory at the full sizes
        ou, op, info = oracle_lib.solve_problem(prob, tol=1e-13, max_iters=400, restart=20)
        print("  oracle: iters", info["iters"], "res", info["rel_res_true"], "solve s %.1f" % info["solve_s"],
              flush=True)
        assert info["status"] == 0 or info["rel_res_true"] <= 1e-12, info
        _ORACLE[name] = (ou, op, info)
    return _ORACLE[name]


ORACLE_CASES = [
    ("config3_64", lambda: W.config3(scale=2)),
    ("config4_256x24x24", lambda: W.config4(scale=4)),
    ("config5_64", lambda: W.config5(n_cells=64)),
    # finest level of 884,736 cells: the pipelined fused sweep (levels between 2^18 and 2^20 cells)
    ("config5_96", lambda: W.config5(n_cells=96)),
    # config 3 at its stated 128^3: the finest level runs the 64x16 fused sweep and the
    # z-marching residual + restriction
    ("config3_128", lambda: W.config3()),
    # config 4's geometry at half its stated size per axis (1,179,648 cells: the 64x16
    # fused sweep on the finest level); the stated size is checked below by the
    # oracle's operator, as its oracle FGMRES at tol 1e-13 takes minutes of host time
    ("config4_512x48x48", lambda: W.config4(scale=2)),
]


@pytest.mark.parametrize("name,maker", ORACLE_CASES)
def test_solve_matches_oracle_fgmres(oracle_lib, name, maker):
    prob = maker()
    print("solve", name, prob.n, flush=True)
    ou, op, info = _oracle_solution(oracle_lib, name, prob)
    xu, xp, st, stats = gpu_solve(prob, tol=1e-13, max_iters=400)
    print("  status", st, "iters", stats.iters, "oracle iters", info["iters"], flush=True)
    _converged_or_stagnated(st, stats)
    _check_solution(prob, xu, xp, ou, op)


def _oracle_residuals(oracle_lib, prob, xu, xp):
    """Relative residual of (xu, xp) by the oracle's own operator, in the plain
    2-norm and in the norm weighted by the oracle's continuity weight; the
    right-hand side's pressure block with its mean removed, as both solvers do."""
    sigma = oracle_lib.auto_sigma(prob)
    yu, yp = oracle_lib.apply_problem(prob, xu, xp)
    r2 = sum(np.sum((prob.rhs_u[c] - yu[c]) ** 2) for c in range(prob.dim))
    b2 = sum(np.sum(prob.rhs_u[c] ** 2) for c in range(prob.dim))
    g = prob.rhs_p - prob.rhs_p.mean()
    rp2 = np.sum((g - yp) ** 2)
    g2 = np.sum(g ** 2)
    plain = np.sqrt((r2 + rp2) / (b2 + g2))
    weighted = np.sqrt((r2 + sigma ** 2 * rp2) / (b2 + sigma ** 2 * g2))
    return plain, weighted, sigma


def test_config4_full_size_residual_by_oracle(oracle_lib):
    """Config 4 at its stated 1024x96x96, FP64 at tol 1e-13: the oracle's operator and
    its own continuity weight confirm the residual of the GPU solution in both norms
    (with the kernel-level parity at this size in test_gpu_pressure_ops.py)."""
    prob = W.config4()
    print("config 4 full size", prob.n, flush=True)
    xu, xp, st, stats = gpu_solve(prob, tol=1e-13, max_iters=400)
    print("  status", st, "iters", stats.iters, "res", stats.rel_res_true, flush=True)
    _converged_or_stagnated(st, stats)
    plain, weighted, _ = _oracle_residuals(oracle_lib, prob, xu, xp)
    print("  oracle residual plain %.2e weighted %.2e" % (plain, weighted), flush=True)
    assert plain <= 1e-12 and weighted <= 1e-12


FP32_CASES = [
    ("config2_512", lambda: W.config2()),
    ("config3_128", lambda: W.config3()),
    ("config4_512x48x48", lambda: W.config4(scale=2)),
    ("config4_1024x96x96", lambda: W.config4()),
]


@pytest.mark.parametrize("name,maker", FP32_CASES)
def test_fp32_multigrid_at_stated_sizes(oracle_lib, name, maker):
    """FP32 multigrid inside FP64 FGMRES at the workloads' stated sizes and tol: the
    oracle's operator confirms the FP64 residual, and the error against the oracle's
    FP64 solution (tol 1e-13) is stated."""
    prob = maker()
    print("FP32 multigrid", name, prob.n, "tol", prob.tol, flush=True)
    if prob.dim == 2:
        ru, rp = D.solve_problem(prob, A.from_problem(prob))
    elif name == "config4_1024x96x96":
        ru = rp = None           # residual only at the stated size (see above)
    else:
        ru, rp, _ = _oracle_solution(oracle_lib, name, prob)
    xu, xp, st, stats = gpu_solve(prob, precision=1)
    print("  status", st, "iters", stats.iters, "res", stats.rel_res_true, flush=True)
    assert st == 0
    plain, weighted, _ = _oracle_residuals(oracle_lib, prob, xu, xp)
    print("  oracle residual plain %.2e weighted %.2e" % (plain, weighted), flush=True)
    assert plain <= 1.01 * prob.tol and weighted <= 1.01 * prob.tol
    if ru is None:
        return
    errs = [rel(xu[c], ru[c]) for c in range(prob.dim)] + [rel(xp - xp.mean(), rp - rp.mean())]
    print("  FP32 multigrid: rel error per field vs the oracle's FP64 solution",
          ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= 1e-5, errs


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_solve_residual_by_oracle(oracle_lib, precision):
    """256^3 density ratio 1000 at tol 1e-8, in the configuration the benchmark times:
    the oracle's independent operator and its own continuity weight confirm the
    returned residual, in the weighted and the plain 2-norm."""
    prob = W.config5()
    print("full solve", prob.n, "precision", precision, flush=True)
    xu, xp, st, stats = gpu_solve(prob, precision=precision)
    print("  status", st, "iters", stats.iters, "res", stats.rel_res_true, "plain", stats.rel_res_plain,
          "ms", stats.ms_total, flush=True)
    assert st == 0
    plain, weighted, sigma = _oracle_residuals(oracle_lib, prob, xu, xp)
    print("  oracle residual plain %.3e weighted %.3e (sigma %.6g, GPU %.6g)" % (plain, weighted, sigma, stats.sigma),
          flush=True)
    assert plain <= prob.tol
    assert weighted <= 1.01 * prob.tol
    # the plain norm involves no weight: the GPU's own figure must agree with the oracle's
    assert abs(plain - stats.rel_res_plain) <= 1e-3 * prob.tol + 1e-2 * plain
    assert abs(xp.mean()) <= 1e-12 * np.abs(xp).max()
