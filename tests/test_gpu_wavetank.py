"""GPU parity of the wave tank's boundaries (open top and Stokes-wave inflow)
with the oracle (oracle/assemble.py open top, oracle/boundary.py).

Operator: stokes_apply with open_top against the assembled matrix, element by
element (1e-13 of max |y|).  Inflow data and right-hand-side lift against the
oracle's (1e-13).  Solve: the wave tank of config 4 (its Stokes-wave free
surface, floating box, density ratio 833) with the open top and the Stokes
inflow, against SuperLU on the oracle's system at tol 1e-13 (relative L2
<= 1e-9 per field; the pressure has no free constant), in 2D and 3D; FP32
multigrid to tol 1e-8 with the residual confirmed by the oracle's matrix; and
the stated size 1024x96x96, whose inflow must leave through the open top."""
import numpy as np
import pytest

import workloads as W
from oracle import assemble as A
from oracle import boundary as B
from oracle import direct as D
from tests.golden_data import paper_wave_cases
from tests.gpu_util import gpu_apply, rel, solver_for, to_dev, to_host

pytestmark = pytest.mark.gpu

H_, DEPTH_, LAM_, G_ = 0.04, 0.5, 1.5, 9.81


def _omega():
    return B.dispersion_omega(B.wave_number(LAM_), DEPTH_, G_)


def _rand_problem(dim, n, h, seed, dt=1e-7):
    rng = np.random.default_rng(seed)
    rho = [rng.uniform(1.2, 1000.0, size=W.face_shape(n, a)) if a < dim else None for a in range(3)]
    mu = np.exp(rng.uniform(np.log(1.8e-5), np.log(1e-3), size=W.cell_shape(n)))
    rhs_u, _ = W.fourier_rhs(rng, dim, n, h)
    return W.Problem(name="rand", dim=dim, n=n, h=h, dt=dt, rho_faces=rho, mu=mu, rhs_u=rhs_u,
                     rhs_p=np.zeros(W.cell_shape(n)), tol=1e-10)


def _vector_with_top(prob, seed):
    xu, xp = W.random_vector(prob, prob.dim, seed)
    rng = np.random.default_rng(seed + 1)
    v = prob.dim - 1
    sl = [slice(None)] * 3
    sl[2 - v] = -1
    xu[v][tuple(sl)] = rng.standard_normal(xu[v][tuple(sl)].shape)
    return xu, xp


APPLY_CASES = [
    ("rand2d_ragged", 2, (13, 7, 1), (0.1, 0.07, 0.1)),
    ("rand3d_ragged", 3, (5, 9, 6), (0.2, 0.1, 0.15)),
    ("rand3d_min", 3, (2, 2, 2), (0.5, 0.5, 0.5)),
    ("rand3d_tiles", 3, (70, 20, 9), (0.01, 0.012, 0.011)),
]


@pytest.mark.parametrize("name,dim,n,h", APPLY_CASES)
@pytest.mark.parametrize("theta,matvec_z", [(1.0, 1), (0.5, 1), (1.0, 0)])
def test_apply_open_top_matches_oracle_matrix(name, dim, n, h, theta, matvec_z):
    prob = _rand_problem(dim, n, h, sum(n))
    print("apply open top", name, n, theta, matvec_z, flush=True)
    g = A.OGrid(dim, n, h, open_top=True)
    sys = A.assemble(g, prob.rho_faces[:dim], prob.mu, prob.dt, theta)
    xu, xp = _vector_with_top(prob, 5)
    yu, yp = gpu_apply(prob, xu, xp, theta, matvec_z=matvec_z, open_top=1)
    y_ref = sys.K @ sys.pack(xu, xp)
    y_gpu = sys.pack(yu, yp)
    assert np.abs(y_gpu - y_ref).max() <= 1e-13 * np.abs(y_ref).max()
    # the bottom faces of the vertical component are walls, the top ones unknowns
    v = dim - 1
    sl = [slice(None)] * 3
    sl[2 - v] = 0
    assert np.all(yu[v][tuple(sl)] == 0.0)
    sl[2 - v] = -1
    assert np.abs(yu[v][tuple(sl)]).max() > 0.0


@pytest.mark.parametrize("dim,n,h", [(2, (64, 24, 1), (1 / 24,) * 3), (3, (32, 6, 24), (1 / 24,) * 3)])
def test_wave_inflow_data_matches_oracle(dim, n, h):
    import torch
    import paper_1901_07892_amd as S
    om = _omega()
    grid = S._binding.make_grid(dim, n, h)
    nv, nl = n[dim - 1], (n[1] if dim == 3 else 1)
    un = torch.full((nv, nl), np.nan, dtype=torch.float64, device="cuda")
    ut = torch.full((nv + 1, nl), np.nan, dtype=torch.float64, device="cuda")
    for t in (0.0, 0.31, 1.7):
        S.stokes_wave_inflow(grid, S.make_wave(H_, DEPTH_, LAM_, om, G_, 1.5), t, un, ut)
        torch.cuda.synchronize()
        oun, out = B.stokes_inflow(dim, n, h, H_, DEPTH_, LAM_, om, G_, t, DEPTH_, 1.5)
        oun = oun.T if dim == 2 else oun                  # oracle 2D shape (1, Ny) -> (Ny, 1)
        out = out.T if dim == 2 else out
        scale = max(np.abs(oun).max(), np.abs(out).max())
        print("  t %.2f max |u_n| %.3e max diff %.1e %.1e" % (t, np.abs(oun).max(),
              np.abs(to_host(un) - oun).max(), np.abs(to_host(ut) - out).max()), flush=True)
        assert np.abs(to_host(un) - oun).max() <= 1e-13 * scale
        assert np.abs(to_host(ut) - out).max() <= 1e-13 * scale


@pytest.mark.parametrize("case", ["A", "B", "C"])
def test_wave_inflow_paper_cases_match_oracle(case):
    """The paper's printed wave cases (Sec. 7.2, Table tab_wave_cases, read from
    tests/golden/stokes_wave_cases.txt) on its coarsest wave-tank grid: 442 x 66
    cells over 68 d x 1.3 d with the still level 0.3 d below the top, one cell of
    smearing; the inflow data on x = 0 equal the oracle's within 1e-13."""
    import torch
    import paper_1901_07892_amd as S
    g, cases = paper_wave_cases()
    _, d, h_d, _, lam_d = [c for c in cases if c[0] == case][0]
    H, lam = h_d * d, float(lam_d) * d
    om = B.dispersion_omega(B.wave_number(lam), d, g)
    n, h = (442, 66, 1), (68.0 * d / 442, 1.3 * d / 66, 68.0 * d / 442)
    grid = S._binding.make_grid(2, n, h)
    un = torch.full((66, 1), np.nan, dtype=torch.float64, device="cuda")
    ut = torch.full((67, 1), np.nan, dtype=torch.float64, device="cuda")
    period = 2.0 * np.pi / om
    for t in (0.0, 0.37 * period, 2.9 * period):
        print("paper wave case", case, "t %.3f" % t, flush=True)
        S.stokes_wave_inflow(grid, S.make_wave(H, d, lam, om, g, 1.0), t, un, ut)
        torch.cuda.synchronize()
        oun, out = B.stokes_inflow(2, n, h, H, d, lam, om, g, t, d, 1.0)
        scale = max(np.abs(oun).max(), np.abs(out).max())
        assert scale > 0.0
        assert np.abs(to_host(un) - oun.T).max() <= 1e-13 * scale
        assert np.abs(to_host(ut) - out.T).max() <= 1e-13 * scale


@pytest.mark.parametrize("dim,n,h", [(2, (24, 16, 1), (0.05, 0.06, 0.05)), (3, (12, 10, 14), (0.05, 0.06, 0.04))])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_inflow_lift_matches_oracle(dim, n, h, theta):
    import torch
    import paper_1901_07892_amd as S
    prob = _rand_problem(dim, n, h, 9, dt=1.0)
    rng = np.random.default_rng(3)
    nv, nl = n[dim - 1], (n[1] if dim == 3 else 1)
    un = rng.standard_normal((nv, nl))
    ut = rng.standard_normal((nv + 1, nl))
    g = A.OGrid(dim, n, h, open_top=True)
    lu, lp = B.inflow_lift(g, prob.mu, theta, un.T if dim == 2 else un, ut.T if dim == 2 else ut)
    s = solver_for(prob, theta=theta, open_top=1, vel_levels=1)
    fu = [torch.zeros(W.face_shape(n, c), dtype=torch.float64, device="cuda") for c in range(dim)]
    fp = torch.zeros(W.cell_shape(n), dtype=torch.float64, device="cuda")
    S.stokes_inflow_lift(s.ctx, to_dev(un), to_dev(ut), fu, fp)
    torch.cuda.synchronize()
    s.close()
    scale = max([np.abs(a).max() for a in lu] + [np.abs(lp).max()])
    for c in range(dim):
        assert np.abs(to_host(fu[c]) + lu[c]).max() <= 1e-13 * scale, c
    assert np.abs(to_host(fp) + lp).max() <= 1e-13 * scale


def _tank_rhs(prob, t):
    """The workload's right-hand side with the Stokes inflow lifted (oracle side)."""
    g = A.OGrid(prob.dim, prob.n, prob.h, open_top=True)
    un, ut = B.stokes_inflow(prob.dim, prob.n, prob.h, H_, DEPTH_, LAM_, _omega(), G_, t, DEPTH_, 1.5)
    lu, lp = B.inflow_lift(g, prob.mu, 1.0, un, ut)
    return g, [prob.rhs_u[c] - lu[c] for c in range(prob.dim)], prob.rhs_p - lp


def _gpu_tank(prob, t, tol, **opts):
    """GPU: inflow data, lift and solve, all through the C-ABI."""
    import torch
    import paper_1901_07892_amd as S
    s = solver_for(prob, open_top=1, **opts)
    dim, n = prob.dim, prob.n
    nv, nl = n[dim - 1], (n[1] if dim == 3 else 1)
    un = torch.zeros((nv, nl), dtype=torch.float64, device="cuda")
    ut = torch.zeros((nv + 1, nl), dtype=torch.float64, device="cuda")
    S.stokes_wave_inflow(s.grid, S.make_wave(H_, DEPTH_, LAM_, _omega(), G_, 1.5), t, un, ut)
    rhs_u = [to_dev(f) for f in prob.rhs_u[:dim]]
    rhs_p = to_dev(prob.rhs_p)
    S.stokes_inflow_lift(s.ctx, un, ut, rhs_u, rhs_p)
    xu = [torch.zeros_like(f) for f in rhs_u]
    xp = torch.zeros_like(rhs_p)
    st, stats = s.solve(rhs_u, rhs_p, tol, xu, xp)
    torch.cuda.synchronize()
    out = [to_host(a) for a in xu], to_host(xp), st, stats, to_host(un)
    s.close()
    return out


TANK_CASES = [
    ("config4_2d_128x12", lambda: W.config4_2d(128, 12)),
    ("config4_2d_512x48", lambda: W.config4_2d(512, 48)),
    ("config4_128x12x12", lambda: W.config4(scale=8)),
]


@pytest.mark.parametrize("name,maker", TANK_CASES)
def test_wave_tank_solve_matches_direct(name, maker):
    prob = maker()
    print("wave tank", name, prob.n, flush=True)
    g, fu, fp = _tank_rhs(prob, 0.3)
    sys = A.assemble(g, prob.rho_faces[:prob.dim], prob.mu, prob.dt, 1.0)
    x, _ = D.solve(sys, sys.pack(fu, fp), dense=False, has_null=False)
    ru, rp = sys.unpack(x)
    xu, xp, st, stats, _ = _gpu_tank(prob, 0.3, 1e-13, max_iters=400)
    print("  status", st, "iters", stats.iters, "res", stats.rel_res_true, flush=True)
    assert st == 0 or (st == 1 and stats.rel_res_true <= 1e-12), stats.as_dict()
    errs = [rel(xu[c], ru[c]) for c in range(prob.dim)] + [rel(xp, rp)]
    print("  rel errors per field", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= 1e-9, errs
    v = prob.dim - 1
    sl = [slice(None)] * 3
    sl[2 - v] = -1
    assert np.abs(xu[v][tuple(sl)]).max() > 0.0          # flow through the open top


@pytest.mark.parametrize("name,maker", [TANK_CASES[1], TANK_CASES[2]])
def test_wave_tank_fp32_multigrid_residual_by_oracle(name, maker):
    prob = maker()
    print("wave tank FP32 multigrid", name, prob.n, flush=True)
    g, fu, fp = _tank_rhs(prob, 0.3)
    sys = A.assemble(g, prob.rho_faces[:prob.dim], prob.mu, prob.dt, 1.0)
    xu, xp, st, stats, _ = _gpu_tank(prob, 0.3, prob.tol, precision=1)
    print("  status", st, "iters", stats.iters, "res", stats.rel_res_true, flush=True)
    assert st == 0
    b = sys.pack(fu, fp)
    r = b - sys.K @ sys.pack(xu, xp)
    nv = sys.n_vel
    w = stats.sigma ** 2
    res_w = np.sqrt((np.sum(r[:nv] ** 2) + w * np.sum(r[nv:] ** 2)) / (np.sum(b[:nv] ** 2) + w * np.sum(b[nv:] ** 2)))
    res_p = np.linalg.norm(r) / np.linalg.norm(b)
    print("  oracle residual weighted %.2e plain %.2e" % (res_w, res_p), flush=True)
    assert res_w <= 1.01 * prob.tol and res_p <= prob.tol


def test_wave_tank_full_size_mass_balance():
    """Config 4 at 1024x96x96 with the open top and the Stokes inflow, FP64 to tol 1e-8:
    converges in the solver's usual handful of iterations, and the discrete volume
    entering through x = 0 leaves through the open top."""
    prob = W.config4()
    print("wave tank full size", prob.n, flush=True)
    prob.rhs_u = [np.zeros_like(f) for f in prob.rhs_u]     # the inflow alone drives the flow
    xu, xp, st, stats, un = _gpu_tank(prob, 0.3, 1e-11)
    print("  status", st, "iters", stats.iters, "res", stats.rel_res_true, "ms", stats.ms_total, flush=True)
    assert st == 0 and stats.iters <= 12
    hx, hy, hz = prob.h
    inflow = float(un.sum()) * hy * hz
    outflow = float(xu[2][-1].sum()) * hx * hy
    print("  inflow %.6e outflow %.6e" % (inflow, outflow), flush=True)
    assert abs(inflow) > 1e-4
    assert abs(outflow - inflow) <= 1e-5 * abs(inflow)


def test_open_top_needs_the_diagonal_velocity_step():
    import paper_1901_07892_amd as S
    prob = _rand_problem(3, (8, 8, 8), (0.125,) * 3, 1, dt=100.0)     # viscous dominated
    with pytest.raises(S.StokesError) as e:
        solver_for(prob, open_top=1)
    assert e.value.status == -1 and "open_top" in str(e.value)
