"""One time step of the built pieces, composed on the device and compared with
the same composition of oracle functions: coefficients from the level sets ->
Crank-Nicolson right-hand side with the well-balanced gravity force -> Stokes
solve with theta = 1/2 -> free-body rigid projection of the immersed sphere.
Config 3's geometry at 64^3 (water column, air, sphere rho_s 700) with a smooth
old velocity; both solves run to 1e-13.

Tolerance: the solution of the step is compared field by field (relative L2
1e-9, as the solve parity), the body velocity to 1e-8 relative (it is an
average of interpolated solution values).  The paper's static-cylinder example
(Sec. 8.4) is run for one step at its stated grid and time step."""
import numpy as np
import pytest

import workloads as W
from oracle import assemble as A
from oracle import coefficients as OC
from oracle import rigid as OR
from tests.gpu_util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_one_time_step_matches_oracle_chain(oracle_lib):
    import torch
    import paper_1901_07892_amd as S
    p = W.config3(scale=2)
    n, h, dt, theta = p.n, p.h, p.dt, 0.5
    gv = (0.0, 0.0, -9.81)
    fl = (W.RHO_WATER, p.rho_air, W.MU_WATER, W.MU_AIR, p.heaviside_cells)
    un = [0.05 * np.asarray(a) for a in p.rhs_u[:3]]
    for c in range(3):                                   # old velocity: zero on wall-normal faces
        for end in (0, -1):
            sl = [slice(None)] * 3
            sl[2 - c] = end
            un[c][tuple(sl)] = 0.0
    Xc, Yc, Zc = W.cell_coords(n, h)
    inside = p.psi[0] < 0
    X = np.stack([Xc[inside], Yc[inside], Zc[inside]], 1)
    dV = float(np.prod(h))
    xc = X.mean(0)

    # device chain
    print("one step on the device: coefficients, rhs, solve, rigid projection", flush=True)
    grid = S._binding.make_grid(3, n, h)
    rho = [torch.empty(W.face_shape(n, c), dtype=torch.float64, device="cuda") for c in range(3)]
    flow = [torch.empty_like(a) for a in rho]
    mu = torch.empty(W.cell_shape(n), dtype=torch.float64, device="cuda")
    S.stokes_coefficients(grid, S.make_fluids(*fl), to_dev(p.phi), [to_dev(q) for q in p.psi], p.rho_solid,
                          [W.MU_SOLID] * len(p.psi), rho, mu, flow)
    f = [torch.empty_like(a) for a in rho]
    S.stokes_explicit_rhs(grid, rho, mu, dt, theta, [to_dev(a) for a in un], f, flow, gv)
    s = S.StokesSolver(3, n, h, rho, mu, dt, visc_scale=theta)
    xu = [torch.zeros_like(a) for a in f]
    xp = torch.zeros_like(mu)
    st, stats = s.solve(f, torch.zeros_like(mu), 1e-13, xu, xp)
    torch.cuda.synchronize()
    assert st == 0 or (st == 1 and stats.rel_res_true <= 1e-12), stats.as_dict()
    s.close()
    ws = torch.empty(S.stokes_rigid_workspace_size(3, len(X)), dtype=torch.uint8, device="cuda")
    body = S.stokes_rigid_projection(grid, xu, to_dev(X), dV, 1, S.make_body(xc), ws)
    torch.cuda.synchronize()
    gu = [to_host(a) for a in xu]
    gp = to_host(xp)

    # oracle chain
    orho, omu, oflow = OC.coefficients(3, h, p.phi, p.psi, p.rho_solid, [W.MU_SOLID] * len(p.psi),
                                       fl[0], fl[1], fl[2], fl[3], fl[4])
    of = A.explicit_rhs(A.OGrid(3, tuple(n), tuple(h)), orho, omu, dt, theta, un, oflow, gv)
    ou, op, info = oracle_lib.solve(3, n, h, dt, theta, orho, omu, of, np.zeros(W.cell_shape(n)), 1e-13,
                                    max_iters=300)
    uc, Ur, Wr = OR.rigid_projection(ou, X, dV, xc, n, h, 3, True)

    for c in range(3):
        assert rel(gu[c], uc[c]) <= 1e-9, (c, rel(gu[c], uc[c]))
    assert rel(gp - gp.mean(), op - op.mean()) <= 1e-9
    np.testing.assert_allclose(list(body.u_r), Ur, rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(list(body.w_r), Wr, rtol=1e-8, atol=1e-12)


def test_paper_static_cylinder_one_step(oracle_lib):
    """The paper's well-balance example (Sec. 8.4, static cylinder on an air-water
    interface) for one time step at its stated sizes: a 5 x 5 tank on a 200 x 200
    grid, dt = 1 / (5 N), water below y = 2.5, a cylinder of diameter 1 at the
    centre with the water's density and viscosity, two cells of smearing, no slip,
    held at rest (prescribed rigid motion with U_b = 0).  From rest, one
    Crank-Nicolson step with the flow-only gravity force leaves the fluid at rest
    to rounding (|u| <= 1e-9 g dt) with the discrete hydrostatic pressure; the full
    density as the force (the solid's water density above the interface) drives a
    flow many orders larger.  Both chains equal the oracle's (relative L2 1e-9
    per field, as the solve parity)."""
    import torch
    import paper_1901_07892_amd as S
    N, L = 200, 5.0
    n, h = (N, N, 1), (L / N, L / N, L / N)
    dt, theta, g = 1.0 / (5 * N), 0.5, -9.81
    gv = (0.0, g, 0.0)
    fl = (W.RHO_WATER, W.RHO_AIR, W.MU_WATER, W.MU_AIR, 2.0)
    Xc, Yc, Zc = W.cell_coords(n, h)
    phi = Yc - 2.5
    psi = [W.sdf_sphere(Xc, Yc, Zc, (2.5, 2.5), 0.5, 2)]
    inside = psi[0] < 0
    X = np.stack([Xc[inside], Yc[inside]], 1)
    dV = h[0] * h[1]
    xc = (2.5, 2.5)
    grid = S._binding.make_grid(2, n, h)
    rho = [torch.empty(W.face_shape(n, c), dtype=torch.float64, device="cuda") for c in range(2)]
    flow = [torch.empty_like(a) for a in rho]
    mu = torch.empty(W.cell_shape(n), dtype=torch.float64, device="cuda")
    S.stokes_coefficients(grid, S.make_fluids(*fl), to_dev(phi), [to_dev(q) for q in psi], [W.RHO_WATER],
                          [W.MU_WATER], rho, mu, flow)
    orho, omu, oflow = OC.coefficients(2, h, phi, psi, [W.RHO_WATER], [W.MU_WATER], *fl)
    un = [np.zeros(W.face_shape(n, c)) for c in range(2)]
    s = S.StokesSolver(2, n, h, rho, mu, dt, visc_scale=theta)
    ws = torch.empty(S.stokes_rigid_workspace_size(2, len(X)), dtype=torch.uint8, device="cuda")
    umax = {}
    for name, force, oforce in (("flow", flow, oflow), ("full", rho, orho)):
        print("static cylinder, %s gravity: device chain" % name, flush=True)
        f = [torch.empty_like(a) for a in rho]
        S.stokes_explicit_rhs(grid, rho, mu, dt, theta, [to_dev(a) for a in un], f, force, gv)
        xu = [torch.zeros_like(a) for a in f]
        xp = torch.zeros_like(mu)
        st, stats = s.solve(f, torch.zeros_like(mu), 1e-13, xu, xp)
        torch.cuda.synchronize()
        assert st == 0 or (st == 1 and stats.rel_res_true <= 1e-12), stats.as_dict()
        S.stokes_rigid_projection(grid, xu, to_dev(X), dV, 0, S.make_body(xc), ws)
        torch.cuda.synchronize()
        gu = [to_host(a) for a in xu]
        gp = to_host(xp)
        of = A.explicit_rhs(A.OGrid(2, n, h), orho, omu, dt, theta, un, oforce, gv)
        ou, op, info = oracle_lib.solve(2, n, h, dt, theta, orho, omu, of, np.zeros(W.cell_shape(n)), 1e-13,
                                        max_iters=400)
        uc, _, _ = OR.rigid_projection(ou, X, dV, np.array(xc), n, h, 2, False, np.zeros(3), np.zeros(3))
        umax[name] = max(np.abs(a).max() for a in gu) / (abs(g) * dt)
        print("  max |u| / (g dt) = %.3e" % umax[name], flush=True)
        if name == "flow":
            ph = np.zeros(W.cell_shape(n))
            fy = to_host(flow[1])                       # (1, N + 1, N): y-faces
            for j in range(1, N):
                ph[:, j, :] = ph[:, j - 1, :] + h[1] * fy[:, j, :] * g
            assert rel(gp - gp.mean(), ph - ph.mean()) <= 1e-11
        else:
            for c in range(2):
                assert rel(gu[c], uc[c]) <= 1e-9, (c, rel(gu[c], uc[c]))
            assert rel(gp - gp.mean(), op - op.mean()) <= 1e-9
    s.close()
    assert umax["flow"] <= 1e-9
    assert umax["full"] > 1e4 * max(umax["flow"], 1e-14)
