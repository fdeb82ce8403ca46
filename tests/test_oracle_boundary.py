"""Pins of the wave tank's boundaries in the oracle (oracle/boundary.py and the
open top of oracle/assemble.py): the Dirichlet-top Poisson spectrum in closed
form, second-order convergence of a manufactured solution with inflow on
x = 0 and the open top, the global mass balance, and the Stokes wave formulas
(divergence-free, no flow through the bottom, the linear kinematic condition,
the textbook second-order amplitude, and the paper's printed wave cases, whose
periods and wavelengths the dispersion relation must reproduce to the printed
digits: tests/golden/stokes_wave_cases.txt).  CPU only."""
import math

import numpy as np
import pytest
import sympy as S

import workloads as W
from oracle import assemble as A
from oracle import boundary as B
from oracle import direct as D
from tests.golden_data import paper_wave_cases


def test_dirichlet_top_poisson_spectrum():
    """A column of N cells, Neumann bottom, zero pressure on the top face: the
    eigenvalues of -D beta G are 4 beta / h^2 sin^2((2m+1) pi / (4N))."""
    N, h, beta = 12, 0.1, 0.37
    g = A.OGrid(2, (1, N, 1), (h, h, h), open_top=True)
    rho = [np.full(W.face_shape((1, N, 1), c), 1.0 / beta) for c in range(2)]
    Lp = A.pressure_laplacian(g, rho).toarray()
    ev = np.sort(np.linalg.eigvalsh(0.5 * (Lp + Lp.T)))
    want = np.sort(4 * beta / h ** 2 * np.sin((2 * np.arange(N) + 1) * np.pi / (4 * N)) ** 2)
    assert np.allclose(ev, want, rtol=1e-12, atol=0)
    assert np.allclose(Lp, Lp.T)


def test_open_top_unknowns_and_gradient():
    n, h = (3, 4, 1), (0.5, 0.25, 0.5)
    g = A.OGrid(2, n, h, open_top=True)
    rho = [np.ones(W.face_shape(n, c)) for c in range(2)]
    sys = A.assemble(g, rho, np.ones(W.cell_shape(n)), 1.0)
    # v unknowns: interior y-faces plus the top ones, u: interior x-faces
    assert sys.sizes == [2 * 4, 3 * 4, 12]
    G = sys.G.toarray()
    Dm = sys.D.toarray()
    nu = sys.sizes[0]
    # top v-face of column i: G = -2 p / h_y of the cell below; D has +1/h_y
    for i in range(3):
        row = nu + 3 * 3 + i                  # v unknowns ordered (j = 1..4) x (i)
        cell = 3 * 3 + i
        assert G[row, cell] == pytest.approx(-2.0 / h[1])
        assert Dm[cell, row] == pytest.approx(1.0 / h[1])
        assert np.count_nonzero(G[row]) == 1


X, Y = S.symbols("x y")


def _mms_open_top(N, dt=5e-3, theta=1.0):
    """Inflow on x = 0 (normal and vertical tangential velocity), no slip on the
    bottom and on x = 1, the open top at y = 1: u = psi_y, v = -psi_x with
    psi = (1 - x)^2 y^2 (3 - 2 y) (u = 0 and d v / d y = 0 on the top), and
    p = cos(pi x) cos(pi y / 2) (zero on the top)."""
    psi = (1 - X) ** 2 * Y ** 2 * (3 - 2 * Y)
    u = [S.diff(psi, Y), -S.diff(psi, X)]
    p = S.cos(S.pi * X) * S.cos(S.pi * Y / 2)
    rho = 1 + S.Rational(1, 2) * S.sin(S.pi * X + S.Rational(3, 10)) * S.cos(S.pi * Y)
    mu = 1 + S.Rational(1, 2) * S.cos(S.pi * X) * S.sin(S.pi * Y + S.Rational(1, 5))
    coords = [X, Y]
    f = []
    for c in range(2):
        visc = sum(S.diff(mu * (S.diff(u[c], coords[d]) + S.diff(u[d], coords[c])), coords[d]) for d in range(2))
        f.append(rho / dt * u[c] - theta * visc + S.diff(p, coords[c]))
    lam = lambda e: S.lambdify((X, Y), e, "numpy")
    n, h = (N, N, 1), (1.0 / N,) * 3
    g = A.OGrid(2, n, h, open_top=True)
    rho_f, f_f, u_f = [], [], []
    for c in range(2):
        Xc, Yc, _ = W.face_coords(n, h, c)
        rho_f.append(np.broadcast_to(lam(rho)(Xc, Yc), Xc.shape).astype(float).copy())
        f_f.append(np.broadcast_to(lam(f[c])(Xc, Yc), Xc.shape).astype(float).copy())
        u_f.append(np.broadcast_to(lam(u[c])(Xc, Yc), Xc.shape).astype(float).copy())
    Xc, Yc, _ = W.cell_coords(n, h)
    mu_c = np.broadcast_to(lam(mu)(Xc, Yc), Xc.shape).astype(float).copy()
    p_c = np.broadcast_to(lam(p)(Xc, Yc), Xc.shape).astype(float).copy()
    yc = (np.arange(N) + 0.5) * h[1]
    yn = np.arange(N + 1) * h[1]
    un = np.broadcast_to(lam(u[0])(0.0 * yc, yc), yc.shape).astype(float)[None, :]
    ut = np.broadcast_to(lam(u[1])(0.0 * yn, yn), yn.shape).astype(float)[None, :]
    return g, rho_f, mu_c, dt, theta, f_f, u_f, p_c, un, ut


def _solve_open(g, rho_f, mu_c, dt, theta, f_f, un, ut):
    sys = A.assemble(g, rho_f, mu_c, dt, theta)
    lu, lp = B.inflow_lift(g, mu_c, theta, un, ut)
    fu = [f_f[c] - lu[c] for c in range(g.dim)]
    gp = np.zeros(g.cell_shape()) - lp
    x, _ = D.solve(sys, sys.pack(fu, gp), dense=False, has_null=False)
    return sys, sys.unpack(x)


def test_mms_inflow_open_top_second_order():
    errs = []
    for N in (16, 32, 64):
        g, rho_f, mu_c, dt, theta, f_f, u_f, p_c, un, ut = _mms_open_top(N)
        sys, (xu, xp) = _solve_open(g, rho_f, mu_c, dt, theta, f_f, un, ut)
        cell = g.h[0] * g.h[1]
        mask = [sys.sel[c].T @ np.ones(sys.sizes[c]) for c in range(2)]   # unknown faces
        eu = math.sqrt(sum(np.sum(((xu[c] - u_f[c]).ravel() * mask[c]) ** 2) for c in range(2)) * cell)
        ep = math.sqrt(np.sum((xp - p_c) ** 2) * cell)
        errs.append((eu, ep))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    print("MMS inflow + open top: errors", errs.tolist(), "rates", rates.tolist())
    assert np.all(rates[-1] >= 1.8), rates
    assert errs[-1, 0] < 1e-3 and errs[-1, 1] < 1e-2


def test_mass_balance_inflow_equals_top_outflow():
    g, rho_f, mu_c, dt, theta, f_f, u_f, p_c, un, ut = _mms_open_top(24)
    sys, (xu, xp) = _solve_open(g, rho_f, mu_c, dt, theta, f_f, un, ut)
    inflow = float(np.sum(un) * g.h[1])
    outflow = float(np.sum(xu[1][0, -1, :]) * g.h[0])
    assert outflow == pytest.approx(inflow, rel=1e-10)
    assert inflow > 0.5                                     # the manufactured flow does cross


# ------------------------------------------------------------------ Stokes wave
H_, D_, LAM_, G_ = 0.04, 0.5, 1.5, 9.81


def _omega():
    return B.dispersion_omega(B.wave_number(LAM_), D_, G_)


def test_stokes_wave_is_divergence_free_and_closed_at_the_bottom():
    om = _omega()
    x = np.linspace(0.0, 3.0, 301)
    y = np.linspace(-D_, 0.1, 121)
    Xg, Yg = np.meshgrid(x, y, indexing="ij")
    for t in (0.0, 0.37):
        dx = 1e-5
        up, _ = B.stokes_velocity(H_, D_, LAM_, om, G_, Xg + dx, Yg, t)
        um, _ = B.stokes_velocity(H_, D_, LAM_, om, G_, Xg - dx, Yg, t)
        _, vp = B.stokes_velocity(H_, D_, LAM_, om, G_, Xg, Yg + dx, t)
        _, vm = B.stokes_velocity(H_, D_, LAM_, om, G_, Xg, Yg - dx, t)
        div = (up - um + vp - vm) / (2 * dx)
        u0, _ = B.stokes_velocity(H_, D_, LAM_, om, G_, Xg, Yg, t)
        assert np.abs(div).max() <= 1e-6 * np.abs(u0).max() * B.wave_number(LAM_)
        _, vb = B.stokes_velocity(H_, D_, LAM_, om, G_, x, -D_, t)
        assert np.abs(vb).max() == 0.0


def test_stokes_wave_linear_kinematic_condition_and_second_order_amplitude():
    om = _omega()
    k = B.wave_number(LAM_)
    x = np.linspace(0.0, 1.5, 61)
    Hs = 1e-7                                   # second-order terms negligible
    for t in (0.0, 0.2, 0.9):
        dt = 1e-6
        deta = (B.stokes_eta(Hs, D_, LAM_, om, x, t + dt) - B.stokes_eta(Hs, D_, LAM_, om, x, t - dt)) / (2 * dt)
        _, v0 = B.stokes_velocity(Hs, D_, LAM_, om, G_, x, 0.0, t)
        assert np.allclose(v0, deta, rtol=1e-5, atol=1e-6 * Hs * om)
    # second harmonic of the elevation: (k H^2 / 16) cosh(kd) (2 + cosh 2kd) / sinh^3(kd)
    a2 = k * H_ ** 2 / 16 * np.cosh(k * D_) * (2 + np.cosh(2 * k * D_)) / np.sinh(k * D_) ** 3
    e = B.stokes_eta(H_, D_, LAM_, om, 0.0, 0.0)
    assert e == pytest.approx(H_ / 2 + a2, rel=1e-13)
    assert a2 == pytest.approx(W.stokes_wave_second_order_coeff(H_, D_, LAM_), rel=1e-12)


def test_boundary_heaviside():
    eps = 0.03
    phi = np.array([-1.0, -eps, 0.0, eps, 1.0])
    Hh = B.boundary_heaviside(phi, eps)
    assert np.allclose(Hh, [0.0, 0.0, 0.5, 1.0, 1.0], atol=1e-15)
    p = np.linspace(-eps, eps, 11)
    assert np.allclose(B.boundary_heaviside(p, eps) + B.boundary_heaviside(-p, eps), 1.0)


def test_stokes_inflow_drives_the_liquid_only():
    n, h = (16, 8, 32), (1 / 32,) * 3
    om = _omega()
    un, ut = B.stokes_inflow(3, n, h, H_, D_, LAM_, om, G_, 0.3, 0.5, 1.5)
    assert un.shape == (32, 8) and ut.shape == (33, 8)
    eta0 = B.stokes_eta(H_, D_, LAM_, om, 0.0, 0.3)
    zc = (np.arange(32) + 0.5) / 32 - 0.5
    eps = 1.5 / 32
    assert np.all(un[zc - eta0 > eps, :] == 0.0)            # air: not driven
    deep = zc - eta0 < -eps
    uc, _ = B.stokes_velocity(H_, D_, LAM_, om, G_, 0.0, zc, 0.3)
    assert np.allclose(un[deep, 0], uc[deep], rtol=1e-15)
    assert np.all(un[:, 0:1] == un)                         # uniform across y


def test_paper_wave_cases_satisfy_the_dispersion_relation():
    """Each printed (period, wavelength, depth) triple of the paper's wave cases
    satisfies the oracle's dispersion relation (eq. eq_disp) to the printed digits:
    the period the oracle gives for the wavelength rounded down by half a unit of
    its last printed digit, and for it rounded up, brackets the printed period
    widened by half a unit of its own last digit (the period grows with the
    wavelength).  A wrong depth inside tanh, a missing square root or k = 1 / lambda
    moves the period far outside that bracket."""
    g, cases = paper_wave_cases()
    assert g == 9.81 and [c[0] for c in cases] == ["A", "B", "C"]
    for name, d, _, t_c, lam_d in cases:
        half = 0.5 * 10.0 ** -len(lam_d.split(".")[1])
        scale = math.sqrt(d / g)

        def period(lam_over_d):
            return 2.0 * math.pi / B.dispersion_omega(B.wave_number(lam_over_d * d), d, g) / scale

        lo, hi = period(float(lam_d) - half), period(float(lam_d) + half)
        assert lo < hi, name
        assert lo <= t_c + 0.5e-4 and hi >= t_c - 0.5e-4, (name, lo, t_c, hi)
        # the bracket is tight: half a unit of the wavelength's last digit moves the
        # period by less than 1e-3 of sqrt(d / g)
        assert hi - lo < 1e-3, name


def test_paper_wave_case_a_velocity_scale():
    """Case A of the paper (Sec. 7.2) in the oracle's wave formulas: the crest
    elevation exceeds half the height by the second-order term, which is positive
    and below a tenth of the first-order amplitude (the case sits in the second-order
    Stokes regime), and the horizontal velocity under the crest at the still level
    is H g k / (2 omega) plus the second-order part."""
    g, cases = paper_wave_cases()
    _, d, h_d, _, lam_d = cases[0]
    H, lam = h_d * d, float(lam_d) * d
    k = B.wave_number(lam)
    om = B.dispersion_omega(k, d, g)
    crest = B.stokes_eta(H, d, lam, om, 0.0, 0.0)
    second = crest - 0.5 * H
    assert 0.0 < second < 0.1 * 0.5 * H
    trough = B.stokes_eta(H, d, lam, om, 0.5 * lam, 0.0)
    assert crest - trough == pytest.approx(H, rel=1e-12)   # the second harmonic cancels
    u_crest, v_crest = B.stokes_velocity(H, d, lam, om, g, 0.0, 0.0, 0.0)
    first = H * g * k / (2.0 * om)
    assert first < u_crest < 1.1 * first
    assert v_crest == pytest.approx(0.0, abs=1e-15)
