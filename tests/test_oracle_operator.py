"""Pins of the oracle's discrete operator (O1 assembly, O2 stencil loop).

Each pin checks the oracle against something other than itself: matrix
symmetry (the strain-rate form with G = -D^T must give a symmetric saddle
point matrix), Fourier symbols of the constant-coefficient periodic operator
(closed forms), a 1D shear reduction solved by the Thomas algorithm, and the
spectrum of the variable-coefficient Poisson operator.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assemble as A
from oracle import direct as D


def _rand_coeffs(g, seed, rho_range=(1.2, 1000.0), mu_range=(1.8e-5, 1e-3)):
    rng = np.random.default_rng(seed)
    rho = [rng.uniform(*rho_range, size=g.comp_shape(c)) for c in range(g.dim)]
    mu = np.exp(rng.uniform(np.log(mu_range[0]), np.log(mu_range[1]), size=g.cell_shape()))
    return rho, mu


@pytest.mark.parametrize("dim,n,theta", [(2, (7, 5, 1), 1.0), (2, (6, 6, 1), 0.5),
                                         (3, (5, 4, 3), 1.0), (3, (4, 6, 5), 0.5)])
def test_symmetric_saddle_point(dim, n, theta):
    h = (0.3, 0.2, 0.25)
    g = A.OGrid(dim, n, h)
    rho, mu = _rand_coeffs(g, 3)
    s = A.assemble(g, rho, mu, dt=1e-3, theta=theta)
    K = s.K
    asym = abs(K - K.T).max() / abs(K).max()
    assert asym <= 1e-14
    # G = -D^T exactly (structural)
    assert abs(s.G + s.D.T).max() == 0.0
    # A is positive definite (mass + viscous dissipation)
    ev = np.linalg.eigvalsh(s.A.toarray())
    assert ev.min() > 0.0


@pytest.mark.parametrize("dim,n,seed", [(2, (9, 7, 1), 1), (3, (6, 5, 4), 2), (3, (3, 3, 3), 3),
                                         (2, (1, 4, 1), 4)])
def test_stencil_loop_matches_assembly(oracle_lib, dim, n, seed):
    """O2 (independent C stencil loop) equals O1 (Kronecker assembly) on random vectors."""
    h = (0.1, 0.13, 0.07)[:dim] + ((0.1,) if dim == 2 else ())
    g = A.OGrid(dim, n, h)
    rho, mu = _rand_coeffs(g, seed)
    for theta in (1.0, 0.5):
        s = A.assemble(g, rho, mu, dt=2e-4, theta=theta)
        xu, xp = W.random_vector(n, dim, seed + 10)
        yu, yp = oracle_lib.apply(dim, n, h, 2e-4, theta, rho, mu, xu[:dim], xp)
        y1 = s.K @ s.pack(xu, xp)
        y2 = s.pack(yu, yp)
        assert np.linalg.norm(y1 - y2) <= 1e-14 * np.linalg.norm(y1)
        # wall-normal entries come back as zero
        for c in range(dim):
            sl = [slice(None)] * 3
            sl[2 - c] = 0
            assert np.all(yu[c][tuple(sl)] == 0.0)


def _mode(g, k, comp):
    """exp(2 pi i sum_d k_d x_d / L_d) on component comp's faces (comp None: cells), periodic grid."""
    xs = []
    for a in range(3):
        if a < g.dim:
            N, hh = g.n[a], g.h[a]
            if comp == a:
                xs.append(np.arange(N) * hh)
            else:
                xs.append((np.arange(N) + 0.5) * hh)
        else:
            xs.append(np.array([0.0]))
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    Lx = [g.n[a] * g.h[a] for a in range(3)]
    ph = k[0] * X / Lx[0] + k[1] * Y / Lx[1] + (k[2] * Z / Lx[2] if g.dim == 3 else 0.0)
    return np.exp(2j * np.pi * ph)


@pytest.mark.parametrize("dim", [2, 3])
def test_fourier_symbols(dim):
    """Constant coefficients on a periodic grid: every block is diagonal in Fourier space.

    A_cc = rho/dt + theta mu (8 s_c^2/h_c^2 + sum_{d != c} 4 s_d^2/h_d^2),
    A_cd = 4 theta mu s_c s_d / (h_c h_d), G_c = (2i/h_c) s_c, -D_c = -(2i/h_c) s_c,
    with s_d = sin(pi k_d h_d); the viscous part is mu (Lap + grad div).
    """
    n = (8, 6, 5)[:dim] + ((1,) if dim == 2 else ())
    L = (1.0, 0.9, 1.1)
    h = tuple(L[a] / n[a] for a in range(3))
    g = A.OGrid(dim, n, h, periodic=(True, True, True))
    rho0, mu0, dt, th = 7.0, 0.3, 0.05, 0.8
    rho = [np.full(g.comp_shape(c), rho0) for c in range(dim)]
    mu = np.full(g.cell_shape(), mu0)
    s = A.assemble(g, rho, mu, dt, th)
    nv = s.n_vel
    offs = np.cumsum([0] + s.sizes)
    rng = np.random.default_rng(0)
    for _ in range(6):
        k = [int(rng.integers(-n[a] // 2, n[a] // 2 + 1)) if a < dim else 0 for a in range(3)]
        sn = [math.sin(math.pi * k[a] / n[a]) if a < dim else 0.0 for a in range(3)]
        for c in range(dim):
            x = np.zeros(s.K.shape[0], dtype=complex)
            x[offs[c]:offs[c + 1]] = _mode(g, k, c).ravel()
            y = s.K.astype(complex) @ x
            for d in range(dim):
                got = y[offs[d]:offs[d + 1]]
                if d == c:
                    lam = rho0 / dt + th * mu0 * (8 * sn[c] ** 2 / h[c] ** 2 + sum(
                        4 * sn[e] ** 2 / h[e] ** 2 for e in range(dim) if e != c))
                else:
                    lam = 4 * th * mu0 * sn[c] * sn[d] / (h[c] * h[d])
                np.testing.assert_allclose(got, lam * _mode(g, k, d).ravel(), atol=1e-9 * (rho0 / dt))
            gotp = y[nv:]
            np.testing.assert_allclose(gotp, -(2j / h[c]) * sn[c] * _mode(g, k, None).ravel(), atol=1e-10)
        x = np.zeros(s.K.shape[0], dtype=complex)
        x[nv:] = _mode(g, k, None).ravel()
        y = s.K.astype(complex) @ x
        for c in range(dim):
            np.testing.assert_allclose(y[offs[c]:offs[c + 1]], (2j / h[c]) * sn[c] * _mode(g, k, c).ravel(),
                                       atol=1e-10)


def _thomas(a, b, c, d):
    """Tridiagonal solve: a sub-, b main, c super-diagonal."""
    n = len(b)
    cp = np.zeros(n)
    dp = np.zeros(n)
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / m if i < n - 1 else 0.0
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m
    x = np.zeros(n)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_shear_reduction_thomas(theta):
    """x-periodic, walls in y, rho and mu functions of y only, f = (f(y), 0).

    Then v = 0, p = const and u(y) solves the tridiagonal problem
    (rho/dt) u - theta d_y(mu_e d_y u) = f with mu_e the harmonic mean of the two
    cells around each edge (a wall edge takes its one cell and the ghost -u).
    """
    nx, ny = 6, 40
    h = (1.0 / nx, 1.0 / ny, 1.0)
    g = A.OGrid(2, (nx, ny, 1), h, periodic=(True, False, False))
    y = (np.arange(ny) + 0.5) * h[1]
    # sharp air/water contrast in y and a viscous-dominated dt
    Hs = W.heaviside(y - 0.5, 1.5 * h[1])
    rho_c = 1000.0 + (1.2 - 1000.0) * Hs
    mu_c = 1e-3 + (1.8e-5 - 1e-3) * Hs
    dt = 1e-3 * h[1] ** 2 / 1.8e-5
    rho_x = np.broadcast_to(rho_c[None, :, None], g.comp_shape(0)).copy()
    rho_y = np.broadcast_to(W.face_average(rho_c[None, :, None], 1)[:, :, :1], g.comp_shape(1)).copy()
    mu = np.broadcast_to(mu_c[None, :, None], g.cell_shape()).copy()
    f = np.sin(3 * y) + 0.3
    s = A.assemble(g, [rho_x, rho_y], mu, dt, theta)
    fu = [np.broadcast_to(f[None, :, None], g.comp_shape(0)).copy(), np.zeros(g.comp_shape(1))]
    x, _ = D.solve(s, s.pack(fu, np.zeros(g.cell_shape())))
    (u, v), p = s.unpack(x)
    # edge viscosities: harmonic of the two y-neighbours; mirrored at the walls
    me = np.empty(ny + 1)
    me[1:-1] = 2.0 / (1.0 / mu_c[:-1] + 1.0 / mu_c[1:])
    me[0], me[-1] = mu_c[0], mu_c[-1]
    hy2 = h[1] ** 2
    a = np.zeros(ny)
    b = rho_c / dt + theta * (me[:-1] + me[1:]) / hy2
    c = np.zeros(ny)
    a[1:] = -theta * me[1:-1] / hy2
    c[:-1] = -theta * me[1:-1] / hy2
    b[0] += theta * me[0] / hy2      # ghost -u at the bottom wall doubles the edge term
    b[-1] += theta * me[-1] / hy2
    ut = _thomas(a, b, c, f)
    np.testing.assert_allclose(u[0, :, 0], ut, rtol=1e-11, atol=1e-14 * np.abs(ut).max())
    assert np.abs(u - u[:, :, :1]).max() <= 1e-12 * np.abs(ut).max()
    assert np.abs(v).max() <= 1e-12 * np.abs(ut).max()
    assert np.abs(p).max() <= 1e-9


def test_pressure_poisson_spectrum():
    """-D beta G: symmetric, positive semidefinite, null space exactly the constants."""
    g = A.OGrid(2, (8, 8, 1), (1 / 8, 1 / 8, 1.0))
    prob = W.config1(scale=8)
    Lp = A.pressure_laplacian(g, prob.rho_faces).toarray()
    assert abs(Lp - Lp.T).max() <= 1e-15 * abs(Lp).max()
    ev, vec = np.linalg.eigh(Lp)
    assert ev[0] > -1e-12 * ev[-1]
    assert abs(ev[0]) < 1e-12 * ev[-1]
    assert ev[1] > 1e-8 * ev[-1]
    np.testing.assert_allclose(np.abs(vec[:, 0]), 1.0 / 8.0, rtol=1e-10)


def _rhs_grid(dim):
    n = (10, 12, 9) if dim == 3 else (10, 12, 1)
    return A.OGrid(dim, n, (0.1, 1 / 12, 0.11))


@pytest.mark.parametrize("dim", [2, 3])
def test_explicit_rhs_special_cases(dim):
    """Zero old velocity leaves only the gravity term; theta = 1 leaves the mass
    term and gravity; wall-normal entries are written as zero."""
    g = _rhs_grid(dim)
    rng = np.random.default_rng(40 + dim)
    rho = [rng.uniform(1, 1000, g.comp_shape(c)) for c in range(dim)]
    rf = [rng.uniform(1, 1000, g.comp_shape(c)) for c in range(dim)]
    mu = rng.uniform(1e-5, 1e-3, g.cell_shape())
    un = [rng.standard_normal(g.comp_shape(c)) for c in range(dim)]
    gv = (0.3, -9.81, 1.7)
    f0 = A.explicit_rhs(g, rho, mu, 1e-3, 0.5, [np.zeros_like(a) for a in un], rf, gv)
    f1 = A.explicit_rhs(g, rho, mu, 1e-3, 1.0, un, rf, gv)
    for c in range(dim):
        inner = [slice(None)] * 3
        inner[2 - c] = slice(1, -1)
        inner = tuple(inner)
        np.testing.assert_allclose(f0[c][inner], (rf[c] * gv[c])[inner], rtol=1e-15)
        np.testing.assert_allclose(f1[c][inner], (rho[c] / 1e-3 * un[c] + rf[c] * gv[c])[inner], rtol=1e-14)
        for end in (0, -1):
            sl = [slice(None)] * 3
            sl[2 - c] = end
            assert np.all(f0[c][tuple(sl)] == 0) and np.all(f1[c][tuple(sl)] == 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_explicit_rhs_viscous_part_of_shear_profiles(dim):
    """Constant mu, u = u(y) only (v = w = 0): the viscous part of the x-rows is
    mu u'' exactly for rows whose neighbours are interior: 0 for a linear
    profile, -2 mu for y(1 - y); a linear profile through zero at y = 0 is also
    exact next to that wall (the ghost is its odd reflection)."""
    g = _rhs_grid(dim)
    mu0 = 2.5e-3
    mu = np.full(g.cell_shape(), mu0)
    rho = [np.zeros(g.comp_shape(c)) for c in range(dim)]
    _, Yc, _ = W.face_coords(g.n, g.h, 0)
    for prof, want in ((Yc, 0.0), (Yc * (1.0 - Yc), -2.0 * mu0)):
        un = [prof] + [np.zeros(g.comp_shape(c)) for c in range(1, dim)]
        f = A.explicit_rhs(g, rho, mu, 1.0, 0.0, un)
        rows = slice(0 if want == 0.0 else 1, -1)        # y rows (the top wall row differs)
        # x rows 2..nx-2: their x-neighbours are interior faces (the profile is cut to zero on
        # the x-walls, where u is wall-normal)
        zs = slice(1, -1) if dim == 3 else slice(None)   # in 3D the z-walls' ghosts see u too
        np.testing.assert_allclose(f[0][zs, rows, 2:-2], want, rtol=0, atol=1e-12)
