"""Periodic axes through the C-ABI (stokes_grid.periodic): the MAC operator on a
periodic axis wraps cells, faces and edges (Sec. 3.1's staggered layout with
no wall), checked three ways that do not depend on the GPU's own arithmetic:

* the constant-coefficient operator's Fourier symbol in closed form (every
  axis periodic): a mode sampled at each field's positions is mapped to the
  symbol matrix [[rho/dt - theta mu (S + s s^T), s], [-s^T, 0]] times the mode,
  with s_d = (2i/h_d) sin(kappa_d h_d / 2) and S = sum_d s_d^2;
* the 1D shear reduction: x-periodic, rho and mu varying in y only and f =
  (f_x(y), 0): v = 0, p = const and u(y) solves a tridiagonal system (a
  Thomas solve with the harmonic edge viscosity and the wall ghosts);
* the oracle's assembled operator and its direct solves on periodic grids with
  variable coefficients (mixed periodic / wall axes, 2D and 3D).

Caller arrays keep the wall layouts: along a periodic axis a face array has
N + 1 faces, the last repeating face 0 (ignored on input, face 0 on output).
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble as A
from oracle import direct as D
from tests.gpu_util import gpu_apply, gpu_solve, rel

pytestmark = pytest.mark.gpu


def _to_caller(a, comp, periodic):
    """Oracle face array (N faces along a periodic comp axis) -> caller layout (N + 1)."""
    if not periodic[comp]:
        return a
    ax = 2 - comp
    first = np.take(a, [0], axis=ax)
    return np.concatenate([a, first], axis=ax)


def _from_caller(a, comp, periodic):
    if not periodic[comp]:
        return a
    ax = 2 - comp
    n = a.shape[ax] - 1
    last = np.take(a, [n], axis=ax)
    assert np.array_equal(last, np.take(a, [0], axis=ax)), "face N must repeat face 0"
    return np.take(a, np.arange(n), axis=ax)


def _problem(dim, n, h, periodic, seed, dt=1e-3, contrast=True):
    """Random variable coefficients in the oracle's layouts (plus the caller's)."""
    rng = np.random.default_rng(seed)
    g = A.OGrid(dim, n, h, periodic=tuple(bool(p) for p in periodic))
    rho_o = [rng.uniform(1.2, 1000.0 if contrast else 2.0, size=g.comp_shape(c)) for c in range(dim)]
    mu = np.exp(rng.uniform(np.log(1.8e-5), np.log(1e-3), size=g.cell_shape()))
    fu_o = [rng.standard_normal(g.comp_shape(c)) for c in range(dim)]
    prob = W.Problem(name="periodic", dim=dim, n=n, h=h, dt=dt,
                     rho_faces=[_to_caller(rho_o[c], c, periodic) for c in range(dim)] + [None] * (3 - dim),
                     mu=mu, rhs_u=[_to_caller(fu_o[c], c, periodic) for c in range(dim)] + [None] * (3 - dim),
                     rhs_p=np.zeros(g.cell_shape()), tol=1e-12)
    return g, rho_o, mu, fu_o, prob


APPLY = [
    (2, (16, 12, 1), (1, 0, 0)),
    (2, (16, 12, 1), (0, 1, 0)),
    (2, (8, 6, 1), (1, 1, 0)),
    (3, (8, 6, 4), (1, 0, 0)),
    (3, (6, 8, 4), (0, 1, 1)),
    (3, (4, 6, 8), (1, 1, 1)),
    (3, (2, 2, 2), (1, 1, 1)),
    # at least 256 cells along x: the finest box's rows are padded (periodic x wraps at nx)
    (3, (256, 4, 4), (1, 0, 0)),
]


@pytest.mark.parametrize("dim,n,periodic", APPLY)
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_periodic_apply_matches_oracle_matrix(dim, n, periodic, theta):
    h = (0.11, 0.07, 0.09)
    g, rho_o, mu, _, prob = _problem(dim, n, h, periodic, 3, dt=1e-7)
    print("periodic apply", n, periodic, theta, flush=True)
    sys = A.assemble(g, rho_o, mu, prob.dt, theta)
    rng = np.random.default_rng(4)
    xu_o = [rng.standard_normal(g.comp_shape(c)) for c in range(dim)]
    xp = rng.standard_normal(g.cell_shape())
    xu = [_to_caller(xu_o[c], c, periodic) for c in range(dim)]
    # the ignored last face: garbage there must not matter
    for c in range(dim):
        if periodic[c]:
            sl = [slice(None)] * 3
            sl[2 - c] = -1
            xu[c][tuple(sl)] = 1e30
    yu, yp = gpu_apply(prob, xu, xp, theta, periodic=periodic)
    yu_o = [_from_caller(yu[c], c, periodic) for c in range(dim)]
    y_ref = sys.K @ sys.pack(xu_o, xp)
    y_gpu = sys.pack(yu_o, yp)
    assert np.abs(y_gpu - y_ref).max() <= 1e-13 * np.abs(y_ref).max()
    # wall-normal faces of the wall axes are still written as zero
    for c in range(dim):
        if not periodic[c]:
            sl = [slice(None)] * 3
            for end in (0, -1):
                sl[2 - c] = end
                assert np.all(yu[c][tuple(sl)] == 0.0)


def _positions(dim, n, h, comp):
    """Coordinates (x, y, z) of the unknowns of comp (0..dim-1 faces, dim cells),
    all axes periodic: faces at i h along their own axis, cells at (i + 1/2) h."""
    idx = np.indices((n[2], n[1], n[0])).astype(float)
    k, j, i = idx
    pos = [(i + 0.5) * h[0], (j + 0.5) * h[1], (k + 0.5) * h[2]]
    if comp < dim:
        pos[comp] = [i, j, k][comp] * h[comp]
    return pos


@pytest.mark.parametrize("dim,n,modes", [
    (2, (16, 16, 1), [(1, 0, 0), (0, 3, 0), (2, -5, 0), (8, 8, 0)]),
    (3, (8, 8, 8), [(1, 0, 0), (1, 2, -3), (4, 4, 4), (0, 0, 1)]),
])
def test_periodic_fourier_symbol(dim, n, modes):
    h = (1.0 / n[0], 1.0 / n[1], 1.0 / max(n[2], 1))
    rho, mu_v, dt, theta = 700.0, 3e-3, 1e-3, 0.5
    cells = (n[2], n[1], n[0])
    prob = W.Problem(name="fourier", dim=dim, n=n, h=h, dt=dt,
                     rho_faces=[np.full(W.face_shape(n, c), rho) for c in range(dim)] + [None] * (3 - dim),
                     mu=np.full(cells, mu_v), rhs_u=[None] * 3, rhs_p=np.zeros(cells), tol=1e-10)
    per = (1, 1, 1 if dim == 3 else 0)
    rng = np.random.default_rng(11)
    for m in modes:
        kap = [2 * np.pi * m[d] / (n[d] * h[d]) for d in range(dim)]
        s = np.array([2j / h[d] * np.sin(kap[d] * h[d] / 2) for d in range(dim)])
        S = np.sum(s ** 2)
        Kh = np.zeros((dim + 1, dim + 1), dtype=complex)
        Kh[:dim, :dim] = (rho / dt) * np.eye(dim) - theta * mu_v * (S * np.eye(dim) + np.outer(s, s))
        Kh[:dim, dim] = s
        Kh[dim, :dim] = -s
        amp = rng.standard_normal(dim + 1) + 1j * rng.standard_normal(dim + 1)
        out = Kh @ amp
        wave = lambda comp: np.exp(1j * sum(kap[d] * _positions(dim, n, h, comp)[d] for d in range(dim)))
        xu = [_to_caller(np.real(amp[c] * wave(c)), c, per) for c in range(dim)]
        xp = np.real(amp[dim] * wave(dim))
        yu, yp = gpu_apply(prob, xu, xp, theta, periodic=per)
        scale = np.abs(out[:dim]).max()
        for c in range(dim):
            ref = np.real(out[c] * wave(c))
            got = _from_caller(yu[c], c, per)
            assert np.abs(got - ref).max() <= 1e-12 * scale, (m, c)
        pscale = np.abs(s).max() * np.abs(amp[:dim]).max() * dim
        assert np.abs(yp - np.real(out[dim] * wave(dim))).max() <= 1e-12 * pscale, m


def _thomas(a, b, c, d):
    """Tridiagonal solve (sub a, diag b, super c)."""
    n = len(d)
    cp, dp = np.zeros(n), np.zeros(n)
    cp[0], dp[0] = c[0] / b[0], d[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / m if i < n - 1 else 0.0
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m
    x = np.zeros(n)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_shear_reduction(dim):
    """x-periodic (and z-periodic in 3D), walls in y, rho and mu of y only with an
    air/water contrast of 1000, f = (f_x(y), 0, 0): the solve gives v = w = 0,
    p = const and the u(y) of the tridiagonal shear problem."""
    ny = 32
    n = (8, ny, 4 if dim == 3 else 1)
    h = (1.0 / 8, 1.0 / ny, 1.0 / 4)
    per = (1, 0, 1 if dim == 3 else 0)
    dt, theta = 2e-2, 1.0
    yc = (np.arange(ny) + 0.5) * h[1]
    H = 0.5 * (1 + np.tanh((yc - 0.5) / 0.03))
    rho_c = 1.2 + (1000.0 - 1.2) * (1 - H)               # water below, air above
    mu_c = 1.8e-5 + (1e-3 - 1.8e-5) * (1 - H)
    f = np.sin(np.pi * yc) + 0.3 * np.cos(3 * np.pi * yc)
    cells = (n[2], n[1], n[0])
    bc = lambda v, comp: np.broadcast_to(v.reshape(1, ny, 1), W.face_shape(n, comp) if comp is not None else cells).copy()
    rho_faces = [bc(rho_c, 0), None, None]
    # y-faces: harmonic... any positive values; v stays zero whatever they are
    rho_faces[1] = np.broadcast_to(np.concatenate([[rho_c[0]], 0.5 * (rho_c[1:] + rho_c[:-1]), [rho_c[-1]]]
                                                  ).reshape(1, ny + 1, 1), W.face_shape(n, 1)).copy()
    if dim == 3:
        rho_faces[2] = bc(rho_c, 2)
    rhs_u = [bc(f, 0), np.zeros(W.face_shape(n, 1)), np.zeros(W.face_shape(n, 2)) if dim == 3 else None]
    prob = W.Problem(name="shear", dim=dim, n=n, h=h, dt=dt, rho_faces=rho_faces, mu=bc(mu_c, None),
                     rhs_u=rhs_u, rhs_p=np.zeros(cells), tol=1e-13)
    xu, xp, st, stats = gpu_solve(prob, tol=1e-13, periodic=per, max_iters=400)
    print("shear reduction dim %d: status %d iters %d res %.2e" % (dim, st, stats.iters, stats.rel_res_true))
    assert st == 0 or stats.rel_res_true <= 1e-12
    # Thomas: (rho/dt) u_j - theta/h^2 [mu_{j+1/2}(u_{j+1} - u_j) - mu_{j-1/2}(u_j - u_{j-1})] = f_j,
    # mu at the nodes the harmonic mean of the two cells (of the mirrored cell at a wall),
    # wall ghosts -u
    hy2 = h[1] ** 2
    mn = np.empty(ny + 1)
    mn[1:-1] = 2.0 / (1 / mu_c[1:] + 1 / mu_c[:-1])
    mn[0], mn[-1] = mu_c[0], mu_c[-1]
    a = -theta * mn[:-1] / hy2
    c = -theta * mn[1:] / hy2
    b = rho_c / dt + theta * (mn[1:] + mn[:-1]) / hy2
    b[0] += theta * mn[0] / hy2                           # ghost -u_0 doubles the wall term
    b[-1] += theta * mn[-1] / hy2
    a[0] = c[-1] = 0.0
    u_ref = _thomas(a, b, c, f)
    u = _from_caller(xu[0], 0, per)
    for col in u.reshape(-1, ny, n[0]).transpose(0, 2, 1).reshape(-1, ny):
        assert np.abs(col - u_ref).max() <= 1e-9 * np.abs(u_ref).max()
    assert np.abs(xu[1]).max() <= 1e-9 * np.abs(u_ref).max()
    if dim == 3:
        assert np.abs(xu[2]).max() <= 1e-9 * np.abs(u_ref).max()
    assert np.abs(xp - xp.mean()).max() <= 1e-8 * np.abs(f).max()


SOLVE = [
    (2, (32, 16, 1), (1, 0, 0), 1e-3),
    (2, (16, 16, 1), (1, 1, 0), 1e-3),
    (3, (16, 8, 8), (1, 1, 0), 1e-3),
    (3, (8, 8, 8), (1, 1, 1), 1e-3),
    (2, (16, 16, 1), (1, 0, 0), 100.0),                   # viscous-dominated: velocity multigrid
    (3, (256, 8, 8), (1, 0, 0), 1e-3),                    # padded finest rows
]


@pytest.mark.parametrize("dim,n,periodic,dt", SOLVE)
@pytest.mark.parametrize("precision", [0, 1])
def test_periodic_solve_matches_direct(dim, n, periodic, dt, precision):
    h = (1.0 / n[0], 1.0 / n[1], 1.0 / max(n[2], 1))
    g, rho_o, mu, fu_o, prob = _problem(dim, n, h, periodic, 21, dt=dt)
    print("periodic solve", n, periodic, "dt", dt, "precision", precision, flush=True)
    sys = A.assemble(g, rho_o, mu, prob.dt, 1.0)
    x, _ = D.solve(sys, sys.pack(fu_o, prob.rhs_p), dense=sys.K.shape[0] <= 3000)
    ru, rp = sys.unpack(x)
    xu, xp, st, stats = gpu_solve(prob, tol=1e-13, periodic=periodic, precision=precision, max_iters=400)
    print("  status %d iters %d res %.2e" % (st, stats.iters, stats.rel_res_true), flush=True)
    assert st == 0 or (st == 1 and stats.rel_res_true <= 1e-12), stats.as_dict()
    errs = [rel(_from_caller(xu[c], c, periodic), ru[c]) for c in range(dim)]
    errs.append(rel(xp - xp.mean(), rp - rp.mean()))
    print("  rel errors", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= 1e-9, errs


def test_periodic_rejected_where_walls_are_needed():
    import paper_1901_07892_amd as S
    import torch
    n = (8, 8, 1)
    g = S._binding.make_grid(2, n, (0.1, 0.1, 0.1), (1, 0, 0))
    # an odd periodic count and an open top over a periodic vertical axis are refused
    rho = [torch.ones(W.face_shape(n, c), dtype=torch.float64, device="cuda") for c in range(2)]
    mu = torch.ones((1, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(S.StokesError):
        S.StokesSolver(2, (7, 8, 1), (0.1, 0.1, 0.1), [torch.ones(W.face_shape((7, 8, 1), c), dtype=torch.float64,
                                                                device="cuda") for c in range(2)],
                       torch.ones((1, 8, 7), dtype=torch.float64, device="cuda"), 1e-3, periodic=(1, 0, 0))
    with pytest.raises(S.StokesError):
        S.StokesSolver(2, n, (0.1, 0.1, 0.1), rho, mu, 1e-3, periodic=(0, 1, 0), open_top=1)
    # the steps around the solve need walls
    un = torch.zeros(8, dtype=torch.float64, device="cuda")
    ut = torch.zeros(9, dtype=torch.float64, device="cuda")
    wave = S.make_wave(0.02, 0.5, 1.5, 5.0, 9.81, 1.5)
    with pytest.raises(S.StokesError):
        S.stokes_wave_inflow(g, wave, 0.0, un, ut)
