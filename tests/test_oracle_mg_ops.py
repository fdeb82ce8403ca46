"""Pins of the oracle's multigrid kernels (oracle/mg_ops.py) against the
Kronecker-assembled Poisson operator, brute-force loops and their defining
invariants.  CPU only."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble as A
from oracle import mg_ops as M


def _random_case(dim, n, seed):
    rng = np.random.default_rng(seed)
    h = tuple(rng.uniform(0.05, 0.2, size=3))
    rho = [rng.uniform(1.0, 1000.0, size=W.face_shape(n, c)) for c in range(dim)]
    e = rng.standard_normal(W.cell_shape(n))
    r = rng.standard_normal(W.cell_shape(n))
    return h, rho, e, r


CASES = [(2, (7, 5, 1)), (2, (8, 6, 1)), (3, (5, 4, 3)), (3, (6, 4, 8))]


@pytest.mark.parametrize("dim,n", CASES)
def test_apply_equals_assembled_operator(dim, n):
    h, rho, e, _ = _random_case(dim, n, 1)
    g = A.OGrid(dim, n, h)
    Lp = A.pressure_laplacian(g, rho)
    y_ref = (Lp @ e.ravel()).reshape(e.shape)
    y = M.apply(dim, h, M.betas(dim, rho), e)
    assert np.abs(y - y_ref).max() <= 1e-13 * np.abs(y_ref).max()
    d = M.diagonal(dim, h, M.betas(dim, rho), e.shape)
    assert np.allclose(d.ravel(), Lp.diagonal(), rtol=1e-14, atol=0)


def _brute_rb_sweep(dim, n, h, rho, e, r, omega=1.0):
    """Point-by-point red-black Gauss-Seidel (relaxed by omega) from the face
    densities, cell by cell."""
    nx, ny, nz = n
    e = e.copy()
    ext = (nx, ny, nz)
    for colour in (0, 1):
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            if (i + j + k) % 2 != colour:
                continue
            num, den = r[k, j, i], 0.0
            for a in range(dim):
                for side in (-1, 1):
                    p = [i, j, k]
                    p[a] += side
                    if not 0 <= p[a] < ext[a]:
                        continue                      # wall: no flux
                    f = [i, j, k]
                    if side == 1:
                        f[a] += 1
                    w = 1.0 / rho[a][f[2], f[1], f[0]] / h[a] ** 2
                    num += w * e[p[2], p[1], p[0]]
                    den += w
            e[k, j, i] = (1.0 - omega) * e[k, j, i] + omega * (num / den)
    return e


@pytest.mark.parametrize("omega", [1.0, 1.1, 0.7])
@pytest.mark.parametrize("dim,n", CASES)
def test_rb_sweep_equals_brute_force(dim, n, omega):
    h, rho, e, r = _random_case(dim, n, 2)
    ref = _brute_rb_sweep(dim, n, h, rho, e, r, omega)
    got = M.rb_gs_sweep(dim, h, M.betas(dim, rho), e, r, omega=omega)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dim,n", CASES)
def test_relaxed_colour_scales_its_residual_rows(dim, n):
    """Red-black SOR: a cell's own row has the residual d_c (g_c - e_c), and the
    relaxed update leaves the fraction 1 - omega of it (same-colour cells do not
    neighbour, so the other rows of the colour keep their neighbour sums)."""
    h, rho, e, r = _random_case(dim, n, 6)
    beta = M.betas(dim, rho)
    omega = 1.1
    res0 = r - M.apply(dim, h, beta, e)
    for colour in (0, 1):
        e1 = M.gs_colour(dim, h, beta, e, r, colour, omega=omega)
        res1 = r - M.apply(dim, h, beta, e1)
        m = M.colour_mask(e.shape, colour)
        assert np.abs(res1[m] - (1.0 - omega) * res0[m]).max() <= 1e-12 * np.abs(res0).max() * 1e3
        assert np.array_equal(e1[~m], e[~m])


@pytest.mark.parametrize("dim,n", CASES)
def test_each_colour_zeroes_its_residual_rows(dim, n):
    h, rho, e, r = _random_case(dim, n, 3)
    beta = M.betas(dim, rho)
    e1 = M.gs_colour(dim, h, beta, e, r, 0)
    res = r - M.apply(dim, h, beta, e1)
    m0 = M.colour_mask(e.shape, 0)
    assert np.abs(res[m0]).max() <= 1e-12 * np.abs(r).max() * 1e3
    assert np.array_equal(e1[~m0], e[~m0])            # the other colour is untouched
    e2 = M.gs_colour(dim, h, beta, e1, r, 1)
    res = r - M.apply(dim, h, beta, e2)
    assert np.abs(res[~m0]).max() <= 1e-12 * np.abs(r).max() * 1e3
    assert np.array_equal(e2[m0], e1[m0])


def test_sweep_leaves_the_exact_solution_fixed():
    dim, n = 3, (6, 4, 4)
    h, rho, _, r = _random_case(dim, n, 4)
    g = A.OGrid(dim, n, h)
    Lp = A.pressure_laplacian(g, rho).tocsc()
    r = r - r.mean()                                   # compatible with the Neumann walls
    # pin the first cell, solve, and check the residual before using the solution
    keep = np.arange(1, r.size)
    x = np.zeros(r.size)
    x[keep] = spla.spsolve(Lp[keep][:, keep], r.ravel()[keep])
    assert np.abs(Lp @ x - r.ravel()).max() <= 1e-9 * np.abs(r).max()
    e = x.reshape(r.shape)
    for omega in (1.0, 1.1):
        out = M.rb_gs_sweep(dim, h, M.betas(dim, rho), e, r, omega=omega)
        assert np.abs(out - e).max() <= 1e-8 * np.abs(e).max()


@pytest.mark.parametrize("dim,n", [(2, (8, 6, 1)), (3, (6, 4, 8))])
def test_residual_restriction(dim, n):
    h, rho, e, r = _random_case(dim, n, 5)
    beta = M.betas(dim, rho)
    # zero iterate: block means of r, brute force
    rc = M.residual_restrict(dim, h, beta, np.zeros_like(e), r)
    nx, ny, nz = n
    for K, J, I in itertools.product(range(max(nz // 2, 1)), range(ny // 2), range(nx // 2)):
        ks = [2 * K, 2 * K + 1] if dim == 3 else [0]
        vals = [r[k, j, i] for k in ks for j in (2 * J, 2 * J + 1) for i in (2 * I, 2 * I + 1)]
        assert rc[K, J, I] == pytest.approx(np.mean(vals), rel=1e-14, abs=1e-15)
    # a constant iterate is in the null space
    rc1 = M.residual_restrict(dim, h, beta, np.full_like(e, 3.7), r)
    assert np.abs(rc1 - rc).max() <= 1e-12 * np.abs(rc).max()
    # the coarse sum carries the fine residual sum (times the 2^d child volume ratio)
    rc2 = M.residual_restrict(dim, h, beta, e, r)
    res = r - M.apply(dim, h, beta, e)
    assert rc2.sum() * 2 ** dim == pytest.approx(res.sum(), rel=1e-10, abs=1e-10)


def test_prolongation():
    rng = np.random.default_rng(6)
    ec = rng.standard_normal((3, 4, 5))
    f = M.prolong(3, ec, lin=False)
    assert f.shape == (6, 8, 10)
    for k, j, i in itertools.product(range(6), range(8), range(10)):
        assert f[k, j, i] == ec[k // 2, j // 2, i // 2]
    # trilinear: constants everywhere, linear functions away from the walls
    assert np.allclose(M.prolong(3, np.full((3, 4, 5), 2.5), lin=True), 2.5, rtol=0, atol=1e-14)
    Kc, Jc, Ic = np.indices((3, 4, 5)).astype(float)
    lin_c = 1.0 + 2.0 * (Ic + 0.5) * 2 - 3.0 * (Jc + 0.5) * 2 + 0.5 * (Kc + 0.5) * 2   # in fine cell units
    Kf, Jf, If = np.indices((6, 8, 10)).astype(float)
    lin_f = 1.0 + 2.0 * (If + 0.5) - 3.0 * (Jf + 0.5) + 0.5 * (Kf + 0.5)
    got = M.prolong(3, lin_c, lin=True)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.abs(got[inner] - lin_f[inner]).max() <= 1e-12
    # 2D: only the x and y axes are refined
    e2 = rng.standard_normal((1, 3, 4))
    assert M.prolong(2, e2, lin=False).shape == (1, 6, 8)


@pytest.mark.parametrize("dim,n", [(2, (7, 6, 1)), (3, (5, 4, 6))])
def test_open_top_apply_equals_assembled_operator(dim, n):
    h, rho, e, r = _random_case(dim, n, 7)
    g = A.OGrid(dim, n, h, open_top=True)
    Lp = A.pressure_laplacian(g, rho)
    y_ref = (Lp @ e.ravel()).reshape(e.shape)
    beta = M.betas(dim, rho, open_top=True)
    y = M.apply(dim, h, beta, e, open_top=True)
    assert np.abs(y - y_ref).max() <= 1e-13 * np.abs(y_ref).max()
    d = M.diagonal(dim, h, beta, e.shape, open_top=True)
    assert np.allclose(d.ravel(), Lp.diagonal(), rtol=1e-14, atol=0)
    # the sweep zeroes the residual rows of each colour with the Dirichlet top too
    e1 = M.gs_colour(dim, h, beta, e, r, 0, open_top=True)
    res = r - M.apply(dim, h, beta, e1, open_top=True)
    assert np.abs(res[M.colour_mask(e.shape, 0)]).max() <= 1e-9 * np.abs(r).max()
