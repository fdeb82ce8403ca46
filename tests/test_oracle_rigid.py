"""Pins of the rigid-body projection oracle (oracle/rigid.py) against closed forms,
brute force and invariants:

* Peskin's four-point kernel satisfies the conditions that define it: unit sum,
  zero first moment, sum of squares 3/8, even and odd sums 1/2, continuity at
  |r| = 1 and 2, phi(0) = 1/2;
* interpolation equals a brute-force sum of u delta_h over EVERY face of a grid
  extended by ghost layers that hold the odd reflection of u across the walls
  (no stencil, no index arithmetic shared with the oracle);
* interpolation reproduces linear fields exactly away from walls, and linear
  fields vanishing on a wall exactly near that wall;
* spreading is the adjoint of interpolation, walls included;
* free-body projection: the spread correction carries zero linear and zero
  angular momentum; a rigid velocity field is returned unchanged with its own
  (U_r, W_r); a prescribed motion equal to the field changes nothing."""
import math

import numpy as np
import pytest

from oracle import rigid as R
import workloads as W


def test_peskin_kernel_defining_conditions():
    r = np.random.default_rng(1).uniform(0.0, 1.0, 200)
    js = np.arange(-3, 4)
    phi = R.peskin4(r[:, None] - js[None, :])
    np.testing.assert_allclose(phi.sum(1), 1.0, atol=1e-15)
    np.testing.assert_allclose(((r[:, None] - js[None, :]) * phi).sum(1), 0.0, atol=1e-15)
    np.testing.assert_allclose((phi ** 2).sum(1), 3.0 / 8.0, atol=1e-15)
    np.testing.assert_allclose(phi[:, js % 2 == 0].sum(1), 0.5, atol=1e-15)
    assert R.peskin4(0.0) == 0.5 and R.peskin4(2.0) == 0.0 and R.peskin4(-2.5) == 0.0
    for a in (1.0, 2.0):
        assert abs(R.peskin4(a - 1e-12) - R.peskin4(a + 1e-12)) < 1e-11


def _ghost_extended(u, comp, n, dim, g=3):
    """u on a grid extended by g ghost layers per side: odd reflection across every
    wall (normal component: about the wall face, which holds 0; tangential: about
    the wall between the first cell and its ghost)."""
    a = np.asarray(u, dtype=np.float64)
    for d in range(dim):
        ax = a.ndim - 1 - d
        m = a.shape[ax]
        idx = []
        sgn = []
        if d == comp:                                  # faces 0..n, walls at 0 and n
            nn = m - 1
            for i in range(-g, nn + g + 1):
                if i < 0:
                    idx.append(-i), sgn.append(-1.0)
                elif i > nn:
                    idx.append(2 * nn - i), sgn.append(-1.0)
                else:
                    idx.append(i), sgn.append(0.0 if i in (0, nn) else 1.0)
        else:                                          # cells 0..n-1
            for j in range(-g, m + g):
                if j < 0:
                    idx.append(-1 - j), sgn.append(-1.0)
                elif j >= m:
                    idx.append(2 * m - 1 - j), sgn.append(-1.0)
                else:
                    idx.append(j), sgn.append(1.0)
        a = np.take(a, idx, axis=ax)
        shp = [1] * a.ndim
        shp[ax] = len(sgn)
        a = a * np.asarray(sgn).reshape(shp)
    return a


def _brute_interp(u, comp, X, n, h, dim, g=3):
    ext = _ghost_extended(u, comp, n, dim, g)
    coords = []
    for d in range(dim):
        m = n[d] + (1 if d == comp else 0)
        pos = (np.arange(-g, m + g) + (0.0 if d == comp else 0.5)) * h[d]
        coords.append(pos)
    # separable kernel: contract x, then y, then z (each the last remaining axis)
    val = ext
    for d in range(dim):
        val = val @ R.peskin4((coords[d] - X[d]) / h[d])
    return float(val)


@pytest.mark.parametrize("dim", [2, 3])
def test_interpolation_equals_brute_force_with_ghosts(dim):
    rng = np.random.default_rng(2 + dim)
    n = (7, 6, 5) if dim == 3 else (9, 7, 1)
    h = (0.1, 0.12, 0.09) if dim == 3 else (0.1, 0.12, 0.1)
    L = [n[d] * h[d] for d in range(dim)]
    u = [rng.standard_normal(W.face_shape(n, c)) for c in range(dim)]
    if dim == 2:
        u = [a[0] for a in u]          # (Ny, Nx+1) arrays for the brute force; oracle takes 3D layout
    X = np.stack([rng.uniform(0, L[d], 12) for d in range(dim)], 1)
    X[0, 0] = 0.0                       # on a wall
    X[1, 1] = L[1]                      # on the opposite wall
    uo = [rng_a.reshape(W.face_shape(n, c)) for c, rng_a in enumerate(u)]
    JU = R.interpolate(uo, X, n, h, dim)
    for m in range(X.shape[0]):
        for c in range(dim):
            assert abs(JU[m, c] - _brute_interp(u[c], c, X[m], n, h, dim)) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_fields_interpolated_exactly(dim):
    rng = np.random.default_rng(4 + dim)
    n = (12, 10, 11) if dim == 3 else (12, 10, 1)
    h = (0.1, 0.1, 0.1)
    L = [n[d] * h[d] for d in range(dim)]
    a = rng.standard_normal((dim, dim + 1))
    u = []
    for c in range(dim):
        X_, Y_, Z_ = W.face_coords(n, h, c)
        xyz = [X_, Y_, Z_]
        u.append(a[c, 0] + sum(a[c, 1 + d] * xyz[d] for d in range(dim)))
    Xin = np.stack([rng.uniform(2.2 * h[d], L[d] - 2.2 * h[d], 20) for d in range(dim)], 1)
    np.testing.assert_allclose(R.interpolate(u, Xin, n, h, dim), (a[:, :1] + a[:, 1:] @ Xin.T).T, atol=1e-13)
    # near the x = 0 wall: fields that vanish there (odd about the wall) are exact too
    b = rng.standard_normal(dim)
    u0 = []
    for c in range(dim):
        X_, _, _ = W.face_coords(n, h, c)
        u0.append(b[c] * X_)
    Xw = np.stack([rng.uniform(0.0, 1.5 * h[0], 15)] +
                  [rng.uniform(2.2 * h[d], L[d] - 2.2 * h[d], 15) for d in range(1, dim)], 1)
    np.testing.assert_allclose(R.interpolate(u0, Xw, n, h, dim), b[None, :] * Xw[:, :1], atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_spreading_is_adjoint_of_interpolation(dim):
    rng = np.random.default_rng(6 + dim)
    n = (8, 7, 6) if dim == 3 else (8, 7, 1)
    h = (0.1, 0.11, 0.12)
    L = [n[d] * h[d] for d in range(dim)]
    u = [rng.standard_normal(W.face_shape(n, c)) for c in range(dim)]
    X = np.stack([rng.uniform(0, L[d], 25) for d in range(dim)], 1)
    F = rng.standard_normal((25, dim))
    dV = 0.37 * np.prod(h[:dim])
    f = R.spread(F, X, dV, n, h, dim, [a.shape for a in u])
    lhs = (R.interpolate(u, X, n, h, dim) * F).sum() * dV
    rhs = sum((u[c] * f[c]).sum() for c in range(dim)) * np.prod(h[:dim])
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


def _ball(center, radius, h, dim):
    """Markers at the cell centres (spacing h) inside a ball, and their volume."""
    rng = [np.arange(math.floor((center[d] - radius) / h[d]), math.ceil((center[d] + radius) / h[d]) + 1)
           for d in range(dim)]
    pts = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, dim)
    X = (pts + 0.5) * np.asarray(h[:dim])
    X = X[np.linalg.norm(X - np.asarray(center[:dim]), axis=1) <= radius]
    return X, float(np.prod(h[:dim]))


@pytest.mark.parametrize("dim", [2, 3])
def test_free_body_correction_conserves_momentum(dim):
    rng = np.random.default_rng(8 + dim)
    n = (16, 16, 16) if dim == 3 else (24, 24, 1)
    h = (1.0 / n[0],) * 3
    u = [rng.standard_normal(W.face_shape(n, c)) for c in range(dim)]
    X, dV = _ball((0.47, 0.52, 0.5), 0.2, h, dim)
    xc = X.mean(0)
    unew, Ur, Wr = R.rigid_projection(u, X, dV, xc, n, h, dim, True)
    vol = np.prod(h[:dim])
    d = [unew[c] - u[c] for c in range(dim)]
    # linear momentum of the correction (unit density): zero
    for c in range(dim):
        assert abs(d[c].sum() * vol) < 1e-12 * np.abs(u[c]).sum() * vol
    # angular momentum about x_com of the correction: zero
    pos = [W.face_coords(n, h, c) for c in range(dim)]
    if dim == 2:
        Lz = ((pos[1][0] - xc[0]) * d[1]).sum() - ((pos[0][1] - xc[1]) * d[0]).sum()
        assert abs(Lz) < 1e-12
    else:
        for (a, b) in ((1, 2), (2, 0), (0, 1)):
            L = ((pos[b][a] - xc[a]) * d[b]).sum() - ((pos[a][b] - xc[b]) * d[a]).sum()
            assert abs(L) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_field_is_left_unchanged(dim):
    rng = np.random.default_rng(10 + dim)
    n = (16, 16, 16) if dim == 3 else (24, 24, 1)
    h = (1.0 / n[0],) * 3
    X, dV = _ball((0.5, 0.45, 0.55), 0.18, h, dim)
    xc = X.mean(0)
    U0 = rng.standard_normal(dim)
    W0 = rng.standard_normal(1 if dim == 2 else 3)
    u = []
    for c in range(dim):
        P = W.face_coords(n, h, c)
        r = [P[d] - xc[d] for d in range(dim)]
        if dim == 2:
            rot = [-W0[0] * r[1], W0[0] * r[0]][c]
        else:
            rot = (W0[(c + 1) % 3] * r[(c + 2) % 3] - W0[(c + 2) % 3] * r[(c + 1) % 3])
        u.append(U0[c] + rot)
    unew, Ur, Wr = R.rigid_projection(u, X, dV, xc, n, h, dim, True)
    np.testing.assert_allclose(Ur, U0, atol=1e-12)
    np.testing.assert_allclose(np.ravel(Wr), W0, atol=1e-11)
    for c in range(dim):
        np.testing.assert_allclose(unew[c], u[c], atol=1e-12)
    unew2, _, _ = R.rigid_projection(u, X, dV, xc, n, h, dim, False, U0, W0)
    for c in range(dim):
        np.testing.assert_allclose(unew2[c], u[c], atol=1e-12)
