"""Pins of the face-density transport oracle (oracle/transport.py): the CUI
limiter's defining properties, the flux divergence against a point-by-point
loop over control volumes, free-stream preservation, exact derivatives of
linear profiles, the SSP-RK3 weights in closed form, mirror symmetry of the
upwinding and conservation of mass.  CPU only."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import transport as T


# ------------------------------------------------------------------ CUI limiter
def test_cui_limiter_definition_points():
    U, D = np.zeros(7), np.ones(7)
    r = np.array([-0.5, 0.1, 2.0 / 13.0, 0.5, 0.8, 0.9, 1.5])
    want = np.array([-0.5, 0.3, 6.0 / 13.0, 5.0 / 12.0 + 1.0 / 3.0, 1.0, 1.0, 1.5])
    got = T.cui_face(U, r, D)
    assert np.allclose(got, want, rtol=0, atol=1e-15)
    # continuous at both break points
    for rb in (2.0 / 13.0, 0.8):
        lo = T.cui_face(np.zeros(1), np.array([rb - 1e-12]), np.ones(1))
        hi = T.cui_face(np.zeros(1), np.array([rb + 1e-12]), np.ones(1))
        assert abs(hi[0] - lo[0]) < 1e-10
    # D = U: the upwind value
    assert T.cui_face(np.array([2.0]), np.array([5.0]), np.array([2.0]))[0] == 5.0


def test_cui_is_bounded_and_affine_invariant():
    rng = np.random.default_rng(1)
    U, C, D = rng.standard_normal((3, 2000))
    f = T.cui_face(U, C, D)
    mono = (C - U) * (D - C) >= 0
    lo, hi = np.minimum(C, D), np.maximum(C, D)
    assert np.all(f[mono] >= lo[mono] - 1e-14) and np.all(f[mono] <= hi[mono] + 1e-14)
    assert np.allclose(f[~mono], C[~mono])               # first-order upwind outside
    for a, b in ((3.0, -1.0), (-2.0, 0.5)):
        assert np.allclose(T.cui_face(a * U + b, a * C + b, a * D + b), a * f + b, rtol=1e-12, atol=1e-12)


def test_cui_is_third_order_upwind_on_smooth_monotone_data():
    # cell averages of (x + 3)^2 on cells -1, 0, 1: the face value at x = 1/2 is exact
    avg = lambda i: (i + 3.0) ** 2 + 1.0 / 12.0
    f = T.cui_face(np.array([avg(-1)]), np.array([avg(0)]), np.array([avg(1)]))
    assert f[0] == pytest.approx(3.5 ** 2, rel=1e-14)
    # linear point data: the face midpoint value
    f = T.cui_face(np.array([1.0]), np.array([3.0]), np.array([5.0]))
    assert f[0] == pytest.approx(4.0, rel=1e-15)


# ------------------------------------------------------------------ flux divergence
def _brute_R(dim, n, h, u, rho):
    """R by looping over every interior face and its 2 * dim control-volume faces."""
    nx, ny, nz = n
    ext = (nx, ny, nz)
    out = []
    for c in range(dim):
        shape = W.face_shape(n, c)
        R = np.zeros(shape)
        rc = rho[c]
        for k, j, i in itertools.product(*(range(s) for s in shape)):
            idx = [i, j, k]
            if idx[c] == 0 or idx[c] == ext[c]:
                continue                                    # wall-normal face
            tot = 0.0
            for d in range(dim):
                nd = shape[2 - d]

                def val(m):                                  # rho_c at index m along d, mirrored
                    if d == c:
                        mm = -m if m < 0 else (2 * (nd - 1) - m if m > nd - 1 else m)
                    else:
                        mm = -m - 1 if m < 0 else (2 * nd - 1 - m if m > nd - 1 else m)
                    p = list(idx)
                    p[d] = mm
                    return rc[p[2], p[1], p[0]]

                def adv(m):                                  # CV face between entries m-1 and m
                    if d == c:
                        if m == 0 or m == nd:
                            return 0.0
                        p0, p1 = list(idx), list(idx)
                        p0[d], p1[d] = m - 1, m
                        return 0.5 * (u[d][p0[2], p0[1], p0[0]] + u[d][p1[2], p1[1], p1[0]])
                    p0, p1 = list(idx), list(idx)
                    p0[c] -= 1
                    p0[d] = m
                    p1[d] = m
                    return 0.5 * (u[d][p0[2], p0[1], p0[0]] + u[d][p1[2], p1[1], p1[0]])

                def flux(m):
                    a = adv(m)
                    if a > 0:
                        lim = T.cui_face(np.array([val(m - 2)]), np.array([val(m - 1)]), np.array([val(m)]))[0]
                    else:
                        lim = T.cui_face(np.array([val(m + 1)]), np.array([val(m)]), np.array([val(m - 1)]))[0]
                    return a * lim

                m = idx[d]
                tot += (flux(m + 1) - flux(m)) / h[d]
            R[k, j, i] = tot
        out.append(R)
    return out


def _rand_fields(dim, n, seed):
    rng = np.random.default_rng(seed)
    rho = [rng.uniform(1.0, 1000.0, size=W.face_shape(n, c)) for c in range(dim)]
    u = []
    for c in range(dim):
        a = rng.standard_normal(W.face_shape(n, c))
        sl = [slice(None)] * 3
        for end in (0, -1):
            sl[2 - c] = end
            a[tuple(sl)] = 0.0
        u.append(a)
    return rho, u


@pytest.mark.parametrize("dim,n", [(2, (5, 4, 1)), (2, (3, 6, 1)), (3, (4, 3, 5)), (3, (3, 4, 2))])
def test_flux_divergence_equals_control_volume_loop(dim, n):
    h = (0.3, 0.2, 0.25)
    rho, u = _rand_fields(dim, n, sum(n))
    got = T.flux_divergence(dim, h, u, rho)
    want = _brute_R(dim, n, h, u, rho)
    for c in range(dim):
        assert np.abs(got[c] - want[c]).max() <= 1e-12 * np.abs(want[c]).max()


def _divergence_free(dim, n, h, seed, margin=0):
    """A MAC velocity field with zero discrete divergence in every cell: curls of
    node / edge stream functions that vanish within `margin` cells of the walls."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    u = [np.zeros(W.face_shape(n, c)) for c in range(dim)]
    planes = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
    for a, b in planes:
        # psi on the edges normal to the (a, b) plane: index along a and b are node
        # indices 0..n, along the third axis cell indices; zero near the walls
        shape = [nz, ny, nx]
        shape[2 - a] += 1
        shape[2 - b] += 1
        psi = rng.standard_normal(shape)
        ia = np.arange(shape[2 - a])
        ib = np.arange(shape[2 - b])
        keep_a = (ia > margin) & (ia < shape[2 - a] - 1 - margin)
        keep_b = (ib > margin) & (ib < shape[2 - b] - 1 - margin)
        psi *= np.expand_dims(keep_a, [k for k in range(3) if k != 2 - a]).astype(float)
        psi *= np.expand_dims(keep_b, [k for k in range(3) if k != 2 - b]).astype(float)
        # u_a = d psi / d x_b, u_b = -d psi / d x_a (faces of a: node index along a, cells along b)
        u[a] += np.diff(psi, axis=2 - b) / h[b]
        u[b] -= np.diff(psi, axis=2 - a) / h[a]
    return u


def _cell_divergence(dim, n, h, u):
    return sum(np.diff(u[c], axis=2 - c) / h[c] for c in range(dim))


@pytest.mark.parametrize("dim,n", [(2, (12, 10, 1)), (3, (8, 6, 10))])
def test_constant_density_is_preserved_by_divergence_free_flow(dim, n):
    h = (0.1, 0.12, 0.09)
    u = _divergence_free(dim, n, h, 3)
    assert np.abs(_cell_divergence(dim, n, h, u)).max() <= 1e-10 * max(np.abs(a).max() for a in u)
    for c in range(dim):                                  # wall-normal faces hold zero
        assert np.all(np.take(u[c], [0, -1], axis=2 - c) == 0.0)
    rho = [np.full(W.face_shape(n, c), 7.5) for c in range(dim)]
    R = T.flux_divergence(dim, h, u, rho)
    umax = max(np.abs(a).max() for a in u)
    assert max(np.abs(r).max() for r in R) <= 1e-12 * 7.5 * umax / min(h)
    out = T.ssp_rk3(dim, h, 0.01, rho, [u, u, u])
    assert max(np.abs(o - 7.5).max() for o in out) <= 1e-12 * 7.5


def _uniform_x_flow(dim, n, U):
    u = [np.zeros(W.face_shape(n, c)) for c in range(dim)]
    u[0][..., 1:-1] = U
    return u


@pytest.mark.parametrize("dim,n", [(2, (24, 6, 1)), (3, (24, 5, 4))])
def test_linear_profile_in_uniform_flow_and_rk3_weights(dim, n):
    """rho = a + b x and u = (U, 0, 0) away from the x-walls: R = U b exactly on
    every face whose stencils see only the uniform region, and three stages with
    stage velocities U1, U2, U3 give rho - dt b (U1/6 + U2/6 + 2 U3/3)."""
    h = (0.05, 0.07, 0.06)
    a0, b = 3.0, 2.5
    rho = []
    for c in range(dim):
        shp = W.face_shape(n, c)
        x = (np.arange(shp[2]) + (0.0 if c == 0 else 0.5)) * h[0]
        rho.append(np.broadcast_to(a0 + b * x, shp).copy())
    U = (0.7, -1.1, 0.4)

    def region(c, lo):
        """Interior faces of component c with x index in [lo, n_x - lo)."""
        shp = W.face_shape(n, c)
        m = np.zeros(shp, dtype=bool)
        m[..., lo:n[0] - lo] = True
        sl = [slice(None)] * 3
        for end in (0, -1):
            sl[2 - c] = end
            m[tuple(sl)] = False
        return m

    R = T.flux_divergence(dim, h, _uniform_x_flow(dim, n, U[0]), rho)
    for c in range(dim):
        m = region(c, 3)
        assert m.sum() > 0
        assert np.allclose(R[c][m], U[0] * b, rtol=1e-12, atol=0)
    dt = 0.01
    out = T.ssp_rk3(dim, h, dt, rho, [_uniform_x_flow(dim, n, Us) for Us in U])
    shift = dt * b * (U[0] / 6 + U[1] / 6 + 2 * U[2] / 3)
    for c in range(dim):
        m = region(c, 8)
        assert np.allclose(out[c][m], rho[c][m] - shift, rtol=0, atol=1e-12 * a0)


def test_upwinding_is_mirror_symmetric():
    """Reflecting the grid in x (arrays flipped, x-velocity negated) reflects R."""
    dim, n, h = 3, (7, 5, 6), (0.2, 0.15, 0.1)
    rho, u = _rand_fields(dim, n, 9)
    R = T.flux_divergence(dim, h, u, rho)
    fl = lambda a: a[..., ::-1].copy()
    rho_f = [fl(a) for a in rho]
    u_f = [fl(u[0]) * -1.0] + [fl(a) for a in u[1:]]
    Rf = T.flux_divergence(dim, h, u_f, rho_f)
    for c in range(dim):
        assert np.allclose(fl(Rf[c]), R[c], rtol=1e-12, atol=1e-12 * np.abs(R[c]).max())


@pytest.mark.parametrize("dim,n", [(2, (16, 14, 1)), (3, (12, 10, 14))])
def test_mass_is_conserved(dim, n):
    """With a divergence-free flow that vanishes within two cells of the walls, the
    density summed over the faces (each face's control volume) is conserved to
    round-off, for any density field."""
    h = (0.1, 0.1, 0.1)
    rng = np.random.default_rng(4)
    rho = [rng.uniform(1.0, 1000.0, size=W.face_shape(n, c)) for c in range(dim)]
    u = _divergence_free(dim, n, h, 5, margin=2)
    umax = max(np.abs(a).max() for a in u)
    dt = 0.2 * min(h) / umax
    out = T.ssp_rk3(dim, h, dt, rho, [u, u, u])
    for c in range(dim):
        m0, m1 = rho[c].sum(), out[c].sum()
        assert abs(m1 - m0) <= 1e-12 * m0
        assert np.abs(out[c] - rho[c]).max() > 1e-6        # the density did move
