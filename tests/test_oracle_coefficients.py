"""Pins of the coefficient-step oracle (oracle/coefficients.py) against what the
paper and the mathematics fix, not against its own formulas:

* the Heaviside is exactly 0 / 1 outside the band and 1/2 on the interface,
  odd about 1/2 (H(phi) + H(-phi) = 1), has slope 1/eps on the interface and
  zero slope at the band edges (it is C1: a sign error in its sine term breaks
  both slope checks), integrates to eps over the band, and is monotone;
* the property law orientation: liquid where phi < 0, solid where psi < 0, the
  solid overriding the flowing phase, several solids applied in turn;
* face averaging: an affine level set is reproduced exactly at interior face
  centres, boundary faces take their one cell, and a brute-force loop over the
  faces of a ragged 3D grid names the same two cells per face."""
import numpy as np
import pytest

from oracle import coefficients as C
import workloads as W


EPS = 1.5 / 64


def test_heaviside_outside_band_and_on_interface():
    x = np.array([-1.0, -EPS * (1 + 1e-12), EPS * (1 + 1e-12), 1.0, 0.0])
    np.testing.assert_array_equal(C.heaviside(x, EPS), [0.0, 0.0, 1.0, 1.0, 0.5])
    # the band formula meets 0 and 1 at the band edges (sin(pi) is 1.2e-16, not 0)
    assert abs(C.heaviside(np.array([-EPS]), EPS)[0]) < 1e-16
    assert abs(C.heaviside(np.array([EPS]), EPS)[0] - 1.0) < 1e-16


def test_heaviside_odd_about_one_half_and_monotone():
    x = np.linspace(-2 * EPS, 2 * EPS, 4001)
    hx = C.heaviside(x, EPS)
    np.testing.assert_allclose(hx + C.heaviside(-x, EPS), 1.0, rtol=0, atol=2e-16)
    assert np.all(np.diff(hx) >= -1e-16)     # sin(+-pi) leaves +-2e-17 at the band edges


def test_heaviside_slopes_pin_the_sine_term():
    """H'(0) = 1/eps and H'(+-eps) = 0; with the sine term's sign flipped they
    would be 0 and 1/eps, and without it 1/(2 eps) everywhere in the band."""
    d = 1e-6 * EPS
    s0 = (C.heaviside(np.array([d]), EPS) - C.heaviside(np.array([-d]), EPS))[0] / (2 * d)
    assert abs(s0 * EPS - 1.0) < 1e-6
    for edge in (-EPS, EPS):
        inner = edge - np.sign(edge) * d
        s = abs((C.heaviside(np.array([edge]), EPS) - C.heaviside(np.array([inner]), EPS))[0] / d)
        assert s * EPS < 1e-5


def test_heaviside_integrates_to_eps_over_the_band():
    """int_{-eps}^{eps} H = eps (odd symmetry about 1/2), by composite Simpson."""
    n = 2000
    x = np.linspace(-EPS, EPS, n + 1)
    f = C.heaviside(x, EPS)
    simpson = (x[1] - x[0]) / 3 * (f[0] + f[-1] + 4 * f[1:-1:2].sum() + 2 * f[2:-1:2].sum())
    assert abs(simpson / EPS - 1.0) < 1e-12


def test_property_law_orientation_and_precedence():
    h = (1 / 64,) * 3
    phi = np.array([[[-1.0, 1.0, -1.0, 1.0]]])          # liquid, gas, liquid, gas (cells along x)
    psi1 = np.array([[[1.0, 1.0, -1.0, -1.0]]])         # solid 1 covers the last two cells
    psi2 = np.array([[[1.0, -1.0, 1.0, 1.0]]])          # solid 2 covers the second cell
    rho, mu, flow = C.coefficients(3, h, phi, [psi1, psi2], [500.0, 700.0], [2e-3, 3e-3],
                                   1000.0, 1.0, 1e-3, 1.8e-5, 1.5)
    np.testing.assert_allclose(mu[0, 0], [1e-3, 3e-3, 2e-3, 2e-3], rtol=1e-15)
    # x-faces: boundary faces take their one cell; interior faces average the level sets, so
    # faces 1-3 sit on the liquid/gas interface (averaged phi = 0, H = 1/2).  Face 1: solid 2's
    # surface (half-way to 700).  Face 2: the surfaces of both solids (half-way to 500, then
    # half-way to 700).  Face 3: inside solid 1.  Face 4: gas cell inside solid 1.
    mid = 0.5 * (1000.0 + 1.0)
    fl = [1000.0, mid, mid, mid, 1.0]
    np.testing.assert_allclose(flow[0][0, 0], fl, rtol=1e-15)
    ref = [1000.0, 0.5 * (mid + 700.0), 0.5 * (0.5 * (mid + 500.0) + 700.0), 500.0, 500.0]
    np.testing.assert_allclose(rho[0][0, 0], ref, rtol=1e-14)


def test_affine_level_set_reproduced_on_interior_faces():
    rng = np.random.default_rng(11)
    n = (7, 5, 6)
    h = (0.1, 0.1, 0.1)
    a = rng.standard_normal(4)
    xs = [(np.arange(m) + 0.5) * hh for m, hh in zip(n, h)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    phi = a[0] * X + a[1] * Y + a[2] * Z + a[3]
    for ax in range(3):
        f = C.to_faces(phi, ax)
        fs = W.face_shape(n, ax)
        assert f.shape == fs
        # exact value at the face centres (interior faces only)
        c = [xs[0], xs[1], xs[2]]
        c[ax] = np.arange(n[ax] + 1) * h[ax]
        Zf, Yf, Xf = np.meshgrid(c[2], c[1], c[0], indexing="ij")
        exact = a[0] * Xf + a[1] * Yf + a[2] * Zf + a[3]
        sl = [slice(None)] * 3
        sl[2 - ax] = slice(1, -1)
        np.testing.assert_allclose(f[tuple(sl)], exact[tuple(sl)], rtol=0, atol=1e-14)
        for end, cell in ((0, 0), (-1, -1)):
            sf = [slice(None)] * 3
            sf[2 - ax] = end
            np.testing.assert_array_equal(f[tuple(sf)], np.take(phi, cell, axis=2 - ax))


def test_faces_name_the_right_cells_brute_force():
    rng = np.random.default_rng(12)
    nx, ny, nz = 5, 4, 3
    phi = rng.standard_normal((nz, ny, nx))
    for ax, (mx, my, mz) in enumerate([(nx + 1, ny, nz), (nx, ny + 1, nz), (nx, ny, nz + 1)]):
        f = C.to_faces(phi, ax)
        assert f.shape == (mz, my, mx)
        for k in range(mz):
            for j in range(my):
                for i in range(mx):
                    idx = [i, j, k]
                    lo, hi = list(idx), list(idx)
                    lo[ax] = max(idx[ax] - 1, 0)
                    hi[ax] = min(idx[ax], (nx, ny, nz)[ax] - 1)
                    want = 0.5 * (phi[lo[2], lo[1], lo[0]] + phi[hi[2], hi[1], hi[0]])
                    assert f[k, j, i] == want


def test_generated_problems_carry_the_same_fields():
    """The seeded workloads build their coefficients with the same law, so the
    oracle reproduces them from the stored level sets (2D and 3D, with solids)."""
    for p in (W.config1(), W.config3(scale=4)):
        rho, mu, flow = C.coefficients(p.dim, p.h, p.phi, p.psi, p.rho_solid, [W.MU_SOLID] * len(p.psi),
                                       W.RHO_WATER, p.rho_air, W.MU_WATER, W.MU_AIR, p.heaviside_cells)
        np.testing.assert_allclose(mu, p.mu, rtol=1e-14)
        for ax in range(p.dim):
            np.testing.assert_allclose(rho[ax], p.rho_faces[ax], rtol=1e-14)
            np.testing.assert_allclose(flow[ax], p.rho_flow_faces[ax], rtol=1e-14)
