"""Pins of the input generator's closed forms (level-set material law, Stokes wave)."""
import math

import numpy as np

import workloads as W


def test_heaviside_closed_form():
    # Sec. 4.1 eq_heaviside: 0 below -eps, 1 above eps, 1/2 at the interface,
    # continuous with zero slope at the band edges, odd symmetry about 1/2.
    eps = 1.5 / 64
    phi = np.linspace(-3 * eps, 3 * eps, 2001)
    H = W.heaviside(phi, eps)
    assert H[0] == 0.0 and H[-1] == 1.0
    assert abs(W.heaviside(np.array([0.0]), eps)[0] - 0.5) < 1e-15
    assert abs(W.heaviside(np.array([-eps]), eps)[0]) < 1e-15
    assert abs(W.heaviside(np.array([eps]), eps)[0] - 1.0) < 1e-15
    assert np.all(np.diff(H) >= -1e-15)
    np.testing.assert_allclose(H + H[::-1], 1.0, atol=1e-14)
    d = 1e-7 * eps
    slope = (W.heaviside(np.array([eps]), eps) - W.heaviside(np.array([eps - d]), eps)) / d
    assert abs(slope[0]) < 1e-4 / eps
    # interior value at phi = eps/2: 1/2 (1 + 1/2 + 1/pi)
    assert abs(W.heaviside(np.array([eps / 2]), eps)[0] - 0.5 * (1.5 + 1.0 / math.pi)) < 1e-15


def test_two_stage_property_law():
    # Sec. 4.1 eq_ls_flow / eq_ls_solid: liquid for H_flow = 0, gas for 1; the solid
    # overrides both where H_body = 0.
    z = W.two_stage(1000.0, 1.2, np.array([0.0, 1.0, 0.5, 1.0]),
                    [(500.0, np.array([1.0, 1.0, 1.0, 0.0]))])
    np.testing.assert_allclose(z, [1000.0, 1.2, 500.6, 500.0])


def test_stokes_wave_second_harmonic():
    # Sec. 7.1 eq_stokes_eta.  Value for H = 0.04, d = 0.5, lambda = 1.5 worked by
    # hand: k d = 2.0944, cosh = 4.1218, cosh 2kd = 33.00, sinh^3 = 63.94 -> 9.45e-4.
    a2 = W.stokes_wave_second_order_coeff(0.04, 0.5, 1.5)
    assert abs(a2 - 9.45e-4) < 5e-6
    # deep water limit: the classical k H^2 / 8
    H, lam = 0.04, 1.5
    k = 2 * math.pi / lam
    assert abs(W.stokes_wave_second_order_coeff(H, 50.0, lam) - k * H * H / 8) < 1e-12


def test_sdfs():
    X, Y, Z = np.meshgrid([0.0, 0.5, 1.0], [0.5], [0.5], indexing="xy")
    d = W.sdf_box(np.array([0.5, 0.9, 1.0]), np.array([0.5, 0.5, 0.8]), np.array([0.5, 0.5, 0.5]),
                  (0.5, 0.5, 0.5), (0.1, 0.1, 0.1), 3)
    np.testing.assert_allclose(d, [-0.1, 0.3, math.hypot(0.4, 0.2)])
    q = W.sdf_quarter_space(np.array([0.0, 0.5, 0.5]), np.array([0.0, 0.0, 0.7]), 0.4, 0.6)
    np.testing.assert_allclose(q, [-0.4, 0.1, math.hypot(0.1, 0.1)])


def test_generator_is_seeded_and_shaped():
    a = W.config2(scale=8)
    b = W.config2(scale=8)
    np.testing.assert_array_equal(a.rhs_u[0], b.rhs_u[0])
    np.testing.assert_array_equal(a.rho_faces[1], b.rho_faces[1])
    assert a.rho_faces[0].shape == (1, 64, 65) and a.rho_faces[1].shape == (1, 65, 64)
    p = W.config3(scale=8)
    assert p.rho_faces[2].shape == (17, 16, 16)
    assert p.mu.min() >= W.MU_AIR - 1e-12 and p.mu.max() <= W.MU_WATER + 1e-12
    for c in range(3):
        r = p.rho_faces[c]
        assert r.min() >= W.RHO_AIR - 1e-9 and r.max() <= 1000.0 + 1e-9
    c5 = W.config5(n_cells=32)
    rmin = min(r.min() for r in c5.rho_faces)
    assert abs(rmin - 1.0) < 1e-12          # density ratio exactly 1000 at the headline
