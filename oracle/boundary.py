"""Oracle for the wave tank's boundaries (Sec. 7.1, "Stokes wave theory and numerics").

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module;
only ``tests/`` does.

Two pieces:

* The second-order Stokes wave of eqs. eq_stokes_eta, eq_stokes_u and
  eq_stokes_v (height H, still depth d, wavelength lambda, wave number
  k = 2 pi / lambda, angular frequency omega, gravity g), with the vertical
  coordinate measured from the still level (bottom at -d), and the inflow
  velocities it prescribes on the x = 0 side: the normal velocity on the x-faces
  there and the vertical tangential velocity on the wall, each multiplied by
  1 - H~(phi) with phi = -eta(0, t) + vertical coordinate and H~ the smoothed
  Heaviside of eq. eq_heaviside_normal_bdry of half-width n_cells sqrt(h_x h_v)
  (only the liquid phase is driven).  The lateral tangential velocity (3D) is 0.
* The inflow's contribution to the linear system: with the boundary values
  moved to the right-hand side, K x = b - (A_bc, -D_bc), where A_bc is the
  momentum operator applied to the boundary data alone (normal velocity on the
  x = 0 faces, and the tangential wall value entering through the ghost
  2 t_bc - interior) and D_bc the divergence of the normal boundary velocity.
  ``inflow_lift`` builds it from the same Kronecker-product operators as
  ``assemble`` (oracle/assemble.py).

The open top itself (zero pressure, zero tangential velocity) is part of the
assembled operator (``OGrid.open_top``).
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import scipy.sparse as sp

from .assemble import Assembler, OGrid


def wave_number(lam: float) -> float:
    return 2.0 * np.pi / lam


def dispersion_omega(k: float, d: float, g: float) -> float:
    """Linear dispersion relation omega^2 = g k tanh(k d) (the caller's choice of omega)."""
    return float(np.sqrt(g * k * np.tanh(k * d)))


def stokes_eta(H, d, lam, omega, x, t):
    """Free-surface elevation of eq. eq_stokes_eta."""
    k = wave_number(lam)
    c2 = np.pi * H * H / (8.0 * lam) * np.cosh(k * d) * (2.0 + np.cosh(2.0 * k * d)) / np.sinh(k * d) ** 3
    return 0.5 * H * np.cos(k * x - omega * t) + c2 * np.cos(2.0 * k * x - 2.0 * omega * t)


def stokes_velocity(H, d, lam, omega, g, x, y, t):
    """(u_w, v_w) of eqs. eq_stokes_u and eq_stokes_v; y is measured from the still level."""
    k = wave_number(lam)
    a1 = H * g * k / (2.0 * omega) / np.cosh(k * d)
    a2 = 3.0 * H * H * omega * k / 16.0 / np.sinh(k * d) ** 4
    ph1 = k * x - omega * t
    ph2 = 2.0 * k * x - 2.0 * omega * t
    u = a1 * np.cosh(k * (d + y)) * np.cos(ph1) + a2 * np.cosh(2.0 * k * (d + y)) * np.cos(ph2)
    v = a1 * np.sinh(k * (d + y)) * np.sin(ph1) + a2 * np.sinh(2.0 * k * (d + y)) * np.sin(ph2)
    return u, v


def boundary_heaviside(phi, eps):
    """The smoothed Heaviside of eq. eq_heaviside_normal_bdry (0 below -eps, 1 above eps)."""
    phi = np.asarray(phi, dtype=np.float64)
    out = 0.5 * (1.0 + phi / eps + np.sin(np.pi * phi / eps) / np.pi)
    return np.where(phi < -eps, 0.0, np.where(phi > eps, 1.0, out))


def stokes_inflow(dim, n, h, H, d, lam, omega, g, t, z_still, n_cells):
    """Inflow data on the x = 0 side.

    Returns (un, ut): un the normal velocity on the x-faces at x = 0, shape
    (Nz, Ny) (2D: (1, Ny)), at the faces' vertical coordinates (cell centres);
    ut the vertical tangential velocity on the wall at the vertical faces'
    positions (nodes along the vertical axis), shape (Nz+1, Ny) in 3D and
    (1, Ny+1) in 2D."""
    nx, ny, nz = n
    v = dim - 1
    hv = h[v]
    nv = n[v]
    eps = n_cells * np.sqrt(h[0] * hv)
    eta0 = stokes_eta(H, d, lam, omega, 0.0, t)
    zc = (np.arange(nv) + 0.5) * hv - z_still           # cell-centre heights from the still level
    zn = np.arange(nv + 1) * hv - z_still               # node heights
    uc, _ = stokes_velocity(H, d, lam, omega, g, 0.0, zc, t)
    _, vn = stokes_velocity(H, d, lam, omega, g, 0.0, zn, t)
    un1 = (1.0 - boundary_heaviside(-eta0 + zc, eps)) * uc
    ut1 = (1.0 - boundary_heaviside(-eta0 + zn, eps)) * vn
    if dim == 2:
        return un1[None, :], ut1[None, :]
    return np.repeat(un1[:, None], ny, axis=1), np.repeat(ut1[:, None], ny, axis=1)


def _full(g: OGrid, comp: int) -> np.ndarray:
    return np.zeros(g.comp_shape(comp))


def inflow_lift(g: OGrid, mu_cell: np.ndarray, theta: float, un: np.ndarray, ut: np.ndarray):
    """Right-hand-side contribution of Dirichlet inflow data on the x = 0 side.

    Returns (lift_u, lift_p) in the full face / cell layouts: subtract lift_u from
    the momentum right-hand side and lift_p from the continuity right-hand side
    (the equation -D u = g).  Wall-normal rows hold 0."""
    asm = Assembler(g)
    d = g.dim
    v = d - 1
    L = asm.viscous(np.asarray(mu_cell, dtype=np.float64))
    # the normal boundary velocity as a full x-face array (nonzero on x = 0 only)
    ub = [_full(g, c) for c in range(d)]
    ub[0][..., 0] = un.reshape(ub[0][..., 0].shape)
    lift = [-theta * sum(L[c][e] @ ub[e].ravel() for e in range(d)) for c in range(d)]
    # the vertical tangential wall value: the ghost beyond x = 0 is 2 t - interior, so the
    # x-strain of the vertical component on the wall edges gains -2 t / h_x (the rest of
    # the ghost is in the operator); shear stress = edge viscosity x strain, returned to
    # the vertical faces by the edge-to-face difference along x
    me = asm.edge_mu(np.asarray(mu_cell, dtype=np.float64), 0, v)
    epos = asm._pos(None, (0, v))
    shape_e = [g.n[2], g.n[1], g.n[0]]
    for a in (0, v):
        shape_e[2 - a] = g.nf(a)
    s_edge = np.zeros(shape_e)
    s_edge[..., 0] = -2.0 * ut.reshape(s_edge[..., 0].shape) / g.h[0]
    Dv = asm._op_along(0, "e2t", epos)
    lift[v] = lift[v] - theta * (Dv @ (me * s_edge.ravel()))
    # zero the rows that are not unknowns
    S = [asm.select(c) for c in range(d)]
    lift = [(S[c].T @ (S[c] @ lift[c])).reshape(g.comp_shape(c)) for c in range(d)]
    # continuity: -D u_b
    lift_p = -sum(asm.div(c) @ ub[c].ravel() for c in range(d)).reshape(g.cell_shape())
    return lift, lift_p
