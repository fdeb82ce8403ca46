"""Oracle of the coefficient step: material fields from level sets.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module;
only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark do.

What is computed (plain definitions, FP64, vectorised numpy):

* the smoothed Heaviside of a signed distance over ``eps = n_cells * hx``
  (Sec. 4.1, eq_heaviside): 0 below -eps, 1 above +eps, and in the band
  H = (1 + phi/eps + sin(pi phi/eps)/pi) / 2;
* the two-step property law (Sec. 4.1): first the flowing phase from the
  liquid/gas level set, zeta_flow = zeta_l + (zeta_g - zeta_l) H(phi)
  (eq_ls_flow; liquid where phi < 0), then the solid,
  zeta = zeta_s + (zeta_flow - zeta_s) H(psi) (eq_ls_solid; solid where
  psi < 0).  Several solids, each with its own level set and density, are
  applied in turn in the order given;
* viscosity at cell centres from the cell level sets; density on the faces
  of the staggered grid from the level sets averaged onto the faces
  (Sec. 4.2.2: the face density is set from level sets averaged onto faces),
  an interior face taking the mean of its two cells and a boundary face the
  one cell it touches (a mirror ghost);
* the flow-only face density (no solid), which the well-balanced gravity
  force uses (Sec. 5).

Layouts are C order with x fastest: cell fields (Nz, Ny, Nx), x-faces
(Nz, Ny, Nx+1), y-faces (Nz, Ny+1, Nx), z-faces (Nz+1, Ny, Nx).  In 2D
Nz = 1 and there are no z-faces.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np


def heaviside(phi, eps):
    """Smoothed Heaviside of eq_heaviside, evaluated pointwise in FP64."""
    phi = np.asarray(phi, dtype=np.float64)
    band = 0.5 * (1.0 + phi / eps + np.sin(np.pi * phi / eps) / np.pi)
    return np.select([phi < -eps, phi > eps], [0.0, 1.0], default=band)


def flow_law(zeta_l, zeta_g, h_flow):
    """eq_ls_flow: the property of the flowing (liquid/gas) phase."""
    return zeta_l + (zeta_g - zeta_l) * h_flow


def solid_law(zeta_s, zeta_flow, h_body):
    """eq_ls_solid: the solid overrides the flowing phase where psi < 0."""
    return zeta_s + (zeta_flow - zeta_s) * h_body


def to_faces(cell, axis):
    """Level set averaged onto the faces normal to ``axis`` (0 = x, 1 = y, 2 = z).

    The cell array is extended by one copy of its first and last layer along
    the axis (mirror ghosts); each face then takes the mean of the two layers
    on either side of it.
    """
    a = 2 - axis                                  # numpy axis of this grid axis
    pad = [(0, 0)] * cell.ndim
    pad[a] = (1, 1)
    e = np.pad(np.asarray(cell, dtype=np.float64), pad, mode="edge")
    lo = np.take(e, np.arange(0, e.shape[a] - 1), axis=a)
    hi = np.take(e, np.arange(1, e.shape[a]), axis=a)
    return 0.5 * (lo + hi)


def coefficients(dim: int, h: Sequence[float], phi: np.ndarray, psis: Sequence[np.ndarray],
                 rho_solid: Sequence[float], mu_solid: Sequence[float],
                 rho_l: float, rho_g: float, mu_l: float, mu_g: float, n_cells: float):
    """Face densities, cell viscosity and flow-only face densities.

    Returns (rho_faces, mu_cell, rho_flow_faces), the face lists holding
    ``dim`` arrays (x, y[, z]).
    """
    eps = n_cells * h[0]
    phi = np.asarray(phi, dtype=np.float64)
    mu = flow_law(mu_l, mu_g, heaviside(phi, eps))
    for ps, ms in zip(psis, mu_solid):
        mu = solid_law(ms, mu, heaviside(ps, eps))
    rho_faces: List[np.ndarray] = []
    rho_flow: List[np.ndarray] = []
    for ax in range(dim):
        r = flow_law(rho_l, rho_g, heaviside(to_faces(phi, ax), eps))
        rho_flow.append(r)
        for ps, rs in zip(psis, rho_solid):
            r = solid_law(rs, r, heaviside(to_faces(ps, ax), eps))
        rho_faces.append(r)
    return rho_faces, mu, rho_flow
