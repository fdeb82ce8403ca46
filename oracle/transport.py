"""Oracle for the face-density transport of the conservative scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module;
only ``tests/`` does.

What it computes (Sec. 4.2.2, eqs. eq_rk1, eq_rk2 and eq_rk3): the density
vector on the faces of the staggered grid is advanced by the three-stage
strong-stability-preserving Runge-Kutta scheme

    rho1 = rho_n - dt R(u1, rho_n)
    rho2 = 3/4 rho_n + 1/4 rho1 - 1/4 dt R(u2, rho1)
    rho  = 1/3 rho_n + 2/3 rho2 - 2/3 dt R(u3, rho2)

where R(u, rho) is the divergence of the flux u_adv rho_lim over the control
volume of each face (the face-centred control volume of the MAC grid), and
u1, u2, u3 are the stage velocities (the paper extrapolates them from u^n,
u^{n-1} and the latest iterate; they are the caller's).  The paper defers the
construction of u_adv and rho_lim to an earlier paper; the reading written out
here (recorded in the design notes):

* Control volume of a face normal to axis c: one cell long in every
  direction, centred on the face.  Its two faces normal to c lie at the cell
  centres on either side; its faces normal to another axis d lie on the cell
  edges between the face and its neighbour along d.
* Advective velocity on a control-volume face normal to d: the mean of the two
  d-velocities nearest to it -- along c itself the two c-faces around the cell
  centre, across (d != c) the two d-faces on either side of the edge along c.
  Wall-normal velocities are zero, so nothing crosses a wall.
* Limited density on a control-volume face: cubic upwind interpolation with
  the CUI limiter, in normalised variables along d from the upwind-side
  values U (far upwind), C (upwind), D (downwind) of the density being
  transported: with r = (C - U) / (D - U),
      f(r) = 3 r            for 0 < r <= 2/13
           = 5/6 r + 1/3    for 2/13 < r <= 4/5
           = 1              for 4/5 < r < 1
           = r              otherwise (first-order upwind),
  rho_lim = U + f(r) (D - U), and rho_lim = C when D = U.  The middle branch
  is the unlimited third-order upwind value (-U + 5 C + 2 D) / 6.  This is the
  CUI scheme of Waterson and Deconinck (2007), which the paper cites.
* Density beyond a wall (only ever a far-upwind value U): homogeneous Neumann
  mirror -- along the face's own axis about the wall face (index -1 -> 1),
  across it about the wall (index -1 -> 0).
* Wall-normal faces are not transported: their densities are boundary values
  and are returned as given (rho_n); the solve never uses them.

Everything is plain numpy on full face arrays in the solver's layouts
(C order (Nz, Ny, Nx), x fastest; u (Nz, Ny, Nx+1), v (Nz, Ny+1, Nx),
w (Nz+1, Ny, Nx)).  Pins: tests/test_oracle_transport.py.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

CUI_A = 2.0 / 13.0
CUI_B = 4.0 / 5.0


def cui_face(U, C, D):
    """Limited face value from far-upwind U, upwind C and downwind D (arrays)."""
    U, C, D = (np.asarray(a, dtype=np.float64) for a in (U, C, D))
    den = D - U
    out = C.copy()
    ok = den != 0.0
    r = np.zeros_like(C)
    r[ok] = (C[ok] - U[ok]) / den[ok]
    f = r.copy()
    m1 = ok & (r > 0.0) & (r <= CUI_A)
    m2 = ok & (r > CUI_A) & (r <= CUI_B)
    m3 = ok & (r > CUI_B) & (r < 1.0)
    f[m1] = 3.0 * r[m1]
    f[m2] = (5.0 / 6.0) * r[m2] + 1.0 / 3.0
    f[m3] = 1.0
    out[ok] = U[ok] + f[ok] * den[ok]
    return out


def _ax(comp: int) -> int:
    """Array axis (of a (z, y, x) array) of grid axis comp."""
    return 2 - comp


def _pad_mirror(a: np.ndarray, ax: int, face_axis: bool) -> np.ndarray:
    """Two ghost layers on both ends of array axis ax: mirror about the wall face
    (face_axis: index -1 -> 1, -2 -> 2) or about the wall (-1 -> 0, -2 -> 1)."""
    n = a.shape[ax]
    if face_axis:
        lo = [2, 1]
        hi = [n - 2, n - 3]
    else:
        lo = [1, 0]
        hi = [n - 1, n - 2]
    idx = lo + list(range(n)) + hi
    return np.take(a, idx, axis=ax)


def advective_velocity(dim: int, u: Sequence[np.ndarray], comp: int, d: int) -> np.ndarray:
    """Velocity normal to the control-volume faces of comp-faces that are normal to d.

    Shape: comp's face array shape with one more entry along d (the control
    volume faces at both ends of every face), i.e. index m along d is the
    control-volume face between face m-1 and face m of the array (m = 0 and the
    last are beyond the ends and hold zero flux there)."""
    ud = np.asarray(u[d], dtype=np.float64)
    if d == comp:
        # faces normal to comp at cell centres: mean of the comp-faces on either side;
        # the array of comp-faces has n+1 entries along comp, cell centres n, plus the
        # two outer ends (beyond the wall faces: zero)
        a = 0.5 * (np.take(ud, range(0, ud.shape[_ax(d)] - 1), axis=_ax(d)) +
                   np.take(ud, range(1, ud.shape[_ax(d)]), axis=_ax(d)))
        z = np.zeros_like(np.take(a, [0], axis=_ax(d)))
        return np.concatenate([z, a, z], axis=_ax(d))
    # d != comp: control-volume faces on the edges between comp-faces along d.  For the
    # comp-face with index i along comp, the two nearest d-velocities are the d-faces of
    # the cells i-1 and i (at the edge's index along d).  Wall comp-faces (i = 0 and the
    # last) are not transported; their entries are set to zero.
    pad = [(0, 0)] * 3
    pad[_ax(comp)] = (1, 1)
    ext = np.pad(ud, pad, mode="constant")
    n = ud.shape[_ax(comp)]
    left = np.take(ext, range(0, n + 1), axis=_ax(comp))     # cell i-1
    right = np.take(ext, range(1, n + 2), axis=_ax(comp))    # cell i
    a = 0.5 * (left + right)
    for end in (0, n):
        sl = [slice(None)] * 3
        sl[_ax(comp)] = end
        a[tuple(sl)] = 0.0
    return a


def flux_divergence(dim: int, h: Sequence[float], u: Sequence[np.ndarray], rho: Sequence[np.ndarray]) -> List[np.ndarray]:
    """R(u, rho): per face component, the divergence of u_adv rho_lim over each
    face's control volume; zero on wall-normal faces."""
    out = []
    for c in range(dim):
        rc = np.asarray(rho[c], dtype=np.float64)
        R = np.zeros_like(rc)
        for d in range(dim):
            ax = _ax(d)
            a = advective_velocity(dim, u, c, d)           # n_d + 1 entries along ax
            g = _pad_mirror(rc, ax, face_axis=(d == c))      # 2 ghosts each end
            n = rc.shape[ax]
            # control-volume face m (0..n) between entries m-1 and m: stencil in padded
            # index space p = m + 2: values at m-2, m-1, m, m+1 -> padded m, m+1, m+2, m+3
            v0 = np.take(g, range(0, n + 1), axis=ax)      # m-2
            v1 = np.take(g, range(1, n + 2), axis=ax)      # m-1
            v2 = np.take(g, range(2, n + 3), axis=ax)      # m
            v3 = np.take(g, range(3, n + 4), axis=ax)      # m+1
            pos = a > 0.0
            lim = np.where(pos, cui_face(v0, v1, v2), cui_face(v3, v2, v1))
            F = a * lim
            R += (np.take(F, range(1, n + 1), axis=ax) - np.take(F, range(0, n), axis=ax)) / h[d]
        sl = [slice(None)] * 3
        for end in (0, -1):
            sl[_ax(c)] = end
            R[tuple(sl)] = 0.0
        out.append(R)
    return out


def _keep_walls(dim, rho, rn):
    """Wall-normal faces hold rho_n in every stage."""
    for c in range(dim):
        sl = [slice(None)] * 3
        for end in (0, -1):
            sl[_ax(c)] = end
            rho[c][tuple(sl)] = rn[c][tuple(sl)]
    return rho


def ssp_rk3(dim: int, h: Sequence[float], dt: float, rho_n: Sequence[np.ndarray],
            u_stages: Sequence[Sequence[np.ndarray]]) -> List[np.ndarray]:
    """Three-stage SSP-RK3 update of the face densities; wall-normal faces keep rho_n."""
    rn = [np.asarray(rho_n[c], dtype=np.float64) for c in range(dim)]
    R1 = flux_divergence(dim, h, u_stages[0], rn)
    r1 = _keep_walls(dim, [rn[c] - dt * R1[c] for c in range(dim)], rn)
    R2 = flux_divergence(dim, h, u_stages[1], r1)
    r2 = _keep_walls(dim, [0.75 * rn[c] + 0.25 * r1[c] - 0.25 * dt * R2[c] for c in range(dim)], rn)
    R3 = flux_divergence(dim, h, u_stages[2], r2)
    out = [rn[c] / 3.0 + (2.0 / 3.0) * r2[c] - (2.0 / 3.0) * dt * R3[c] for c in range(dim)]
    return _keep_walls(dim, out, rn)
