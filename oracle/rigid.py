"""Oracle of the rigid-body constraint projection that follows the Stokes solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module;
only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark do.

What is computed (plain FP64 numpy, one marker at a time):

* the four-point regularised delta function of Peskin (2002), cited by the
  paper for its interpolation and spreading (Sec. 3.3):
  phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4r^2)) / 8 for |r| <= 1,
           (5 - 2|r| - sqrt(-7 + 12|r| - 4r^2)) / 8 for 1 <= |r| <= 2, 0 beyond,
  and delta_h(x) = prod_d phi(x_d / h_d) / h_d;
* velocity interpolation U = J u (Sec. 3.3): each component of the marker
  velocity is the sum over that component's face points of u delta_h(x - X)
  times the cell volume;
* force spreading f = S F: each face value is the sum over markers of
  F delta_h(x - X) times the marker volume;
* near the no-slip walls (Sec. 3.3, the adjoint pair S_BC = J_BC^*): stencil
  points beyond a wall take the value of their mirror image across the wall
  with the sign flipped (the velocity vanishes on the wall and the ghost is
  the odd reflection); wall-normal points on the wall itself hold zero; the
  spreading is the exact transpose (spread to the ghost points, then add the
  ghost values, sign flipped, onto their mirror images);
* the rigid-body projection (Sec. 4.2.5, eqs. eq_velocity_correction,
  eq_prescribed_velocity, eq_linear_conservation, eq_angular_conservation):
  u = u~ + S(U_b - J u~) with U_b = U_r + W_r x R, R = X - X_com, where
  (U_r, W_r) are given (prescribed motion) or follow from redistributing the
  linear and angular momentum of J u~ over the markers (free body):
  M U_r = sum J u~ dV,  I W_r = sum R x (J u~) dV,
  M = sum dV,  I = sum (R.R Id - R (x) R) dV.
  (The paper's inertia sum omits the marker volume; with a uniform volume and
  density both sides scale alike, so the volume is kept on both.)  In 2D the
  angular velocity is a scalar about z and I = sum |R|^2 dV.

Layouts as the solver's: u is (Nz, Ny, Nx+1), v (Nz, Ny+1, Nx), w
(Nz+1, Ny, Nx) (2D: Nz = 1, no w); markers X is (n, dim).
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


def peskin4(r):
    """Peskin's four-point kernel phi(r) (vectorised)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    inner = (3.0 - 2.0 * a + np.sqrt(np.maximum(1.0 + 4.0 * a - 4.0 * a * a, 0.0))) / 8.0
    outer = (5.0 - 2.0 * a - np.sqrt(np.maximum(-7.0 + 12.0 * a - 4.0 * a * a, 0.0))) / 8.0
    return np.where(a <= 1.0, inner, np.where(a <= 2.0, outer, 0.0))


def _axis_points(comp: int, axis: int, x: float, h: float, n: int):
    """The four points of one axis of the stencil of component ``comp`` at marker
    coordinate ``x``: list of (array index, kernel weight, sign) after the wall
    mirror.  Index ranges: normal axis faces 0..n (0 and n on the walls),
    tangential axes cells 0..n-1."""
    out = []
    if axis == comp:                              # face positions i*h
        base = math.floor(x / h) - 1
        for i in range(base, base + 4):
            w = float(peskin4(i - x / h))
            if i < 0:
                out.append((-i, w, -1.0))
            elif i > n:
                out.append((2 * n - i, w, -1.0))
            elif i == 0 or i == n:
                out.append((i, w, 0.0))
            else:
                out.append((i, w, 1.0))
    else:                                         # cell-centre positions (j + 1/2) h
        base = math.floor(x / h - 0.5) - 1
        for j in range(base, base + 4):
            w = float(peskin4(j + 0.5 - x / h))
            if j < 0:
                out.append((-1 - j, w, -1.0))
            elif j >= n:
                out.append((2 * n - 1 - j, w, -1.0))
            else:
                out.append((j, w, 1.0))
    return out


def _stencil(comp, X, n, h, dim):
    """(flat index into the component's array, weight*sign) for every stencil point
    of one marker, in the array layout of that component."""
    shape = [n[0], n[1], n[2] if dim == 3 else 1]
    shape[comp] += 1
    axes = [_axis_points(comp, d, X[d], h[d], n[d]) for d in range(dim)]
    pts = []
    if dim == 2:
        for (i, wi, si) in axes[0]:
            for (j, wj, sj) in axes[1]:
                pts.append((i + shape[0] * j, wi * wj * si * sj))
    else:
        for (i, wi, si) in axes[0]:
            for (j, wj, sj) in axes[1]:
                for (k, wk, sk) in axes[2]:
                    pts.append((i + shape[0] * (j + shape[1] * k), wi * wj * wk * si * sj * sk))
    return pts


def interpolate(u: Sequence[np.ndarray], X: np.ndarray, n, h, dim: int) -> np.ndarray:
    """U = J_BC u at every marker, shape (n_markers, dim)."""
    U = np.zeros((X.shape[0], dim))
    flat = [np.asarray(u[c], dtype=np.float64).ravel() for c in range(dim)]
    for m in range(X.shape[0]):
        for c in range(dim):
            U[m, c] = sum(flat[c][q] * w for q, w in _stencil(c, X[m], n, h, dim))
    return U


def spread(F: np.ndarray, X: np.ndarray, dV: float, n, h, dim: int, shapes) -> List[np.ndarray]:
    """f = S_BC F on the face arrays (``shapes`` their shapes): the transpose of
    ``interpolate`` weighted by dV / (cell volume)."""
    vol = float(np.prod(h[:dim]))
    f = [np.zeros(int(np.prod(s))) for s in shapes]
    for m in range(X.shape[0]):
        for c in range(dim):
            for q, w in _stencil(c, X[m], n, h, dim):
                f[c][q] += w * F[m, c] * dV / vol
    return [a.reshape(s) for a, s in zip(f, shapes)]


def cross(a, b, dim):
    if dim == 2:                                  # z-component of a x b
        return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    return np.cross(a, b)


def rigid_velocity(U_r, W_r, R, dim):
    """U_b = U_r + W_r x R for every marker (2D: W_r is the z-rotation rate)."""
    if dim == 2:
        w = float(np.ravel(W_r)[0])
        return np.asarray(U_r)[None, :2] + w * np.stack([-R[:, 1], R[:, 0]], axis=1)
    return np.asarray(U_r)[None, :] + np.cross(np.asarray(W_r)[None, :], R)


def free_body_velocity(JU: np.ndarray, R: np.ndarray, dV: float, dim: int):
    """(U_r, W_r) from the momentum of J u~ over the markers."""
    M = dV * JU.shape[0]
    U_r = JU.sum(axis=0) * dV / M
    L = (cross(R, JU, dim) * dV).sum(axis=0)
    if dim == 2:
        I = float((R * R).sum() * dV)
        return U_r, np.array([L / I])
    I = np.zeros((3, 3))
    for r in R:
        I += (np.dot(r, r) * np.eye(3) - np.outer(r, r)) * dV
    return U_r, np.linalg.solve(I, L)


def rigid_projection(u: Sequence[np.ndarray], X: np.ndarray, dV: float, x_com, n, h, dim: int,
                     free_body: bool, U_r=None, W_r=None):
    """Corrected velocity u = u~ + S(U_b - J u~), and the body's (U_r, W_r)."""
    X = np.asarray(X, dtype=np.float64)
    R = X - np.asarray(x_com, dtype=np.float64)[None, :dim]
    JU = interpolate(u, X, n, h, dim)
    if free_body:
        U_r, W_r = free_body_velocity(JU, R, dV, dim)
    Ub = rigid_velocity(np.asarray(U_r, dtype=np.float64), np.asarray(W_r, dtype=np.float64), R, dim)
    corr = spread(Ub - JU, X, dV, n, h, dim, [np.asarray(a).shape for a in u[:dim]])
    return [np.asarray(u[c], dtype=np.float64) + corr[c] for c in range(dim)], np.asarray(U_r), np.asarray(W_r)
