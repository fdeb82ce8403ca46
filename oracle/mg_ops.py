"""Oracle for single multigrid kernels of the pressure subsolve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module;
only ``tests/`` does.

The projection preconditioner (Sec. 4.2.4 names it; its algebra is this
build's reading) solves the pressure Poisson problem -L_rho phi = s with
L_rho = D beta G, beta = 1/rho on the faces (Sec. 4.2.2 uses the face density),
zero normal flux through walls.  Its multigrid is made of three kernels whose
results have plain definitions, written out here with numpy on full cell
arrays (C order (Nz, Ny, Nx), x fastest):

* ``apply``: y = -L_rho e, the five/seven-point flux form: on every interior
  face between cells a (lower index) and b, the flux F = beta (e_b - e_a) / h
  adds -F/h to cell a and +F/h to cell b; wall faces carry no flux.
* ``gs_colour`` / ``rb_gs_sweep``: red-black Gauss-Seidel.  The cells of one
  colour ((i+j+k) even = 0, odd = 1) are replaced by the value that zeroes
  their own residual row with every other value held fixed,
  g_c = (r_c + sum_nb w_nb e_nb) / sum_nb w_nb; cells of one colour never
  neighbour each other, so this is Gauss-Seidel in any order within the
  colour.  A sweep is colour 0 then colour 1.  With a relaxation factor
  omega != 1 (red-black SOR, the smoother's reading: the paper fixes no
  smoother) the cell takes e_c + omega (g_c - e_c) instead of g_c.
* ``residual_restrict``: the coarse right-hand side, the mean over the 2^d
  children of the fine residual r - (-L_rho) e.
* ``prolong``: the coarse correction on the fine cells, piecewise constant, or
  per axis 3/4 of the parent plus 1/4 of the parent's neighbour on the child's
  side (the parent itself beyond a wall).

``apply`` is pinned against the Kronecker-assembled operator of
``assemble.pressure_laplacian``; the others against brute-force loops and
their defining invariants (``tests/test_oracle_mg_ops.py``).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def betas(dim: int, rho_faces: Sequence[np.ndarray], open_top: bool = False):
    """beta = 1/rho on every interior face; wall faces hold 0 (no flux).  With the
    open top (the upper end of the vertical axis, zero pressure on its faces) the
    top faces keep 1/rho: ``apply`` gives them the Dirichlet flux."""
    out = []
    for c in range(dim):
        b = 1.0 / np.asarray(rho_faces[c], dtype=np.float64)
        sl = [slice(None)] * 3
        ends = (0,) if (open_top and c == dim - 1) else (0, -1)
        for end in ends:
            sl[2 - c] = end
            b[tuple(sl)] = 0.0
        out.append(b)
    return out


def _top(dim, beta):
    """beta on the open top's faces (array of the top cells' shape) or None."""
    v = dim - 1
    sl = [slice(None)] * 3
    sl[2 - v] = -1
    return beta[v][tuple(sl)]


def _top_cells(dim):
    sl = [slice(None)] * 3
    sl[2 - (dim - 1)] = -1
    return tuple(sl)


def _face_slices(c: int):
    """Slices of the lower cell, the upper cell and the interior faces along axis c."""
    ax = 2 - c
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    fi = [slice(None)] * 3
    lo[ax] = slice(0, -1)
    hi[ax] = slice(1, None)
    fi[ax] = slice(1, -1)
    return tuple(lo), tuple(hi), tuple(fi)


def apply(dim: int, h: Sequence[float], beta: Sequence[np.ndarray], e: np.ndarray,
          open_top: bool = False) -> np.ndarray:
    """y = -L_rho e = -D beta G e on cells (flux form, zero flux through walls).  On
    the open top the pressure is zero on the face, half a cell above the top cells'
    centres: the flux through it is beta (0 - e) / (h / 2)."""
    e = np.asarray(e, dtype=np.float64)
    y = np.zeros_like(e)
    for c in range(dim):
        lo, hi, fi = _face_slices(c)
        F = beta[c][fi] * (e[hi] - e[lo]) / h[c]
        y[lo] -= F / h[c]
        y[hi] += F / h[c]
    if open_top:
        v = dim - 1
        tc = _top_cells(dim)
        F = _top(dim, beta) * (0.0 - e[tc]) / (0.5 * h[v])
        y[tc] -= F / h[v]
    return y


def diagonal(dim: int, h: Sequence[float], beta: Sequence[np.ndarray], shape,
             open_top: bool = False) -> np.ndarray:
    """Diagonal of -L_rho: the sum of beta/h^2 over each cell's interior faces (and
    2 beta/h^2 for an open-top face)."""
    d = np.zeros(shape)
    for c in range(dim):
        lo, hi, fi = _face_slices(c)
        w = beta[c][fi] / (h[c] * h[c])
        d[lo] += w
        d[hi] += w
    if open_top:
        v = dim - 1
        d[_top_cells(dim)] += 2.0 * _top(dim, beta) / (h[v] * h[v])
    return d


def colour_mask(shape, colour: int) -> np.ndarray:
    k, j, i = np.indices(shape)
    return ((i + j + k) % 2) == colour


def gs_colour(dim, h, beta, e, r, colour, open_top=False, omega=1.0):
    """One colour of red-black Gauss-Seidel (SOR with factor omega) for
    -L_rho e = r (returns a new array)."""
    e = np.array(e, dtype=np.float64, copy=True)
    d = diagonal(dim, h, beta, e.shape, open_top)
    off = d * e - apply(dim, h, beta, e, open_top)          # sum_nb w_nb e_nb
    m = colour_mask(e.shape, colour)
    g = (r[m] + off[m]) / d[m]
    e[m] = g if omega == 1.0 else e[m] + omega * (g - e[m])
    return e


def rb_gs_sweep(dim, h, beta, e, r, open_top=False, omega=1.0):
    """One red-black Gauss-Seidel (SOR) sweep, colour 0 ((i+j+k) even) first."""
    e = gs_colour(dim, h, beta, e, r, 0, open_top, omega)
    return gs_colour(dim, h, beta, e, r, 1, open_top, omega)


def residual_restrict(dim, h, beta, e, r, open_top=False) -> np.ndarray:
    """Mean over the 2^d children of r - (-L_rho) e (even cell counts)."""
    res = np.asarray(r, dtype=np.float64) - apply(dim, h, beta, e, open_top)
    nz, ny, nx = res.shape
    if dim == 3:
        return res.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))
    return res.reshape(1, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4))


def _prolong_axis(a: np.ndarray, ax: int, lin: bool) -> np.ndarray:
    n = a.shape[ax]
    fine = np.arange(2 * n)
    parent = fine // 2
    out = np.take(a, parent, axis=ax)
    if not lin:
        return out
    nb = np.where(fine % 2 == 1, parent + 1, parent - 1)
    nb = np.clip(nb, 0, n - 1)
    return 0.75 * out + 0.25 * np.take(a, nb, axis=ax)


def prolong(dim: int, ec: np.ndarray, lin: bool = False) -> np.ndarray:
    """Coarse cell array -> fine cells (piecewise constant, or 3/4-1/4 per axis)."""
    out = np.asarray(ec, dtype=np.float64)
    for c in range(dim):
        out = _prolong_axis(out, 2 - c, lin)
    return out
