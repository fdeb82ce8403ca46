"""Oracle O5: direct solves of the assembled Stokes system.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The solve's answer has a plain definition: the solution of K x = b (Sec. 4.2.2,
eq_c_discrete_momentum/eq_c_discrete_continuity) with the pressure fixed to
zero mean.  With no-slip walls on every side the matrix has the one-dimensional
null space (u, p) = (0, const), and every right-hand side whose continuity part
has zero mean is consistent.  The solve borders K with that null vector:

    [ K   n ] [x]   [b]
    [ n^T 0 ] [l] = [0],   n = (0, ..., 0, 1, ..., 1) over the pressure cells,

which is nonsingular, returns l = 0 for consistent b, and gives the zero-mean
pressure.  Small systems use dense LAPACK (numpy) on that bordered matrix;
larger ones use SuperLU (scipy) with one pressure unknown pinned instead,
then shift the pressure to zero mean (the same solution).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import System


def _null_vector(sys: System, has_null: bool):
    n = sys.K.shape[0]
    v = np.zeros(n)
    if has_null:
        v[sys.n_vel:] = 1.0
    return v


def solve(sys: System, b: np.ndarray, dense: bool | None = None, has_null: bool = True):
    """Solve K x = b with the pressure mean fixed at zero.

    ``has_null`` is True when the pressure is defined only up to a constant
    (every boundary a wall, or every axis periodic).  The continuity part of b
    is made mean-free first; the amount removed is returned with the solution.
    """
    b = np.array(b, dtype=np.float64)
    gmean = 0.0
    if has_null:
        gmean = b[sys.n_vel:].mean()
        b[sys.n_vel:] -= gmean
    n = sys.K.shape[0]
    if dense is None:
        dense = n <= 3000
    if dense:
        if has_null:
            nv = _null_vector(sys, True)
            Kb = sp.bmat([[sys.K, sp.csr_matrix(nv[:, None])],
                          [sp.csr_matrix(nv[None, :]), None]], format="csr").toarray()
            rhs = np.concatenate([b, [0.0]])
        else:
            Kb, rhs = sys.K.toarray(), b
        return np.linalg.solve(Kb, rhs)[:n], gmean
    if not has_null:
        return spla.spsolve(sys.K.tocsc(), b), gmean
    # Sparse: a dense border row ruins the fill-reducing ordering, so instead
    # fix the last pressure unknown to zero (drop its row and column; with a
    # consistent b that continuity row is the sum of the others) and shift the
    # pressure to zero mean afterwards.
    keep = np.arange(n - 1)
    Kr = sys.K[keep][:, keep].tocsc()
    xr = spla.spsolve(Kr, b[keep], permc_spec="COLAMD")
    x = np.concatenate([xr, [0.0]])
    x[sys.n_vel:] -= x[sys.n_vel:].mean()
    return x, gmean


def solve_problem(prob, sys: System, dense: bool | None = None):
    """Direct solve of a ``workloads.Problem``; returns (u_list, p) in the API layout."""
    b = sys.pack(prob.rhs_u, prob.rhs_p)
    x, _ = solve(sys, b, dense=dense)
    return sys.unpack(x)
