"""Oracle O1: the discrete Stokes system assembled as one sparse matrix.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module;
only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark do.

What is assembled is the linear system of the conservative momentum and
continuity equations on the MAC grid (Sec. 4.2.2, eq_c_discrete_momentum and
eq_c_discrete_continuity), with the implicit part of the viscous strain-rate
operator scaled by ``theta`` (theta = 1/2 is the Crank-Nicolson half of the
paper; theta = 1 is the full operator) and everything explicit moved to the
right-hand side:

    (rho_face/dt) u - theta * div_h[ mu (grad_h u + grad_h u^T) ] + grad_h p = f
                                                      -div_h u = g

Cell-centred p and mu, face-centred u, v, w (Sec. 3.1).  Viscosity is needed
on cell centres (normal stresses) and on edges (shear stresses); edge values
are the harmonic mean of the cells sharing the edge (Sec. 4.2, footnote on
harmonic averaging), with out-of-domain cells mirrored.

Boundaries: a wall axis has no-slip walls (normal velocity zero and not an
unknown; tangential ghost = -interior, i.e. zero wall value); the pressure
gradient lives only on interior faces.  A periodic axis wraps.  With
``open_top`` the upper end of the vertical axis (y in 2D, z in 3D) is the wave
tank's open top (Sec. 7.1: zero pressure and zero tangential velocity there):
the normal velocity on the top faces is an unknown, the pressure ghost above
the top is minus the cell below (zero pressure on the face, so the gradient on
the top face is -2 p / h), the tangential ghosts keep the no-slip rule, and the
normal viscous stress in the ghost cell above is likewise minus the cell below
(zero normal stress on the face: with zero tangential velocity on the top,
continuity gives d w / d z = 0 there; equivalently the normal velocity above the
top mirrors the one below it).

The matrix is built from 1D staggered difference operators combined with
Kronecker products (C order, x fastest), which is a literal transcription of
the staggered second-order differences rather than a stencil loop: the
independent stencil loop is the C oracle (``stokes_oracle.c``).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class OGrid:
    dim: int
    n: Tuple[int, int, int]
    h: Tuple[float, float, float]
    periodic: Tuple[bool, bool, bool] = (False, False, False)
    open_top: bool = False                 # upper end of axis dim-1: zero pressure, open

    @property
    def vert(self) -> int:
        return self.dim - 1

    def nf(self, axis: int) -> int:
        """Number of face positions along ``axis``."""
        return self.n[axis] if self.periodic[axis] else self.n[axis] + 1

    def comp_shape(self, comp: int) -> Tuple[int, int, int]:
        """(Nz, Ny, Nx)-ordered shape of velocity component ``comp``'s full array."""
        s = [self.n[2], self.n[1], self.n[0]]
        s[2 - comp] = self.nf(comp)
        return tuple(s)

    def cell_shape(self) -> Tuple[int, int, int]:
        return (self.n[2], self.n[1], self.n[0])


# --------------------------------------------------------------------------
# 1D staggered operators along one axis with N cells
# --------------------------------------------------------------------------
def _d1(N: int, h: float, periodic: bool, open_hi: bool = False):
    """Return the 1D building blocks along one axis.

    f2c : faces -> cells, (f[i+1] - f[i]) / h
    c2f : cells -> faces, (c[i] - c[i-1]) / h; zero rows on wall faces; on an
          open upper end (open_hi) the pressure ghost is -c[N-1]: -2 c[N-1] / h
    c2fv: the same for the normal viscous stress (equal to c2f: on an open upper
          end its ghost is also minus the cell below, zero normal stress on the face)
    t2e : cell-positioned tangential values -> face-positioned edges,
          (t[i] - t[i-1]) / h, with ghost t = -interior beyond a wall
    e2t : face-positioned edges -> cell positions, (e[i+1] - e[i]) / h
    avg : cells -> faces, (c[i-1] + c[i]) / 2 with mirrored out-of-domain cells
    """
    nf = N if periodic else N + 1
    f2c = sp.lil_matrix((N, nf))
    c2f = sp.lil_matrix((nf, N))
    t2e = sp.lil_matrix((nf, N))
    e2t = sp.lil_matrix((N, nf))
    avg = sp.lil_matrix((nf, N))
    for i in range(N):
        ip = (i + 1) % nf
        f2c[i, ip] += 1.0 / h
        f2c[i, i] -= 1.0 / h
        e2t[i, ip] += 1.0 / h
        e2t[i, i] -= 1.0 / h
    for i in range(nf):
        if periodic:
            im = (i - 1) % N
            c2f[i, i] += 1.0 / h
            c2f[i, im] -= 1.0 / h
            t2e[i, i] += 1.0 / h
            t2e[i, im] -= 1.0 / h
            avg[i, i] += 0.5
            avg[i, im] += 0.5
        else:
            if 0 < i < N:
                c2f[i, i] += 1.0 / h
                c2f[i, i - 1] -= 1.0 / h
            # t[i] - t[i-1] with t[-1] = -t[0] and t[N] = -t[N-1]
            if i < N:
                t2e[i, i] += 1.0 / h
            else:
                t2e[i, N - 1] -= 1.0 / h
            if i > 0:
                t2e[i, i - 1] -= 1.0 / h
            else:
                t2e[i, 0] += 1.0 / h
            lo = max(i - 1, 0)
            hi = min(i, N - 1)
            avg[i, lo] += 0.5
            avg[i, hi] += 0.5
    if open_hi and not periodic:
        c2f[N, N - 1] -= 2.0 / h
    c2fv = c2f.copy()
    cv = lambda m: sp.csr_matrix(m)
    return dict(f2c=cv(f2c), c2f=cv(c2f), c2fv=cv(c2fv), t2e=cv(t2e), e2t=cv(e2t), avg=cv(avg),
                Ic=sp.identity(N, format="csr"), If=sp.identity(nf, format="csr"))


def _k3(ox, oy, oz):
    """Kronecker product acting on C-ordered (z, y, x) arrays, x fastest."""
    return sp.kron(oz, sp.kron(oy, ox, format="csr"), format="csr")


class Assembler:
    """Assembles the full-array operators for one grid."""

    def __init__(self, g: OGrid):
        self.g = g
        ax = []
        for a in range(3):
            if a < g.dim:
                ax.append(_d1(g.n[a], g.h[a], g.periodic[a], g.open_top and a == g.dim - 1))
            else:
                one = sp.identity(1, format="csr")
                ax.append(dict(Ic=one, If=one))
        self.ax = ax

    def _ops(self, spec):
        """spec[a] names the 1D operator along axis a (x, y, z)."""
        return _k3(self.ax[0][spec[0]], self.ax[1][spec[1]], self.ax[2][spec[2]])

    def _pos(self, comp: Optional[int], edge: Optional[Tuple[int, int]] = None):
        """Position letters for each axis: 'f' on face positions, 'c' on cell positions."""
        pos = ["c", "c", "c"]
        if comp is not None:
            pos[comp] = "f"
        if edge is not None:
            pos[edge[0]] = "f"
            pos[edge[1]] = "f"
        return pos

    def _op_along(self, axis, name, pos_in):
        """Apply 1D op ``name`` along ``axis`` and identities elsewhere."""
        spec = []
        for a in range(3):
            if a == axis:
                spec.append(name)
            else:
                spec.append("If" if pos_in[a] == "f" else "Ic")
        return self._ops(spec)

    # ---- pieces -------------------------------------------------------------
    def grad(self, comp):
        """Pressure gradient onto the faces of component ``comp`` (zero on wall faces)."""
        return self._op_along(comp, "c2f", self._pos(None))

    def div(self, comp):
        """Divergence contribution of component ``comp`` at cells."""
        return self._op_along(comp, "f2c", self._pos(comp))

    def edge_pairs(self):
        d = self.g.dim
        return [(a, b) for a in range(d) for b in range(a + 1, d)]

    def edge_mu(self, mu_cell: np.ndarray, a: int, b: int) -> np.ndarray:
        """Harmonic mean of mu over the cells around each (a, b) edge, mirrored at walls
        (a zero-viscosity cell makes its edges' mean zero: 1/0 = inf, 1/inf = 0)."""
        with np.errstate(divide="ignore"):
            inv = 1.0 / mu_cell.ravel()
        pos = self._pos(None)
        m1 = self._op_along(a, "avg", pos)
        pos_a = list(pos)
        pos_a[a] = "f"
        m2 = self._op_along(b, "avg", pos_a)
        return 1.0 / (m2 @ (m1 @ inv))

    def viscous(self, mu_cell: np.ndarray):
        """Block matrix L[c][d]: component d -> component c of div[mu (grad u + grad u^T)]."""
        d = self.g.dim
        mu = mu_cell.ravel()
        L = [[None] * d for _ in range(d)]
        for c in range(d):
            # normal stress 2 mu du_c/dx_c at cells, differenced back to c-faces
            f2c = self._op_along(c, "f2c", self._pos(c))
            c2f = self._op_along(c, "c2fv", self._pos(None))
            # c2f on a wall axis has zero rows on wall faces; the interior stencil
            # (tau[i] - tau[i-1]) / h is what the momentum row needs.
            L[c][c] = c2f @ sp.diags(2.0 * mu) @ f2c
        for a, b in self.edge_pairs():
            me = sp.diags(self.edge_mu(mu_cell, a, b))
            epos = self._pos(None, (a, b))
            # shear strain at (a,b) edges: du_a/dx_b + du_b/dx_a
            Sa = self._op_along(b, "t2e", self._pos(a))   # from u_a
            Sb = self._op_along(a, "t2e", self._pos(b))   # from u_b
            # divergence of the shear stress back onto each component's faces
            Da = self._op_along(b, "e2t", epos)           # onto u_a faces
            Db = self._op_along(a, "e2t", epos)           # onto u_b faces
            L[a][a] = L[a][a] + Da @ me @ Sa
            L[a][b] = (Da @ me @ Sb) if L[a][b] is None else L[a][b] + Da @ me @ Sb
            L[b][b] = L[b][b] + Db @ me @ Sb
            L[b][a] = (Db @ me @ Sa) if L[b][a] is None else L[b][a] + Db @ me @ Sa
        for c in range(d):
            for e in range(d):
                if L[c][e] is None:
                    L[c][e] = sp.csr_matrix((L[c][c].shape[0], L[e][e].shape[1]))
        return L

    # ---- unknown selection --------------------------------------------------
    def select(self, comp: Optional[int]):
        """Selection matrix from a full array to its unknowns (wall-normal faces dropped)."""
        g = self.g
        if comp is None:
            n = int(np.prod(g.cell_shape()))
            return sp.identity(n, format="csr")
        shape = g.comp_shape(comp)
        mask = np.ones(shape, dtype=bool)
        if not g.periodic[comp]:
            sl = [slice(None)] * 3
            sl[2 - comp] = 0
            mask[tuple(sl)] = False
            if not (g.open_top and comp == g.dim - 1):      # the open top's faces are unknowns
                sl[2 - comp] = -1
                mask[tuple(sl)] = False
        idx = np.flatnonzero(mask.ravel())
        S = sp.csr_matrix((np.ones(idx.size), (np.arange(idx.size), idx)),
                          shape=(idx.size, mask.size))
        return S


@dataclasses.dataclass
class System:
    K: sp.csr_matrix            # [A G; -D 0] on unknowns
    A: sp.csr_matrix
    G: sp.csr_matrix
    D: sp.csr_matrix
    sel: List[sp.csr_matrix]    # per component + pressure
    sizes: List[int]
    grid: OGrid

    def pack(self, fu: Sequence[np.ndarray], fp: np.ndarray) -> np.ndarray:
        parts = [self.sel[c] @ np.asarray(fu[c], dtype=np.float64).ravel()
                 for c in range(self.grid.dim)]
        parts.append(np.asarray(fp, dtype=np.float64).ravel())
        return np.concatenate(parts)

    def unpack(self, x: np.ndarray):
        out = []
        off = 0
        for c in range(self.grid.dim):
            m = self.sizes[c]
            full = self.sel[c].T @ x[off:off + m]
            out.append(full.reshape(self.grid.comp_shape(c)))
            off += m
        p = x[off:].reshape(self.grid.cell_shape())
        return out, p

    @property
    def n_vel(self) -> int:
        return sum(self.sizes[:-1])


def assemble(g: OGrid, rho_faces: Sequence[np.ndarray], mu_cell: np.ndarray, dt: float,
             theta: float = 1.0) -> System:
    """Assemble K = [A G; -D 0] over the unknowns of grid ``g``.

    ``rho_faces[c]`` is the full face array of component c (shape ``g.comp_shape(c)``),
    ``mu_cell`` the cell viscosity.  ``A = diag(rho_face/dt) - theta * L_mu``.
    """
    asm = Assembler(g)
    d = g.dim
    L = asm.viscous(np.asarray(mu_cell, dtype=np.float64))
    S = [asm.select(c) for c in range(d)] + [asm.select(None)]
    blocksA = [[None] * d for _ in range(d)]
    for c in range(d):
        for e in range(d):
            blk = -theta * L[c][e]
            if c == e:
                blk = blk + sp.diags(np.asarray(rho_faces[c], dtype=np.float64).ravel() / dt)
            blocksA[c][e] = S[c] @ blk @ S[e].T
    A = sp.bmat(blocksA, format="csr")
    G = sp.vstack([S[c] @ asm.grad(c) for c in range(d)], format="csr")
    D = sp.hstack([asm.div(c) @ S[c].T for c in range(d)], format="csr")
    K = sp.bmat([[A, G], [-D, None]], format="csr")
    sizes = [S[c].shape[0] for c in range(d)] + [S[d].shape[0]]
    return System(K=K, A=A, G=G, D=D, sel=S, sizes=sizes, grid=g)


def pressure_laplacian(g: OGrid, rho_faces: Sequence[np.ndarray]) -> sp.csr_matrix:
    """-L_rho = -D beta G on cells, beta = 1/rho on faces (the projection's Poisson operator)."""
    asm = Assembler(g)
    terms = []
    for c in range(g.dim):
        beta = 1.0 / np.asarray(rho_faces[c], dtype=np.float64).ravel()
        terms.append(asm.div(c) @ sp.diags(beta) @ asm.grad(c))
    return -sum(terms[1:], terms[0])


def from_problem(prob, theta: float = 1.0, open_top: bool = False) -> System:
    """Assemble the system of a ``workloads.Problem`` (all walls, or the open top)."""
    g = OGrid(prob.dim, tuple(prob.n), tuple(prob.h), open_top=open_top)
    return assemble(g, prob.rho_faces, prob.mu, prob.dt, theta)


def explicit_rhs(g: OGrid, rho_faces: Sequence[np.ndarray], mu_cell: np.ndarray, dt: float,
                 theta: float, u_n: Sequence[np.ndarray],
                 rho_force: Optional[Sequence[np.ndarray]] = None,
                 gravity: Sequence[float] = (0.0, 0.0, 0.0)) -> List[np.ndarray]:
    """Momentum right-hand side of one time step built from the old velocity.

    Moving the explicit terms of the paper's discrete momentum equations to the
    right (Sec. 4.2.2, eq_nc_discrete_momentum; eq_c_discrete_momentum with the
    old density as ``rho_faces``) gives, with the viscous term split as
    theta (new) + (1 - theta) (old) (theta = 1/2: Crank-Nicolson),

        f = (rho/dt) u^n + (1 - theta) L_mu u^n + rho_force g

    on every interior face (0 on wall-normal faces), where L_mu is the same
    strain-rate operator as in the system matrix (built here from ``mu_cell``,
    the old viscosity) and rho_force is the density of the gravity force (the
    flow-only density for the well-balanced form, Sec. 5).  The convective
    term is the caller's.
    """
    asm = Assembler(g)
    d = g.dim
    L = asm.viscous(np.asarray(mu_cell, dtype=np.float64))
    S = [asm.select(c) for c in range(d)]
    mask = [S[c].T @ S[c] for c in range(d)]             # keep interior faces, zero wall-normal ones
    un = [mask[c] @ np.asarray(u_n[c], dtype=np.float64).ravel() for c in range(d)]
    out = []
    for c in range(d):
        f = np.asarray(rho_faces[c], dtype=np.float64).ravel() / dt * un[c]
        f = f + (1.0 - theta) * sum(L[c][e] @ un[e] for e in range(d))
        if rho_force is not None:
            f = f + np.asarray(rho_force[c], dtype=np.float64).ravel() * gravity[c]
        out.append((mask[c] @ f).reshape(g.comp_shape(c)))
    return out
