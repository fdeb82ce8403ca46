"""Seeded synthetic inputs for the variable-coefficient Stokes solve.

This module only *generates* inputs: grids, level sets, material fields and
right-hand sides.  It holds none of the solver's arithmetic (no operator, no
smoother, no Krylov step), so both the oracle under ``oracle/`` and the HIP
path may use it without sharing any of the method itself.

Material fields follow the paper's level-set construction:

* smoothed Heaviside over ``n_cells`` grid cells on either side of an
  interface (Sec. 4.1, eq. "eq_heaviside");
* two-stage property law: the flowing phase from the liquid/gas level set
  ``phi`` (liquid where ``phi < 0``), then the solid from ``psi`` (solid where
  ``psi < 0``) (Sec. 4.1, eqs. "eq_ls_flow" and "eq_ls_solid");
* face densities are evaluated from level sets averaged onto faces
  (Sec. 4.2.2: the face density vector is set from level sets averaged onto faces);
* viscosity lives at cell centres (Sec. 3.1).

Layouts are C order with x fastest: ``u`` is (Nz, Ny, Nx+1), ``v`` is
(Nz, Ny+1, Nx), ``w`` is (Nz+1, Ny, Nx), cell fields are (Nz, Ny, Nx).  2D
problems use Nz = 1 and carry no ``w``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Water / air / solid material constants used by every workload (Sec. 7: water
# rho 1e3 and mu 1e-3, air rho 1.2 and mu 1.8e-5; Sec. 5: the solid's virtual
# viscosity equals the most viscous fluid's).
RHO_WATER = 1000.0
MU_WATER = 1.0e-3
RHO_AIR = 1.2
MU_AIR = 1.8e-5
MU_SOLID = 1.0e-3
N_CELLS = 1.5


@dataclasses.dataclass
class Problem:
    """One Stokes solve: grid, coefficients, right-hand side and tolerance."""

    name: str
    dim: int
    n: Tuple[int, int, int]          # (Nx, Ny, Nz); Nz = 1 in 2D
    h: Tuple[float, float, float]
    dt: float
    rho_faces: List[Optional[np.ndarray]]   # [rho_x, rho_y, rho_z or None]
    mu: np.ndarray                          # (Nz, Ny, Nx)
    rhs_u: List[Optional[np.ndarray]]       # [f_x, f_y, f_z or None]
    rhs_p: np.ndarray                       # (Nz, Ny, Nx)
    tol: float
    phi: Optional[np.ndarray] = None        # cell level sets, kept for tests
    rho_flow_faces: Optional[List[Optional[np.ndarray]]] = None
    seed: Optional[int] = None
    psi: Optional[List[np.ndarray]] = None  # cell level set of each solid (solid where < 0)
    rho_solid: Optional[List[float]] = None # density of each solid
    rho_air: float = RHO_AIR                # gas density of this problem
    heaviside_cells: float = N_CELLS        # Heaviside half-width in cells of hx

    @property
    def n_cells(self) -> int:
        nx, ny, nz = self.n
        return nx * ny * nz

    def face_shape(self, axis: int) -> Tuple[int, int, int]:
        return face_shape(self.n, axis)


def face_shape(n: Sequence[int], axis: int) -> Tuple[int, int, int]:
    """Shape (Nz, Ny, Nx) of the face array normal to ``axis`` (0=x, 1=y, 2=z)."""
    nx, ny, nz = n
    s = [nz, ny, nx]
    s[2 - axis] += 1
    return tuple(s)


def cell_shape(n: Sequence[int]) -> Tuple[int, int, int]:
    nx, ny, nz = n
    return (nz, ny, nx)


# --------------------------------------------------------------------------
# coordinates
# --------------------------------------------------------------------------
def cell_coords(n, h):
    """Cell-centre coordinates x_{ijk} = ((i+1/2)h_x, (j+1/2)h_y, (k+1/2)h_z) (Sec. 3.1)."""
    nx, ny, nz = n
    x = (np.arange(nx) + 0.5) * h[0]
    y = (np.arange(ny) + 0.5) * h[1]
    z = (np.arange(nz) + 0.5) * h[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def face_coords(n, h, axis):
    """Centres of the faces normal to ``axis``: that coordinate sits on i*h."""
    nx, ny, nz = n
    xs = [(np.arange(nx) + 0.5) * h[0], (np.arange(ny) + 0.5) * h[1], (np.arange(nz) + 0.5) * h[2]]
    xs[axis] = np.arange(n[axis] + 1) * h[axis]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return X, Y, Z


# --------------------------------------------------------------------------
# level-set material law
# --------------------------------------------------------------------------
def heaviside(phi: np.ndarray, eps: float) -> np.ndarray:
    """Smoothed Heaviside regularised over ``eps = n_cells*h`` (Sec. 4.1, eq_heaviside).

    0 below -eps, 1 above +eps, and 1/2(1 + phi/eps + sin(pi phi/eps)/pi) in between.
    """
    phi = np.asarray(phi, dtype=np.float64)
    out = 0.5 * (1.0 + phi / eps + np.sin(np.pi * phi / eps) / np.pi)
    out = np.where(phi < -eps, 0.0, out)
    out = np.where(phi > eps, 1.0, out)
    return out


def two_stage(zeta_l: float, zeta_g: float, h_flow: np.ndarray,
              solids: Sequence[Tuple[float, np.ndarray]]) -> np.ndarray:
    """Two-stage property law (Sec. 4.1, eq_ls_flow then eq_ls_solid).

    ``h_flow`` is H(phi); each solid is (zeta_s, H(psi_s)).  Solids are applied in
    turn; they never overlap in the generated layouts, so the order is immaterial.
    """
    z = zeta_l + (zeta_g - zeta_l) * h_flow
    for zeta_s, h_body in solids:
        z = zeta_s + (z - zeta_s) * h_body
    return z


def face_average(cell: np.ndarray, axis: int) -> np.ndarray:
    """Average a cell field onto the faces normal to ``axis``.

    Interior faces take the mean of the two adjacent cells; boundary faces take
    the one adjacent cell (a mirror ghost).
    """
    ax = 2 - axis
    c = np.moveaxis(cell, ax, 0)
    out = np.empty((c.shape[0] + 1,) + c.shape[1:], dtype=np.float64)
    out[1:-1] = 0.5 * (c[:-1] + c[1:])
    out[0] = c[0]
    out[-1] = c[-1]
    return np.moveaxis(out, 0, ax)


# --------------------------------------------------------------------------
# signed distance functions (Sec. 4.1 eq_signed_phi/psi; CSG for boxes)
# --------------------------------------------------------------------------
def sdf_sphere(X, Y, Z, c, r, dim):
    d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2
    if dim == 3:
        d2 = d2 + (Z - c[2]) ** 2
    return np.sqrt(d2) - r


def sdf_box(X, Y, Z, c, half, dim):
    """Exact signed distance to an axis-aligned box (negative inside)."""
    q = [np.abs(X - c[0]) - half[0], np.abs(Y - c[1]) - half[1]]
    if dim == 3:
        q.append(np.abs(Z - c[2]) - half[2])
    outside = np.sqrt(sum(np.maximum(qi, 0.0) ** 2 for qi in q))
    inside = np.minimum(np.maximum.reduce(q), 0.0)
    return outside + inside


def sdf_quarter_space(A, B, a0, b0):
    """Signed distance to {A < a0 and B < b0} (negative inside), exact in (A, B)."""
    da = A - a0
    db = B - b0
    outside = np.sqrt(np.maximum(da, 0.0) ** 2 + np.maximum(db, 0.0) ** 2)
    inside = np.minimum(np.maximum(da, db), 0.0)
    return outside + inside


def stokes_wave_second_order_coeff(H: float, d: float, lam: float) -> float:
    """Amplitude of the second harmonic of a 2nd-order Stokes wave (Sec. 7.1, eq_stokes_eta)."""
    k = 2.0 * math.pi / lam
    kd = k * d
    return (math.pi * H * H / (8.0 * lam)) * math.cosh(kd) * (2.0 + math.cosh(2.0 * kd)) / math.sinh(kd) ** 3


# --------------------------------------------------------------------------
# right-hand side
# --------------------------------------------------------------------------
def fourier_modes(rng: np.random.Generator, dim: int, n_modes: int = 8, kmax: int = 4):
    """Draw (k_m, a_m, theta_m) for a sum of random-phase cosine modes.

    k_m uniform on {-kmax..kmax}^dim without 0, a_m = 1/|k_m| rescaled so that
    sum a_m^2 / 2 = 1 (unit mean square), theta_m uniform on [0, 2 pi).
    """
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=dim)
        if np.any(k != 0):
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    a = 1.0 / np.linalg.norm(ks, axis=1)
    a = a / math.sqrt(0.5 * np.sum(a * a))
    th = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return ks, a, th


def eval_modes(modes, X, Y, Z, dim):
    ks, a, th = modes
    out = np.zeros_like(X, dtype=np.float64)
    for m in range(len(a)):
        arg = ks[m, 0] * X + ks[m, 1] * Y
        if dim == 3:
            arg = arg + ks[m, 2] * Z
        out += a[m] * np.cos(2.0 * math.pi * arg + th[m])
    return out


def fourier_rhs(rng, dim, n, h):
    """Velocity RHS: per component, an independent 8-mode Fourier sum at its face centres."""
    rhs = [None, None, None]
    modes = []
    for ax in range(dim):
        m = fourier_modes(rng, dim)
        modes.append(m)
        X, Y, Z = face_coords(n, h, ax)
        f = eval_modes(m, X, Y, Z, dim)
        # wall faces carry no unknown; store zeros there
        sl = [slice(None)] * 3
        sl[2 - ax] = 0
        f[tuple(sl)] = 0.0
        sl[2 - ax] = -1
        f[tuple(sl)] = 0.0
        rhs[ax] = f
    return rhs, modes


# --------------------------------------------------------------------------
# problem assembly from level sets
# --------------------------------------------------------------------------
def _materials(dim, n, h, phi_fn, solids, rho_air=RHO_AIR, n_cells=N_CELLS):
    """Cell mu, face rho and flow-only face rho from level-set callables.

    ``phi_fn(X, Y, Z)`` gives the liquid/gas level set; ``solids`` is a list of
    (psi_fn, rho_s).  Face values use level sets averaged from cells onto faces.
    """
    eps = n_cells * h[0]
    X, Y, Z = cell_coords(n, h)
    phi = phi_fn(X, Y, Z)
    psis = [(fn(X, Y, Z), rs) for fn, rs in solids]
    mu = two_stage(MU_WATER, MU_AIR, heaviside(phi, eps),
                   [(MU_SOLID, heaviside(ps, eps)) for ps, _ in psis])
    rho_faces = [None, None, None]
    rho_flow = [None, None, None]
    for ax in range(dim):
        phib = face_average(phi, ax)
        hf = heaviside(phib, eps)
        rho_flow[ax] = two_stage(RHO_WATER, rho_air, hf, [])
        rho_faces[ax] = two_stage(RHO_WATER, rho_air, hf,
                                  [(rs, heaviside(face_average(ps, ax), eps)) for ps, rs in psis])
    return phi, mu, rho_faces, rho_flow, psis


def make_problem(name, dim, n, h, dt, tol, phi_fn, solids, seed, rho_air=RHO_AIR,
                 rhs_rng=None, rhs_scale_by_mass=False):
    phi, mu, rho_faces, rho_flow, psis = _materials(dim, n, h, phi_fn, solids, rho_air=rho_air)
    rng = rhs_rng if rhs_rng is not None else np.random.Generator(np.random.PCG64(seed))
    rhs_u, _ = fourier_rhs(rng, dim, n, h)
    if rhs_scale_by_mass:
        for ax in range(dim):
            rhs_u[ax] = rhs_u[ax] * rho_faces[ax] / dt
    rhs_p = np.zeros(cell_shape(n))
    return Problem(name=name, dim=dim, n=tuple(n), h=tuple(h), dt=dt, rho_faces=rho_faces,
                   mu=mu, rhs_u=rhs_u, rhs_p=rhs_p, tol=tol, phi=phi,
                   rho_flow_faces=rho_flow, seed=seed, psi=[ps for ps, _ in psis],
                   rho_solid=[float(rs) for _, rs in psis], rho_air=rho_air)


def _grid(dim, cells, lengths):
    if dim == 2:
        n = (cells[0], cells[1], 1)
        h = (lengths[0] / cells[0], lengths[1] / cells[1], lengths[0] / cells[0])
    else:
        n = tuple(cells)
        h = tuple(L / c for L, c in zip(lengths, cells))
    return n, h


def config1(scale: int = 1, seed: int = 1001) -> Problem:
    """64^2 air over water, flat interface y = 0.5, solid disc r = 0.1 at the centre, rho_s = 500."""
    N = 64 // scale
    n, h = _grid(2, (N, N), (1.0, 1.0))
    phi_fn = lambda X, Y, Z: Y - 0.5
    disc = (lambda X, Y, Z: sdf_sphere(X, Y, Z, (0.5, 0.5), 0.1, 2), 500.0)
    return make_problem("config1_%dx%d" % (N, N), 2, n, h, 1e-4, 1e-10, phi_fn, [disc], seed)


def config2(scale: int = 1, seed: int = 1002) -> Problem:
    """512^2 wavy interface, three seeded discs with rho_s in [300, 1200]."""
    N = 512 // scale
    n, h = _grid(2, (N, N), (1.0, 1.0))
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(1, 5))
    ph0 = float(rng.uniform(0.0, 2.0 * math.pi))
    discs = []
    while len(discs) < 3:
        r = float(rng.uniform(0.03, 0.08))
        c = rng.uniform(0.1, 0.9, size=2)
        if all(np.hypot(*(c - c2)) > r + r2 + 0.02 for c2, r2, _ in discs):
            discs.append((c, r, float(rng.uniform(300.0, 1200.0))))
    phi_fn = lambda X, Y, Z: Y - 0.5 - 0.05 * np.sin(2.0 * math.pi * k * X + ph0)
    solids = [((lambda c, r: (lambda X, Y, Z: sdf_sphere(X, Y, Z, c, r, 2)))(c, r), rs)
              for c, r, rs in discs]
    return make_problem("config2_%dx%d" % (N, N), 2, n, h, 5e-5, 1e-8, phi_fn, solids, seed,
                        rhs_rng=rng)


def config3(scale: int = 1, seed: int = 1003) -> Problem:
    """128^3 dam-break-like water column x < 0.4, z < 0.6, one seeded sphere r = 0.12, rho_s = 700."""
    N = 128 // scale
    n, h = _grid(3, (N, N, N), (1.0, 1.0, 1.0))
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.15, 0.85, size=3)
    phi_fn = lambda X, Y, Z: sdf_quarter_space(X, Z, 0.4, 0.6)
    sph = (lambda X, Y, Z: sdf_sphere(X, Y, Z, c, 0.12, 3), 700.0)
    return make_problem("config3_%d^3" % N, 3, n, h, 2e-5, 1e-8, phi_fn, [sph], seed, rhs_rng=rng)


def config4(scale: int = 1, seed: int = 1004) -> Problem:
    """1024x96x96 wave-tank slab: 2nd-order Stokes wave free surface and a floating box."""
    nx, ny, nz = 1024 // scale, 96 // scale, 96 // scale
    n, h = _grid(3, (nx, ny, nz), (32.0 / 3.0, 1.0, 1.0))
    rng = np.random.Generator(np.random.PCG64(seed))
    ph0 = float(rng.uniform(0.0, 2.0 * math.pi))
    Hw, d, lam = 0.04, 0.5, 1.5
    k = 2.0 * math.pi / lam
    a2 = stokes_wave_second_order_coeff(Hw, d, lam)

    def phi_fn(X, Y, Z):
        eta = 0.5 + 0.5 * Hw * np.cos(k * X + ph0) + a2 * np.cos(2.0 * k * X + 2.0 * ph0)
        deta = -0.5 * Hw * k * np.sin(k * X + ph0) - 2.0 * k * a2 * np.sin(2.0 * k * X + 2.0 * ph0)
        return (Z - eta) / np.sqrt(1.0 + deta * deta)

    box = (lambda X, Y, Z: sdf_box(X, Y, Z, (16.0 / 3.0, 0.5, 0.5), (0.15, 0.15, 0.1), 3), 500.0)
    return make_problem("config4_%dx%dx%d" % (nx, ny, nz), 3, n, h, 1e-5, 1e-8, phi_fn, [box],
                        seed, rhs_rng=rng)


def config4_2d(nx: int = 512, ny: int = 48, seed: int = 1004) -> Problem:
    """The wave tank of config 4 in its vertical x-z plane (2D: x along the tank, y up):
    the same free surface and a floating box 0.3 x 0.2, rho_s = 500, on
    [0, 32/3] x [0, 1] with isotropic spacing (nx = 32/3 ny)."""
    n, h = _grid(2, (nx, ny), (32.0 / 3.0, 1.0))
    rng = np.random.Generator(np.random.PCG64(seed))
    ph0 = float(rng.uniform(0.0, 2.0 * math.pi))
    Hw, d, lam = 0.04, 0.5, 1.5
    k = 2.0 * math.pi / lam
    a2 = stokes_wave_second_order_coeff(Hw, d, lam)

    def phi_fn(X, Y, Z):
        eta = 0.5 + 0.5 * Hw * np.cos(k * X + ph0) + a2 * np.cos(2.0 * k * X + 2.0 * ph0)
        deta = -0.5 * Hw * k * np.sin(k * X + ph0) - 2.0 * k * a2 * np.sin(2.0 * k * X + 2.0 * ph0)
        return (Y - eta) / np.sqrt(1.0 + deta * deta)

    box = (lambda X, Y, Z: sdf_box(X, Y, Z, (16.0 / 3.0, 0.5), (0.15, 0.1), 2), 500.0)
    return make_problem("config4_2d_%dx%d" % (nx, ny), 2, n, h, 1e-5, 1e-8, phi_fn, [box], seed, rhs_rng=rng)


def config5(scale: int = 1, seed: int = 900000, n_cells: Optional[int] = None,
            dt: Optional[float] = None) -> Problem:
    """256^3 random interface surface with 0-4 seeded spheres/boxes, density ratio exactly 1000.

    Training instances use 128^3 (``scale=2``) with dt = 2e-5; the headline instance
    is seed 900000 at 256^3 with dt = 1e-5.
    """
    N = n_cells if n_cells is not None else 256 // scale
    n, h = _grid(3, (N, N, N), (1.0, 1.0, 1.0))
    if dt is None:
        dt = 1e-5 if N >= 256 else 2e-5
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = []
    for _ in range(3):
        kk = rng.integers(-3, 4, size=2)
        while not np.any(kk != 0):
            kk = rng.integers(-3, 4, size=2)
        modes.append((kk.astype(np.float64), float(rng.uniform(0.005, 0.05 / 3.0)),
                      float(rng.uniform(0.0, 2.0 * math.pi))))

    def phi_fn(X, Y, Z):
        eta = 0.5 * np.ones_like(X)
        ex = np.zeros_like(X)
        ey = np.zeros_like(X)
        for kk, A, th in modes:
            arg = 2.0 * math.pi * (kk[0] * X + kk[1] * Y) + th
            eta = eta + A * np.cos(arg)
            ex = ex - A * 2.0 * math.pi * kk[0] * np.sin(arg)
            ey = ey - A * 2.0 * math.pi * kk[1] * np.sin(arg)
        return (Z - eta) / np.sqrt(1.0 + ex * ex + ey * ey)

    n_solids = int(rng.integers(0, 5))
    placed = []
    tries = 0
    while len(placed) < n_solids and tries < 1000:
        tries += 1
        kind = "sphere" if rng.uniform() < 0.5 else "box"
        if kind == "sphere":
            size = np.full(3, float(rng.uniform(0.05, 0.15)))
        else:
            size = rng.uniform(0.05, 0.15, size=3)
        c = rng.uniform(0.2, 0.8, size=3)
        rb = float(np.linalg.norm(size)) if kind == "box" else float(size[0])
        if all(np.linalg.norm(c - c2) > rb + rb2 + 0.02 for _, c2, _, rb2, _ in placed):
            placed.append((kind, c, size, rb, float(rng.uniform(300.0, 1200.0))))
    solids = []
    for kind, c, size, _, rs in placed:
        if kind == "sphere":
            fn = (lambda c, r: (lambda X, Y, Z: sdf_sphere(X, Y, Z, c, r, 3)))(c, float(size[0]))
        else:
            fn = (lambda c, s: (lambda X, Y, Z: sdf_box(X, Y, Z, c, s, 3)))(c, size)
        solids.append((fn, rs))
    p = make_problem("config5_%d^3" % N, 3, n, h, dt, 1e-8, phi_fn, solids, seed,
                     rho_air=1.0, rhs_rng=rng)
    p.solids = placed
    return p


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def config(num: int, **kw) -> Problem:
    return CONFIGS[num](**kw)


def random_vector(problem_or_n, dim, seed):
    """Seeded random (u, v, w, p) in the API layout; wall-normal faces are zero."""
    n = problem_or_n.n if isinstance(problem_or_n, Problem) else problem_or_n
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = []
    for ax in range(3):
        if ax < dim:
            a = rng.standard_normal(face_shape(n, ax))
            sl = [slice(None)] * 3
            sl[2 - ax] = 0
            a[tuple(sl)] = 0.0
            sl[2 - ax] = -1
            a[tuple(sl)] = 0.0
            xs.append(a)
        else:
            xs.append(None)
    p = rng.standard_normal(cell_shape(n))
    return xs, p


def stream_velocity(n, h, dim, seed, n_modes=4, margin=0):
    """Seeded face velocities with zero discrete divergence on the MAC grid and zero
    wall-normal entries: the discrete curl of smooth random stream functions on the
    grid nodes / edges (a few sine modes each), optionally vanishing within
    `margin` cells of every wall; normalised to max |u| = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = n[0], n[1], (n[2] if dim == 3 else 1)
    u = [np.zeros(face_shape((nx, ny, nz), c)) for c in range(dim)]
    planes = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
    for a, b in planes:
        shape = [nz, ny, nx]
        shape[2 - a] += 1
        shape[2 - b] += 1
        coords = []
        for ax in range(3):
            m = shape[2 - ax]
            if ax in (a, b):
                coords.append(np.arange(m) / (m - 1))          # node positions in [0, 1]
            else:
                coords.append((np.arange(m) + 0.5) / m)       # cell positions
        psi = np.zeros(shape)                                  # (z, y, x)
        for _ in range(n_modes):
            kx, ky, kz = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            amp = rng.standard_normal()
            fx = np.sin(np.pi * kx * coords[0])
            fy = np.sin(np.pi * ky * coords[1])
            fz = np.cos(np.pi * kz * coords[2] + ph) if dim == 3 else np.ones(1)
            psi += amp * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
        for ax in (a, b):
            m = psi.shape[2 - ax]
            idx = np.arange(m)
            keep = ((idx > margin) & (idx < m - 1 - margin)).astype(float)
            psi *= np.expand_dims(keep, [k for k in range(3) if k != 2 - ax])
        u[a] += np.diff(psi, axis=2 - b) / h[b]
        u[b] -= np.diff(psi, axis=2 - a) / h[a]
    top = max(float(np.abs(x).max()) for x in u)
    return [x / top for x in u]
