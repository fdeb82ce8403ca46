"""ctypes binding of libstokes.so: the C-ABI of include/stokes.h, same names.

Device arrays are passed as torch tensors (float64, contiguous, on the GPU);
the binding only extracts their pointers and the current HIP stream.  Every
step of the solve runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libstokes.so")
_lib = None

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "BREAKDOWN", -1: "EINVAL", -2: "ESHAPE",
                -3: "ENOMEM", -4: "EHIP", -5: "ENAN"}


class StokesError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class StokesGrid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double * 3), ("periodic", C.c_int * 3)]


class StokesFluids(C.Structure):
    _fields_ = [("rho_liquid", C.c_double), ("rho_gas", C.c_double), ("mu_liquid", C.c_double),
                ("mu_gas", C.c_double), ("n_cells", C.c_double)]


MAX_SOLIDS = 8


class StokesWave(C.Structure):
    _fields_ = [("height", C.c_double), ("depth", C.c_double), ("wavelength", C.c_double),
                ("omega", C.c_double), ("gravity", C.c_double), ("n_cells", C.c_double)]


class StokesBody(C.Structure):
    _fields_ = [("x_com", C.c_double * 3), ("u_r", C.c_double * 3), ("w_r", C.c_double * 3)]

    def as_dict(self):
        return {"x_com": list(self.x_com), "u_r": list(self.u_r), "w_r": list(self.w_r)}


class StokesOptions(C.Structure):
    _fields_ = [("precision", C.c_int), ("visc_scale", C.c_double), ("cont_scale", C.c_double),
                ("restart", C.c_int), ("max_iters", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("vel_cycles", C.c_int), ("p_cycles", C.c_int), ("coarse_sweeps", C.c_int),
                ("vel_levels", C.c_int), ("vel_sweeps", C.c_int), ("p_prolong", C.c_int),
                ("vel_smoother", C.c_int), ("orth", C.c_int), ("matvec_z", C.c_int),
                ("p_gamma", C.c_int), ("p_small", C.c_int),
                ("p_wdepth", C.c_int), ("p_cycles_next", C.c_int), ("p_nu_second", C.c_int),
                ("open_top", C.c_int), ("p_omega", C.c_double)]


class StokesStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("vcycles", C.c_int), ("levels", C.c_int),
                ("rel_res_est", C.c_double), ("rel_res_true", C.c_double),
                ("rel_res_plain", C.c_double), ("rel_res_mom", C.c_double),
                ("rel_res_cont", C.c_double), ("sigma", C.c_double), ("g_mean", C.c_double),
                ("ms_total", C.c_double), ("fell_back", C.c_int),
                ("small_level", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libstokes.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libstokes.so is not built; run python paper_1901_07892_amd/build.py")
    L = C.CDLL(_LIB_PATH)
    dp = C.c_void_p
    L.stokes_default_options.argtypes = [C.POINTER(StokesOptions)]
    L.stokes_default_options.restype = None
    L.stokes_workspace_size.argtypes = [C.POINTER(StokesGrid), C.POINTER(StokesOptions)]
    L.stokes_workspace_size.restype = C.c_size_t
    L.stokes_setup.argtypes = [C.c_void_p * 3, dp, C.c_double, C.POINTER(StokesGrid),
                               C.POINTER(StokesOptions), dp, C.c_size_t, dp, C.POINTER(C.c_void_p)]
    L.stokes_setup.restype = C.c_int
    L.stokes_apply.argtypes = [C.c_void_p, C.c_void_p * 3, dp, C.c_void_p * 3, dp]
    L.stokes_apply.restype = C.c_int
    L.stokes_solve.argtypes = [C.c_void_p, C.c_void_p * 3, dp, C.c_double, C.c_void_p * 3, dp,
                               C.POINTER(StokesStats)]
    L.stokes_solve.restype = C.c_int
    L.stokes_destroy.argtypes = [C.c_void_p]
    L.stokes_destroy.restype = None
    L.stokes_last_error.argtypes = [C.c_void_p]
    L.stokes_last_error.restype = C.c_char_p
    L.stokes_profile_kernel.argtypes = [C.c_void_p, C.c_int]
    L.stokes_profile_kernel.restype = C.c_int
    L.stokes_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                                      C.POINTER(C.c_double)]
    L.stokes_profile_read.restype = C.c_int
    L.stokes_stream_copy.argtypes = [dp, dp, C.c_longlong, dp]
    L.stokes_stream_copy.restype = C.c_int
    L.stokes_coefficients.argtypes = [C.POINTER(StokesGrid), C.POINTER(StokesFluids), dp, C.c_int,
                                      C.POINTER(C.c_void_p), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.c_void_p * 3, dp, C.POINTER(C.c_void_p * 3), dp]
    L.stokes_coefficients.restype = C.c_int
    L.stokes_explicit_rhs.argtypes = [C.POINTER(StokesGrid), C.c_void_p * 3, dp, C.c_double, C.c_double,
                                      C.c_void_p * 3, C.POINTER(C.c_void_p * 3), C.POINTER(C.c_double * 3),
                                      C.c_void_p * 3, dp]
    L.stokes_explicit_rhs.restype = C.c_int
    L.stokes_rigid_workspace_size.argtypes = [C.c_int, C.c_longlong]
    L.stokes_rigid_workspace_size.restype = C.c_size_t
    L.stokes_rigid_projection.argtypes = [C.POINTER(StokesGrid), C.c_void_p * 3, C.c_longlong, dp, C.c_double,
                                          C.c_int, C.POINTER(StokesBody), dp, C.c_size_t, dp]
    L.stokes_rigid_projection.restype = C.c_int
    L.stokes_rigid_projection_noalloc.argtypes = [C.POINTER(StokesGrid), C.c_void_p * 3, C.c_longlong, dp,
                                                  C.c_double, C.c_int, C.POINTER(StokesBody), dp]
    L.stokes_rigid_projection_noalloc.restype = C.c_int
    L.stokes_unet_param_count.argtypes = []
    L.stokes_unet_param_count.restype = C.c_longlong
    L.stokes_unet_forward_flops.argtypes = [C.c_int]
    L.stokes_unet_forward_flops.restype = C.c_double
    L.stokes_unet_workspace_size.argtypes = [C.c_int]
    L.stokes_unet_workspace_size.restype = C.c_size_t
    L.stokes_unet_create.argtypes = [C.c_int, dp, C.c_size_t, dp, C.POINTER(C.c_void_p)]
    L.stokes_unet_create.restype = C.c_int
    L.stokes_unet_init.argtypes = [C.c_void_p, C.c_ulonglong]
    L.stokes_unet_init.restype = C.c_int
    fp = C.POINTER(C.c_float)
    L.stokes_unet_get_params.argtypes = [C.c_void_p, fp, C.c_longlong]
    L.stokes_unet_get_params.restype = C.c_int
    L.stokes_unet_set_params.argtypes = [C.c_void_p, fp, C.c_longlong]
    L.stokes_unet_set_params.restype = C.c_int
    L.stokes_unet_get_grads.argtypes = [C.c_void_p, fp, C.c_longlong]
    L.stokes_unet_get_grads.restype = C.c_int
    L.stokes_unet_forward.argtypes = [C.c_void_p, dp, dp, dp, dp]
    L.stokes_unet_forward.restype = C.c_int
    L.stokes_unet_train_step.argtypes = [C.c_void_p, dp, dp, dp, dp, C.c_float, fp]
    L.stokes_unet_train_step.restype = C.c_int
    L.stokes_unet_size.argtypes = [C.c_void_p]
    L.stokes_unet_size.restype = C.c_int
    L.stokes_unet_destroy.argtypes = [C.c_void_p]
    L.stokes_unet_destroy.restype = None
    L.stokes_attach_learned.argtypes = [C.c_void_p, C.c_void_p, C.c_double]
    L.stokes_attach_learned.restype = C.c_int
    L.stokes_learned_tuple.argtypes = [C.c_void_p, C.c_void_p * 3, dp, C.c_int, C.c_int, dp, dp, dp, dp]
    L.stokes_learned_tuple.restype = C.c_int
    L.stokes_learned_study.argtypes = [C.c_void_p, C.c_void_p * 3, dp, C.c_int, C.c_int, C.POINTER(C.c_double)]
    L.stokes_learned_study.restype = C.c_int
    L.stokes_wave_inflow.argtypes = [C.POINTER(StokesGrid), C.POINTER(StokesWave), C.c_double, dp, dp, dp]
    L.stokes_wave_inflow.restype = C.c_int
    L.stokes_inflow_lift.argtypes = [C.c_void_p, dp, dp, C.c_void_p * 3, dp]
    L.stokes_inflow_lift.restype = C.c_int
    L.stokes_density_workspace_size.argtypes = [C.POINTER(StokesGrid)]
    L.stokes_density_workspace_size.restype = C.c_size_t
    L.stokes_density_rk3.argtypes = [C.POINTER(StokesGrid), C.c_double, C.c_void_p * 3, C.c_void_p * 9,
                                     C.c_void_p * 3, dp, C.c_size_t, dp]
    L.stokes_density_rk3.restype = C.c_int
    L.stokes_pressure_op.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, dp]
    L.stokes_pressure_op.restype = C.c_int
    _lib = L
    return L


# ---------------------------------------------------------------- marshalling helpers
def _ptr(t, need: Optional[int] = None) -> Optional[int]:
    """Device address of a tensor (or an int address as it is).  With ``need``, a
    tensor must hold at least that many values: the kernels index the caller's
    arrays from the grid alone, so a shorter one would be read or written past
    its end."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        import torch
        if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("arrays must be contiguous float64 CUDA/HIP tensors")
        if need is not None and t.numel() < need:
            raise ValueError("array of %d values where the grid needs %d" % (t.numel(), need))
        return t.data_ptr()
    return int(t)


def _ptr3(ts: Sequence, needs: Optional[Sequence[int]] = None) -> "C.Array":
    arr = (C.c_void_p * 3)()
    for a, t in enumerate(list(ts)[:3]):
        arr[a] = _ptr(t, needs[a] if needs is not None and a < len(needs) else None)
    return arr


def _counts(grid) -> Tuple[List[int], int]:
    """Values in the caller's arrays for a grid (layouts of include/stokes.h):
    the face array of each velocity component and the cell array."""
    d = grid.dim
    n = [int(grid.n[a]) if a < d else 1 for a in range(3)]
    faces = [(n[0] + (c == 0)) * (n[1] + (c == 1)) * (n[2] + (c == 2)) for c in range(d)]
    return faces, n[0] * n[1] * n[2]


def _inflow_counts(grid) -> Tuple[int, int]:
    """Values in the inflow arrays on x = 0: u_n (Nv x N_lateral) and u_t
    ((Nv + 1) x N_lateral), Nv the cells along the vertical axis."""
    nv = int(grid.n[grid.dim - 1])
    nl = int(grid.n[1]) if grid.dim == 3 else 1
    return nv * nl, (nv + 1) * nl


# array sizes of each live context's grid, for the checks of the calls that take a context
_CTX_COUNTS: Dict[int, Tuple[List[int], int]] = {}
_CTX_INFLOW: Dict[int, Tuple[int, int]] = {}


def _ctx_counts(ctx) -> Tuple[Optional[List[int]], Optional[int]]:
    return _CTX_COUNTS.get(ctx, (None, None))


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def make_grid(dim: int, n: Sequence[int], h: Sequence[float], periodic: Sequence[int] = (0, 0, 0)) -> StokesGrid:
    g = StokesGrid()
    g.dim = dim
    for a in range(3):
        g.n[a] = int(n[a]) if a < len(n) else 1
        g.h[a] = float(h[a]) if a < len(h) else float(h[0])
        g.periodic[a] = int(bool(periodic[a])) if a < len(periodic) else 0
    return g


# ---------------------------------------------------------------- the C-ABI, same names
def stokes_default_options() -> StokesOptions:
    o = StokesOptions()
    load_library().stokes_default_options(C.byref(o))
    return o


def stokes_workspace_size(grid: StokesGrid, opts: Optional[StokesOptions] = None) -> int:
    return int(load_library().stokes_workspace_size(C.byref(grid), C.byref(opts) if opts else None))


def stokes_setup(rho_face, mu_cell, dt, grid, opts, workspace, ws_bytes, stream=None):
    """Returns an opaque context handle (int); raises StokesError on failure."""
    L = load_library()
    ctx = C.c_void_p()
    faces, cells = _counts(grid) if grid is not None and grid.dim in (2, 3) else (None, None)
    st = L.stokes_setup(_ptr3(list(rho_face) + [None] * 3, faces), _ptr(mu_cell, cells), float(dt), C.byref(grid),
                        C.byref(opts) if opts is not None else None, _ptr(workspace), int(ws_bytes),
                        _stream(stream), C.byref(ctx))
    if st != 0:
        raise StokesError(st, L.stokes_last_error(None).decode())
    _CTX_COUNTS[ctx.value] = (faces, cells)
    _CTX_INFLOW[ctx.value] = _inflow_counts(grid)
    return ctx.value


def stokes_apply(ctx, x_u, x_p, y_u, y_p) -> int:
    L = load_library()
    faces, cells = _ctx_counts(ctx)
    st = L.stokes_apply(ctx, _ptr3(list(x_u) + [None] * 3, faces), _ptr(x_p, cells),
                        _ptr3(list(y_u) + [None] * 3, faces), _ptr(y_p, cells))
    if st < 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())
    return st


def stokes_solve(ctx, rhs_u, rhs_p, tol, x_u, x_p):
    """Returns (status, StokesStats); raises StokesError on negative status."""
    L = load_library()
    stats = StokesStats()
    faces, cells = _ctx_counts(ctx)
    st = L.stokes_solve(ctx, _ptr3(list(rhs_u) + [None] * 3, faces), _ptr(rhs_p, cells), float(tol),
                        _ptr3(list(x_u) + [None] * 3, faces), _ptr(x_p, cells), C.byref(stats))
    if st < 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())
    return st, stats


def stokes_destroy(ctx) -> None:
    if ctx:
        _CTX_COUNTS.pop(ctx, None)
        _CTX_INFLOW.pop(ctx, None)
        load_library().stokes_destroy(ctx)


def stokes_last_error(ctx=None) -> str:
    return load_library().stokes_last_error(ctx).decode()


PROF_MATVEC, PROF_P_SWEEP, PROF_MULTIDOT, PROF_MAXPY = 0, 1, 2, 3


def stokes_profile_kernel(ctx, kernel: int) -> None:
    L = load_library()
    st = L.stokes_profile_kernel(ctx, int(kernel))
    if st < 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())


def stokes_profile_read(ctx):
    """Returns (ms_total, launches, algorithmic_bytes) and resets them."""
    ms, n, b = C.c_double(), C.c_longlong(), C.c_double()
    load_library().stokes_profile_read(ctx, C.byref(ms), C.byref(n), C.byref(b))
    return ms.value, n.value, b.value


def make_wave(height, depth, wavelength, omega, gravity=9.81, n_cells=1.5) -> StokesWave:
    w = StokesWave()
    w.height, w.depth, w.wavelength, w.omega, w.gravity, w.n_cells = (
        float(height), float(depth), float(wavelength), float(omega), float(gravity), float(n_cells))
    return w


def stokes_wave_inflow(grid, wave, t, u_n, u_t, stream=None) -> None:
    """Second-order Stokes wave inflow data on x = 0 into the device tensors u_n, u_t."""
    n_n, n_t = _inflow_counts(grid) if grid.dim in (2, 3) else (None, None)
    st = load_library().stokes_wave_inflow(C.byref(grid), C.byref(wave), float(t), _ptr(u_n, n_n),
                                          _ptr(u_t, n_t), _stream(stream))
    if st != 0:
        raise StokesError(st, "stokes_wave_inflow failed")


def stokes_inflow_lift(ctx, u_n, u_t, rhs_u, rhs_p) -> None:
    """Subtract the inflow data's contribution from (rhs_u, rhs_p), in place."""
    L = load_library()
    faces, cells = _ctx_counts(ctx)
    n_n, n_t = _CTX_INFLOW.get(ctx, (None, None))
    st = L.stokes_inflow_lift(ctx, _ptr(u_n, n_n), _ptr(u_t, n_t), _ptr3(list(rhs_u) + [None] * 3, faces),
                              _ptr(rhs_p, cells))
    if st != 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())


def stokes_density_workspace_size(grid: StokesGrid) -> int:
    return int(load_library().stokes_density_workspace_size(C.byref(grid)))


def stokes_density_rk3(grid, dt, rho_n, u_stages, rho_out, workspace, stream=None) -> None:
    """SSP-RK3 face-density transport: ``u_stages`` is a list of three velocity
    lists (one per stage); all arrays are device float64 tensors."""
    L = load_library()
    faces = _counts(grid)[0] if grid.dim in (2, 3) else None
    us = (C.c_void_p * 9)()
    for st in range(3):
        for c, t in enumerate(list(u_stages[st])[:3]):
            us[3 * st + c] = _ptr(t, faces[c] if faces is not None and c < len(faces) else None)
    st = L.stokes_density_rk3(C.byref(grid), float(dt), _ptr3(list(rho_n) + [None] * 3, faces), us,
                              _ptr3(list(rho_out) + [None] * 3, faces),
                              workspace.data_ptr() if workspace is not None else None,
                              workspace.numel() * workspace.element_size() if workspace is not None else 0,
                              _stream(stream))
    if st != 0:
        raise StokesError(st, "stokes_density_rk3 failed")


POP_SWEEP, POP_SWEEP_FLAT, POP_RESTRICT, POP_RESTRICT_FLAT = 0, 1, 2, 3


def stokes_pressure_op(ctx, op: int, e_in, r, ec, out) -> None:
    """One pressure-multigrid kernel of the finest level on caller cell arrays
    (device float64 tensors; ``e_in`` None = from zero, ``ec`` None = no coarse
    correction).  Blocks until done."""
    L = load_library()
    st = L.stokes_pressure_op(ctx, int(op), _ptr(e_in), _ptr(r), _ptr(ec), _ptr(out))
    if st != 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())


def stokes_stream_copy(src, dst, stream=None) -> None:
    """dst[:] = src[:] (float64 device tensors of equal size) with the library's
    streaming copy kernel, on the current (or given) stream."""
    if src.dtype != dst.dtype or src.numel() != dst.numel() or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous tensors of one size and dtype")
    st = load_library().stokes_stream_copy(src.data_ptr(), dst.data_ptr(), src.numel(), _stream(stream))
    if st < 0:
        raise StokesError(st, "stokes_stream_copy failed")


def make_fluids(rho_liquid, rho_gas, mu_liquid, mu_gas, n_cells) -> StokesFluids:
    f = StokesFluids()
    f.rho_liquid, f.rho_gas, f.mu_liquid, f.mu_gas, f.n_cells = (
        float(rho_liquid), float(rho_gas), float(mu_liquid), float(mu_gas), float(n_cells))
    return f


def stokes_coefficients(grid, fluids, phi, psi, rho_solid, mu_solid, rho_face, mu_cell,
                        rho_flow_face=None, stream=None) -> None:
    """Face densities and cell viscosity from level sets on the device.

    ``psi`` is a list of solid level sets (device tensors, cell layout) with
    ``rho_solid`` / ``mu_solid`` lists of their properties; ``rho_face`` (and
    ``rho_flow_face`` when given) are lists of 2 or 3 face-layout output tensors.
    """
    L = load_library()
    ns = len(psi)
    if len(rho_solid) != ns or len(mu_solid) != ns:
        raise ValueError("psi, rho_solid and mu_solid must have one entry per solid")
    faces, cells = _counts(grid) if grid.dim in (2, 3) else (None, None)
    cap = max(ns, 1)
    ps = (C.c_void_p * cap)(*[_ptr(t, cells) for t in psi])
    rs = (C.c_double * cap)(*[float(v) for v in rho_solid])
    ms = (C.c_double * cap)(*[float(v) for v in mu_solid])
    flow = C.byref(_ptr3(list(rho_flow_face) + [None] * 3, faces)) if rho_flow_face is not None else None
    st = L.stokes_coefficients(C.byref(grid), C.byref(fluids), _ptr(phi, cells), ns,
                               C.cast(ps, C.POINTER(C.c_void_p)) if ns else None,
                               C.cast(rs, C.POINTER(C.c_double)) if ns else None,
                               C.cast(ms, C.POINTER(C.c_double)) if ns else None,
                               _ptr3(list(rho_face) + [None] * 3, faces), _ptr(mu_cell, cells), flow,
                               _stream(stream))
    if st < 0:
        raise StokesError(st, "stokes_coefficients failed")


def stokes_explicit_rhs(grid, rho_face, mu_cell, dt, theta, u_n, f, rho_force=None, gravity=None,
                        stream=None) -> None:
    """f = (rho/dt) u^n + (1 - theta) L_mu u^n (+ rho_force g) on the device."""
    L = load_library()
    faces, cells = _counts(grid) if grid.dim in (2, 3) else (None, None)
    pad = lambda ts: list(ts) + [None] * 3
    rf = C.byref(_ptr3(pad(rho_force), faces)) if rho_force is not None else None
    gv = C.byref((C.c_double * 3)(*[float(x) for x in (list(gravity) + [0.0] * 3)[:3]])) if gravity is not None else None
    st = L.stokes_explicit_rhs(C.byref(grid), _ptr3(pad(rho_face), faces), _ptr(mu_cell, cells), float(dt),
                               float(theta), _ptr3(pad(u_n), faces), rf, gv, _ptr3(pad(f), faces), _stream(stream))
    if st < 0:
        raise StokesError(st, "stokes_explicit_rhs failed")


def make_body(x_com, u_r=(0.0, 0.0, 0.0), w_r=(0.0, 0.0, 0.0)) -> StokesBody:
    b = StokesBody()
    for d in range(3):
        b.x_com[d] = float(x_com[d]) if d < len(x_com) else 0.0
        b.u_r[d] = float(u_r[d]) if d < len(u_r) else 0.0
        b.w_r[d] = float(w_r[d]) if d < len(w_r) else 0.0
    return b


def stokes_rigid_workspace_size(dim: int, n_markers: int) -> int:
    return int(load_library().stokes_rigid_workspace_size(int(dim), int(n_markers)))


def stokes_rigid_projection(grid, u, X, dV, free_body, body, workspace, stream=None) -> StokesBody:
    """Correct the face velocities ``u`` (list of device tensors, in place) for the
    rigid body whose markers are the rows of ``X`` (device tensor, n x dim);
    returns ``body`` with the free-body velocities filled in."""
    L = load_library()
    n = int(X.shape[0]) if X is not None else 0
    faces = _counts(grid)[0] if grid.dim in (2, 3) else None
    st = L.stokes_rigid_projection(C.byref(grid), _ptr3(list(u) + [None] * 3, faces), n,
                                   _ptr(X, n * grid.dim) if n else None, float(dV), int(bool(free_body)),
                                   C.byref(body),
                                   workspace.data_ptr() if workspace is not None else None,
                                   workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                   _stream(stream))
    if st < 0:
        raise StokesError(st, "stokes_rigid_projection failed")
    return body


RIGID_NOALLOC_MAX_MARKERS = 524288


def stokes_rigid_projection_noalloc(grid, u, X, dV, free_body, body, stream=None) -> StokesBody:
    """stokes_rigid_projection without a workspace (the library's fixed scratch)."""
    L = load_library()
    n = int(X.shape[0]) if X is not None else 0
    faces = _counts(grid)[0] if grid.dim in (2, 3) else None
    st = L.stokes_rigid_projection_noalloc(C.byref(grid), _ptr3(list(u) + [None] * 3, faces), n,
                                           _ptr(X, n * grid.dim) if n else None, float(dV), int(bool(free_body)),
                                           C.byref(body), _stream(stream))
    if st < 0:
        raise StokesError(st, "stokes_rigid_projection_noalloc failed: " + L.stokes_last_error(None).decode())
    return body


# ---------------------------------------------------------------- convenience wrapper
class StokesSolver:
    """Owns a workspace tensor and a context for one coefficient set.

    ``rho_face`` (list of 2 or 3 tensors) and ``mu_cell`` are device float64
    tensors in the caller layout of include/stokes.h.
    """

    def __init__(self, dim, n, h, rho_face, mu_cell, dt, opts: Optional[StokesOptions] = None,
                 stream=None, periodic=(0, 0, 0), **overrides):
        import torch
        load_library()
        self.grid = make_grid(dim, n, h, periodic)
        self.opts = opts if opts is not None else stokes_default_options()
        for k, v in overrides.items():
            setattr(self.opts, k, v)
        self.ws_bytes = stokes_workspace_size(self.grid, self.opts)
        if self.ws_bytes == 0:
            raise StokesError(-1, "invalid grid or options")
        dev = mu_cell.device
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream
        self.ctx = stokes_setup(rho_face, mu_cell, dt, self.grid, self.opts, self.workspace.data_ptr(),
                                self.ws_bytes, stream)
        self.dim = dim

    def apply(self, x_u, x_p, y_u, y_p):
        return stokes_apply(self.ctx, x_u, x_p, y_u, y_p)

    def solve(self, rhs_u, rhs_p, tol, x_u, x_p):
        return stokes_solve(self.ctx, rhs_u, rhs_p, tol, x_u, x_p)

    def pressure_op(self, op, e_in, r, ec, out):
        return stokes_pressure_op(self.ctx, op, e_in, r, ec, out)

    def close(self):
        if self.ctx:
            stokes_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned form (U-Net)
def _fptr(t, need: Optional[int] = None):
    if hasattr(t, "data_ptr"):
        import torch
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("U-Net arrays must be contiguous float32 device tensors")
        if need is not None and t.numel() < need:
            raise ValueError("U-Net array of %d values where the grid needs %d" % (t.numel(), need))
        return t.data_ptr()
    return int(t)


def stokes_unet_param_count() -> int:
    return int(load_library().stokes_unet_param_count())


def stokes_unet_forward_flops(n: int) -> float:
    return float(load_library().stokes_unet_forward_flops(int(n)))


def stokes_unet_workspace_size(n: int) -> int:
    return int(load_library().stokes_unet_workspace_size(int(n)))


def _chk(st, what):
    if st != 0:
        raise StokesError(st, what)


class UNet:
    """Owns a workspace tensor and a stokes_unet on the current device/stream."""

    def __init__(self, n: int, seed: int = 0, stream=None):
        import torch
        L = load_library()
        self.n = n
        self.ws_bytes = stokes_unet_workspace_size(n)
        if self.ws_bytes == 0:
            raise StokesError(-1, "U-Net grid must be a multiple of 8, >= 8")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        _chk(L.stokes_unet_create(n, self.workspace.data_ptr(), self.ws_bytes, _stream(stream), C.byref(h)),
             "stokes_unet_create")
        self.handle = h.value
        _chk(L.stokes_unet_init(self.handle, int(seed)), "stokes_unet_init")
        self.count = stokes_unet_param_count()

    def get_params(self):
        import numpy as np
        a = np.zeros(self.count, dtype=np.float32)
        _chk(load_library().stokes_unet_get_params(self.handle, a.ctypes.data_as(C.POINTER(C.c_float)), self.count),
             "get_params")
        return a

    def set_params(self, a):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.size != self.count:
            raise ValueError("%d parameters given, the network has %d" % (a.size, self.count))
        _chk(load_library().stokes_unet_set_params(self.handle, a.ctypes.data_as(C.POINTER(C.c_float)), self.count),
             "set_params")

    def get_grads(self):
        import numpy as np
        a = np.zeros(self.count, dtype=np.float32)
        _chk(load_library().stokes_unet_get_grads(self.handle, a.ctypes.data_as(C.POINTER(C.c_float)), self.count),
             "get_grads")
        return a

    def forward(self, f0, f1, f2, out):
        v = self.n ** 3
        _chk(load_library().stokes_unet_forward(self.handle, _fptr(f0, v), _fptr(f1, v), _fptr(f2, v),
                                                _fptr(out, v)), "stokes_unet_forward")

    def train_step(self, f0, f1, f2, target, lr):
        loss = C.c_float()
        v = self.n ** 3
        _chk(load_library().stokes_unet_train_step(self.handle, _fptr(f0, v), _fptr(f1, v), _fptr(f2, v),
                                                   _fptr(target, v), float(lr), C.byref(loss)),
             "stokes_unet_train_step")
        return loss.value

    def close(self):
        if getattr(self, "handle", None):
            load_library().stokes_unet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stokes_attach_learned(ctx, net, stall_ratio: float = 0.9) -> None:
    L = load_library()
    st = L.stokes_attach_learned(ctx, net.handle if net is not None else None, float(stall_ratio))
    if st != 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())


def stokes_learned_tuple(ctx, rhs_u, rhs_p, n, cycles, f0, f1, s_c, phi_c) -> None:
    L = load_library()
    st = L.stokes_learned_tuple(ctx, _ptr3(list(rhs_u) + [None] * 3), _ptr(rhs_p), int(n), int(cycles),
                                _fptr(f0), _fptr(f1), _fptr(s_c), _fptr(phi_c))
    if st != 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())


STUDY_ROWS = 6


def stokes_learned_study(ctx, rhs_u, rhs_p, ref_cycles: int, max_cycles: int):
    """Relative pressure residuals after 0..max_cycles cycles of the first
    preconditioner application from each start (rows: zero, the network's
    guess, the ideal guess on levels 1..STUDY_ROWS-2); a numpy array."""
    import numpy as np
    L = load_library()
    out = np.full((STUDY_ROWS, int(max_cycles) + 1), np.nan)
    st = L.stokes_learned_study(ctx, _ptr3(list(rhs_u) + [None] * 3), _ptr(rhs_p), int(ref_cycles), int(max_cycles),
                                out.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise StokesError(st, L.stokes_last_error(ctx).decode())
    return out
