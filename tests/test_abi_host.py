"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function include/stokes.h declares, sizes workspaces and rejects bad arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "stokes.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stokes_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def S():
    import paper_1901_07892_amd as S
    S.load_library()
    return S


def test_exports_every_declared_symbol(S):
    names = _declared()
    assert "stokes_solve" in names and "stokes_setup" in names and "stokes_apply" in names
    lib = ctypes.CDLL(S.library_path())
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_size_host_logic(S):
    g = S._binding.make_grid(3, (256, 256, 256), (1 / 256,) * 3)
    o = S.stokes_default_options()
    assert o.restart == 30 and o.nu1 == 2 and o.nu2 == 2
    big = S.stokes_workspace_size(g, o)
    # (m+1) + m + 2 Krylov vectors of 4 padded fields dominate
    vec = 4 * 257 ** 3 * 8
    assert (2 * o.restart + 3) * vec < big < (2 * o.restart + 20) * vec
    o.restart = 10
    assert S.stokes_workspace_size(g, o) < big
    g2 = S._binding.make_grid(2, (64, 64, 1), (1 / 64,) * 3)
    assert 0 < S.stokes_workspace_size(g2, None) < 64 * 2 ** 20


@pytest.mark.parametrize("dim,n,h", [(4, (8, 8, 8), (1, 1, 1)), (2, (1, 8, 1), (1, 1, 1)),
                                     (3, (8, 8, 8), (1, 0, 1))])
def test_bad_grids_rejected_on_host(S, dim, n, h):
    g = S._binding.make_grid(dim, n, h)
    assert S.stokes_workspace_size(g, None) == 0
    with pytest.raises(S.StokesError) as e:
        S.stokes_setup([1, 2, 3], 4, 1e-3, g, None, 8, 16, stream=0)
    assert e.value.status in (-1, -2)
    assert len(S.stokes_last_error(None)) > 0


def test_bad_options_rejected_on_host(S):
    g = S._binding.make_grid(2, (8, 8, 1), (1, 1, 1))
    o = S.stokes_default_options()
    o.p_cycles = -1
    assert S.stokes_workspace_size(g, o) == 0
    o = S.stokes_default_options()
    with pytest.raises(S.StokesError) as e:
        S.stokes_setup([1, 2, None], 4, -1.0, g, o, 8, 1 << 30, stream=0)
    assert e.value.status == -1
    with pytest.raises(S.StokesError) as e:
        S.stokes_setup([1, 2, None], 4, 1e-3, g, o, 8, 16, stream=0)
    assert e.value.status == -3          # workspace too small, detected on the host


def test_options_struct_layout_matches_library(S):
    """The ctypes mirror of stokes_options ends where the C struct ends: the last
    fields read back with their documented defaults, and a bad value in the last
    field is rejected by the library's own validation."""
    o = S.stokes_default_options()
    assert (o.orth, o.matvec_z, o.p_gamma, o.p_small, o.p_wdepth, o.p_cycles, o.p_cycles_next, o.p_nu_second) == \
        (1, 1, 2, 1, 2, 0, 0, 0)
    g = S._binding.make_grid(3, (16, 16, 16), (1 / 16,) * 3)
    assert S.stokes_workspace_size(g, o) > 0
    o.p_wdepth = -1
    assert S.stokes_workspace_size(g, o) == 0
    o.p_wdepth = 0
    o.p_small = 2
    assert S.stokes_workspace_size(g, o) == 0
    o.p_small = 1
    o.p_cycles_next = -1
    assert S.stokes_workspace_size(g, o) == 0
    o.p_cycles_next = 0
    o.p_nu_second = -1
    assert S.stokes_workspace_size(g, o) == 0
    o.p_nu_second = 3
    assert S.stokes_workspace_size(g, o) > 0
    # the last field: the smoother's relaxation (0 = automatic, else in (0, 2))
    assert o.p_omega == 0.0
    for bad in (-0.5, 2.0, 2.5, float("nan")):
        o.p_omega = bad
        assert S.stokes_workspace_size(g, o) == 0, bad
    o.p_omega = 1.1
    assert S.stokes_workspace_size(g, o) > 0


def test_stream_copy_rejects_bad_arguments_on_host(S):
    L = S.load_library()
    assert L.stokes_stream_copy(None, None, -1, None) == -1
    assert L.stokes_stream_copy(None, None, 5, None) == -1
    assert L.stokes_stream_copy(None, None, 0, None) == 0


def test_coefficients_reject_bad_arguments_on_host(S):
    """Every argument check of stokes_coefficients returns before any HIP call
    (the pointers below are never dereferenced)."""
    B = S._binding
    g3 = B.make_grid(3, (8, 8, 8), (1 / 8,) * 3)
    ok = B.make_fluids(1000.0, 1.0, 1e-3, 1.8e-5, 1.5)
    fake = [0x1000, 0x2000, 0x3000]

    def call(grid=g3, fluids=ok, phi=0x4000, psi=(), rs=(), ms=(), rho=fake, mu=0x5000, flow=None):
        with pytest.raises(S.StokesError) as e:
            S.stokes_coefficients(grid, fluids, phi, list(psi), list(rs), list(ms), rho, mu, flow, stream=0)
        return e.value.status

    assert call(grid=B.make_grid(4, (8, 8, 8), (1, 1, 1))) == -1
    assert call(grid=B.make_grid(3, (8, 0, 8), (1, 1, 1))) == -2
    assert call(grid=B.make_grid(3, (2000, 2000, 2000), (1, 1, 1))) == -2
    assert call(grid=B.make_grid(3, (8, 8, 8), (1, -1, 1))) == -1
    assert call(phi=None) == -1
    assert call(mu=None) == -1
    assert call(rho=[0x1000, None, 0x3000]) == -1
    assert call(rho=[0x1000, 0x2000, None]) == -1                 # 3D needs rho_z
    assert call(flow=[0x1000, 0x2000, None]) == -1
    for bad in (B.make_fluids(0.0, 1.0, 1e-3, 1e-5, 1.5), B.make_fluids(1e3, 1.0, -1e-3, 1e-5, 1.5),
                B.make_fluids(1e3, float("nan"), 1e-3, 1e-5, 1.5), B.make_fluids(1e3, 1.0, 1e-3, 1e-5, 0.0)):
        assert call(fluids=bad) == -1
    assert call(psi=[0x6000], rs=[-5.0], ms=[1e-3]) == -1
    assert call(psi=[None], rs=[500.0], ms=[1e-3]) == -1
    assert call(psi=[0x6000] * (S.MAX_SOLIDS + 1), rs=[500.0] * (S.MAX_SOLIDS + 1),
                ms=[1e-3] * (S.MAX_SOLIDS + 1)) == -1
    L = S.load_library()
    assert L.stokes_coefficients(ctypes.byref(g3), ctypes.byref(ok), 0x4000, -1, None, None, None,
                                 B._ptr3(fake), 0x5000, None, None) == -1


def test_rigid_projection_rejects_bad_arguments_on_host(S):
    """Argument checks of stokes_rigid_projection return before any HIP call."""
    B = S._binding
    g = B.make_grid(3, (8, 8, 8), (1 / 8,) * 3)
    u = [0x1000, 0x2000, 0x3000]
    L = S.load_library()

    def call(grid=g, uu=u, n=10, X=0x4000, dV=1e-3, free=1, body=None, ws=0x5000, wsb=1 << 20):
        b = body if body is not None else B.make_body((0.5, 0.5, 0.5))
        return L.stokes_rigid_projection(ctypes.byref(grid), B._ptr3(uu), n, X, dV, free, ctypes.byref(b),
                                         ws, wsb, None)

    assert S.stokes_rigid_workspace_size(3, 10) == (10 * 3 + 13) * 8
    assert S.stokes_rigid_workspace_size(5, 10) == 0 and S.stokes_rigid_workspace_size(2, -1) == 0
    assert call(grid=B.make_grid(4, (8, 8, 8), (1, 1, 1))) == -1
    assert call(grid=B.make_grid(3, (8, 1, 8), (1, 1, 1))) == -2
    assert call(grid=B.make_grid(3, (8, 8, 8), (1, 0, 1))) == -1
    assert call(uu=[0x1000, None, 0x3000]) == -1
    assert call(n=-1) == -1
    assert call(X=None) == -1
    assert call(ws=None) == -1
    assert call(wsb=8) == -3
    assert call(dV=0.0) == -1 and call(dV=float("inf")) == -1
    assert call(free=2) == -1
    assert call(body=B.make_body((0.5, float("nan"), 0.5))) == -1
    assert call(n=0, free=1) == -1                     # a free body needs markers
    assert call(n=0, free=0) == 0                      # nothing to do, no device work


def test_explicit_rhs_rejects_bad_arguments_on_host(S):
    B = S._binding
    g = B.make_grid(3, (8, 8, 8), (1 / 8,) * 3)
    p3 = [0x1000, 0x2000, 0x3000]

    def call(grid=g, rho=p3, mu=0x4000, dt=1e-3, theta=0.5, un=p3, f=p3, rf=None, gv=None):
        with pytest.raises(S.StokesError) as e:
            S.stokes_explicit_rhs(grid, rho, mu, dt, theta, un, f, rf, gv, stream=0)
        return e.value.status

    assert call(grid=B.make_grid(4, (8, 8, 8), (1, 1, 1))) == -1
    assert call(grid=B.make_grid(3, (8, 8, 1), (1, 1, 1))) == -2
    assert call(mu=None) == -1
    assert call(rho=[0x1000, None, 0x3000]) == -1
    assert call(un=[0x1000, 0x2000, None]) == -1
    assert call(f=[None, 0x2000, 0x3000]) == -1
    assert call(dt=0.0) == -1 and call(dt=float("nan")) == -1
    assert call(theta=-0.1) == -1 and call(theta=1.5) == -1
    assert call(rf=p3, gv=(0.0, float("inf"), 0.0)) == -1
    assert call(rf=[0x1000, None, 0x3000], gv=(0, 0, -9.81)) == -1


def test_extreme_extents_rejected_on_host(S):
    """Grids whose point counts overflow 32-bit indices -- up to extents near
    INT_MAX, where the counts overflow 64-bit products as well -- are rejected by
    every entry point's host checks before any device work (the pointers below
    are never dereferenced)."""
    B = S._binding
    L = S.load_library()
    imax = 2 ** 31 - 1
    grids = [B.make_grid(3, (imax, imax, imax), (1.0, 1.0, 1.0)), B.make_grid(3, (imax, 8, 8), (1.0, 1.0, 1.0)),
             B.make_grid(2, (imax, imax, 1), (1.0, 1.0, 1.0)), B.make_grid(3, (2000, 2000, 2000), (1.0, 1.0, 1.0))]
    p3 = [0x1000, 0x2000, 0x3000]
    for g in grids:
        assert S.stokes_workspace_size(g, None) == 0
        with pytest.raises(S.StokesError) as e:
            S.stokes_setup(p3, 0x4000, 1e-3, g, None, 8, 16, stream=0)
        assert e.value.status == -2
        assert S.stokes_density_workspace_size(g) == 0
        with pytest.raises(S.StokesError) as e:
            S.stokes_coefficients(g, B.make_fluids(1e3, 1.0, 1e-3, 1e-5, 1.5), 0x4000, [], [], [], p3, 0x5000,
                                  None, stream=0)
        assert e.value.status == -2
        with pytest.raises(S.StokesError) as e:
            S.stokes_explicit_rhs(g, p3, 0x4000, 1e-3, 0.5, p3, p3, None, None, stream=0)
        assert e.value.status == -2
        us = (ctypes.c_void_p * 9)(*([0x1000] * 9))
        assert L.stokes_density_rk3(ctypes.byref(g), ctypes.c_double(1e-3), B._ptr3(p3), us, B._ptr3(p3),
                                    ctypes.c_void_p(0x6000), ctypes.c_size_t(1 << 62), None) == -2
    # the rigid projection indexes with 64-bit offsets: only beyond 2^40 points
    b = B.make_body((0.5, 0.5, 0.5))
    assert L.stokes_rigid_projection(ctypes.byref(grids[0]), B._ptr3(p3), 10, 0x4000, ctypes.c_double(1e-3), 1,
                                     ctypes.byref(b), 0x5000, 1 << 20, None) == -2
    # the wave inflow's arrays are (Nv + 1) x N_lateral
    w = B.make_wave(0.04, 0.5, 1.5, 2.0)
    assert L.stokes_wave_inflow(ctypes.byref(B.make_grid(2, (8, imax, 1), (1.0, 1.0, 1.0))), ctypes.byref(w),
                                ctypes.c_double(0.0), 0x1000, 0x2000, None) == -2


class _FakeTensor:
    """Stands in for a device tensor in the binding's argument checks (never
    dereferenced: every call below fails in the binding before the library)."""

    def __init__(self, numel):
        import torch
        self.dtype = torch.float64
        self.is_cuda = True
        self._n = numel
        self.shape = (numel,)

    def is_contiguous(self):
        return True

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x100000


def test_binding_refuses_arrays_shorter_than_the_grid(S):
    """The kernels index the caller's arrays from the grid alone, so the binding
    refuses a tensor with fewer values than its layout needs (u: (Nz, Ny, Nx+1),
    p and mu: (Nz, Ny, Nx), ...) instead of letting a kernel run past its end."""
    B = S._binding
    n = (6, 5, 4)
    g = B.make_grid(3, n, (0.1,) * 3)
    faces, cells = B._counts(g)
    assert faces == [7 * 5 * 4, 6 * 6 * 4, 6 * 5 * 5] and cells == 120
    g2 = B.make_grid(2, (6, 5, 1), (0.1,) * 3)
    assert B._counts(g2) == ([7 * 5, 6 * 6], 30)
    F = _FakeTensor
    good = [F(c) for c in faces]
    short_u = [F(faces[0]), F(faces[1] - 1), F(faces[2])]
    fl = B.make_fluids(1e3, 1.0, 1e-3, 1e-5, 1.5)
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_coefficients(g, fl, F(cells - 1), [], [], [], good, F(cells))
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_coefficients(g, fl, F(cells), [F(cells - 2)], [500.0], [1e-3], good, F(cells))
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_coefficients(g, fl, F(cells), [], [], [], short_u, F(cells))
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_explicit_rhs(g, good, F(cells), 1e-3, 0.5, short_u, good)
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_rigid_projection(g, good, _FakeMarkers(10, 2), 1e-3, 1,
                                  B.make_body((0.3, 0.25, 0.2)), None)
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_rigid_projection_noalloc(g, short_u, _FakeMarkers(10, 3), 1e-3, 1, B.make_body((0.3, 0.25, 0.2)))
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_wave_inflow(g, B.make_wave(0.04, 0.5, 1.5, 2.0), 0.0, F(4 * 5 - 1), F(5 * 5))
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_density_rk3(g, 1e-3, good, [good, short_u, good], good, None)
    with pytest.raises(ValueError, match="grid needs"):
        S.stokes_setup(short_u, F(cells), 1e-3, g, None, 0x200000, 1 << 20, stream=0)
    # a context's grid is kept for the calls that take the context
    B._CTX_COUNTS[0xdead0] = (faces, cells)
    B._CTX_INFLOW[0xdead0] = B._inflow_counts(g)
    try:
        with pytest.raises(ValueError, match="grid needs"):
            S.stokes_solve(0xdead0, good, F(cells), 1e-8, short_u, F(cells))
        with pytest.raises(ValueError, match="grid needs"):
            S.stokes_apply(0xdead0, good, F(cells - 1), good, F(cells))
        with pytest.raises(ValueError, match="grid needs"):
            S.stokes_inflow_lift(0xdead0, F(20), F(24), good, F(cells))
    finally:
        B._CTX_COUNTS.pop(0xdead0)
        B._CTX_INFLOW.pop(0xdead0)


class _FakeMarkers(_FakeTensor):
    """n markers with c coordinates each (c < dim is too few for the grid)."""

    def __init__(self, n, c):
        super().__init__(n * c)
        self.shape = (n, c)


def test_binding_passes_arrays_of_the_right_size(S, monkeypatch):
    """Every checked call marshals arrays of exactly the layout sizes (and larger
    ones) without complaint: run against a stand-in library that records the call
    and returns OK, so that no device is touched."""
    B = S._binding
    calls = []

    class _Lib:
        def __getattr__(self, name):
            def f(*a):
                calls.append(name)
                return 0
            return f

    monkeypatch.setattr(B, "_lib", _Lib())
    F = _FakeTensor
    for dim, n in ((3, (6, 5, 4)), (2, (6, 5, 1))):
        g = B.make_grid(dim, n, (0.1,) * 3)
        faces, cells = B._counts(g)
        u = [F(c) for c in faces]
        big = [F(c + 7) for c in faces]
        fl = B.make_fluids(1e3, 1.0, 1e-3, 1e-5, 1.5)
        S.stokes_coefficients(g, fl, F(cells), [F(cells)], [500.0], [1e-3], u, F(cells), big, stream=0)
        S.stokes_explicit_rhs(g, u, F(cells), 1e-3, 0.5, big, u, u, (0.0, -9.81, 0.0), stream=0)
        S.stokes_rigid_projection(g, u, _FakeMarkers(10, dim), 1e-3, 1, B.make_body((0.3, 0.25, 0.2)), None,
                                  stream=0)
        S.stokes_rigid_projection_noalloc(g, u, _FakeMarkers(10, dim), 1e-3, 1, B.make_body((0.3, 0.25, 0.2)),
                                          stream=0)
        n_n, n_t = B._inflow_counts(g)
        S.stokes_wave_inflow(g, B.make_wave(0.04, 0.5, 1.5, 2.0), 0.0, F(n_n), F(n_t), stream=0)
        S.stokes_density_rk3(g, 1e-3, u, [u, big, u], u, None, stream=0)
        ctx = S.stokes_setup(u, F(cells), 1e-3, g, None, 0x200000, 1 << 20, stream=0)
        assert ctx is None                       # the stand-in library writes no context
        B._CTX_COUNTS[0xbeef0] = (faces, cells)
        B._CTX_INFLOW[0xbeef0] = (n_n, n_t)
        try:
            S.stokes_apply(0xbeef0, u, F(cells), big, F(cells + 1))
            S.stokes_solve(0xbeef0, u, F(cells), 1e-8, u, F(cells))
            S.stokes_inflow_lift(0xbeef0, F(n_n), F(n_t), u, F(cells))
        finally:
            B._CTX_COUNTS.pop(0xbeef0)
            B._CTX_INFLOW.pop(0xbeef0)
    for name in ("stokes_coefficients", "stokes_explicit_rhs", "stokes_rigid_projection",
                 "stokes_rigid_projection_noalloc", "stokes_wave_inflow", "stokes_density_rk3", "stokes_setup",
                 "stokes_apply", "stokes_solve", "stokes_inflow_lift"):
        assert calls.count(name) == 2, name
