"""GPU parity of the pressure-multigrid kernels, one launch at a time.

Through the C-ABI test hook stokes_pressure_op, the finest-level red-black
sweep and residual + restriction run exactly as the cycle launches them (the
fused z-marching sweep on 3D levels of more than 2^18 cells, the z-marching
residual + restriction on levels of at least 2^21 cells) and in their flat
forms, on the workloads' own coefficients at their stated sizes (config 3's
128^3, config 4's 1024x96x96, the 256^3 headline) and on ragged grids that
leave partial tiles.  Each result is compared element by element with the
oracle's definition of the kernel (oracle/mg_ops.py); fused and flat forms
are compared with each other as well.  The sweeps run with the relaxation
factor of the 3D default (red-black SOR, omega = 1.1) and, on config 3, as
plain Gauss-Seidel (omega = 1).
"""
import numpy as np
import pytest

import workloads as W
from oracle import mg_ops as M
from tests.gpu_util import solver_for, to_dev, to_host

pytestmark = pytest.mark.gpu

OMEGA = 1.1          # the automatic relaxation of 3D grids


def _rand_coeff_problem(n, seed, h=None):
    rng = np.random.default_rng(seed)
    dim = 3 if n[2] > 1 else 2
    h = h or (1.0 / n[0],) * 3
    rho = [rng.uniform(1.0, 1000.0, size=W.face_shape(n, a)) if a < dim else None for a in range(3)]
    mu = np.full(W.cell_shape(n), 1e-3)
    return W.Problem(name="rand", dim=dim, n=n, h=h, dt=1e-4, rho_faces=rho, mu=mu,
                     rhs_u=[np.zeros(W.face_shape(n, a)) for a in range(dim)],
                     rhs_p=np.zeros(W.cell_shape(n)), tol=1e-8)


CASES = [
    # 2^21 cells: fused 64x16 sweep and z-marching residual + restriction
    ("config3_128", lambda: W.config3()),
    # 1,105,920 cells: fused 64x16 sweep with partial tiles in x and y, per-cell restriction
    ("rand_136x72x113_odd_z", lambda: _rand_coeff_problem((136, 72, 113), 11)),
    # 2,220,032 cells: fused sweep and z-marching restriction with partial tiles in x, y and z chunks
    ("rand_136x136x120", lambda: _rand_coeff_problem((136, 136, 120), 12)),
    # between 2^18 and 2^20 cells: the pipelined 32x16 fused sweep
    ("config5_96", lambda: W.config5(n_cells=96)),
    # at most 2^18 cells: two flat colour passes, the prolongation folded into them
    ("config5_64", lambda: W.config5(n_cells=64)),
    ("rand_64x48x40", lambda: _rand_coeff_problem((64, 48, 40), 14)),
    ("config2_512", lambda: W.config2()),
]


def _tol(precision):
    return 1e-13 if precision == 0 else 2e-5


def _inputs(prob, seed):
    rng = np.random.default_rng(seed)
    shape = W.cell_shape(prob.n)
    e = rng.standard_normal(shape)
    r = rng.standard_normal(shape) * 1e3
    nc = tuple(max(v // 2, 1) for v in prob.n[:prob.dim]) + ((1,) if prob.dim == 2 else ())
    ec = rng.standard_normal(W.cell_shape(nc))
    return e, r, ec


def _as_precision(a, precision):
    return a if precision == 0 else a.astype(np.float32).astype(np.float64)


def _run(prob, precision, ops, p_prolong=0, open_top=0, omega=OMEGA):
    import torch
    extra = {"vel_levels": 1} if open_top else {}          # the open top needs the diagonal velocity step
    s = solver_for(prob, precision=precision, p_prolong=p_prolong, open_top=open_top, p_omega=omega, **extra)
    e, r, ec = _inputs(prob, 7)
    out = {}
    try:
        for name, op, use_e, use_ec in ops:
            coarse = op in (2, 3)
            shape = W.cell_shape(tuple(v // 2 for v in prob.n[:prob.dim]) + ((1,) if prob.dim == 2 else ())) \
                if coarse else W.cell_shape(prob.n)
            y = torch.full(shape, np.nan, dtype=torch.float64, device="cuda")
            print("  op", name, prob.n, "precision", precision, flush=True)
            s.pressure_op(op, to_dev(e) if use_e else None, to_dev(r), to_dev(ec) if use_ec else None, y)
            torch.cuda.synchronize()
            out[name] = to_host(y)
    finally:
        s.close()
    return e, r, ec, out


OPS = [("sweep", 0, True, False), ("sweep_flat", 1, True, False),
       ("sweep_zero", 0, False, False), ("sweep_zero_flat", 1, False, False),
       ("sweep_ec", 0, True, True), ("sweep_ec_flat", 1, True, True),
       ("restrict", 2, True, False), ("restrict_flat", 3, True, False)]


def _oracle(prob, precision, e, r, ec, names, lin=False, open_top=False, omega=OMEGA):
    """The oracle's result of each kernel in ``names`` on the same (rounded) inputs."""
    dim = prob.dim
    rho = [np.asarray(prob.rho_faces[c]) for c in range(dim)]
    beta = M.betas(dim, rho, open_top)
    if precision == 1:
        beta = [_as_precision(b, 1) for b in beta]
    e, r, ec = (_as_precision(a, precision) for a in (e, r, ec))
    h = prob.h
    ot = open_top
    make = {
        "sweep": lambda: M.rb_gs_sweep(dim, h, beta, e, r, ot, omega),
        "sweep_zero": lambda: M.rb_gs_sweep(dim, h, beta, np.zeros_like(e), r, ot, omega),
        "sweep_ec": lambda: M.rb_gs_sweep(dim, h, beta, e + M.prolong(dim, ec, lin), r, ot, omega),
        "restrict": lambda: M.residual_restrict(dim, h, beta, e, r, ot),
    }
    return {k: make[k]() for k in names}


def _check(prob, precision, got, ref):
    tol = _tol(precision)
    for name, want in ref.items():
        for form in (name, name + "_flat"):
            err = np.abs(got[form] - want).max() / np.abs(want).max()
            print("  %-16s max rel err vs oracle %.2e" % (form, err), flush=True)
            assert np.all(np.isfinite(got[form])), form
            assert err <= tol, (form, err)
        d = np.abs(got[name] - got[name + "_flat"]).max() / np.abs(want).max()
        assert d <= (1e-14 if precision == 0 else 1e-5), (name, d)


@pytest.mark.parametrize("name,maker", CASES)
def test_pressure_kernels_match_oracle(name, maker):
    prob = maker()
    if prob.n[2] % 2 and prob.dim == 3:
        ops = [o for o in OPS if o[1] in (0, 1) and not o[3]]   # odd z: no coarser level
    else:
        ops = OPS
    print("pressure kernels", name, prob.n, flush=True)
    e, r, ec, got = _run(prob, 0, ops)
    _check(prob, 0, got, _oracle(prob, 0, e, r, ec, [k for k in got if not k.endswith("_flat")]))


def test_pressure_kernels_gauss_seidel_match_oracle():
    """omega = 1: the unrelaxed update (the Gauss-Seidel value itself, no blend)."""
    prob = W.config3()
    print("pressure kernels, Gauss-Seidel", prob.n, flush=True)
    e, r, ec, got = _run(prob, 0, OPS, omega=1.0)
    _check(prob, 0, got, _oracle(prob, 0, e, r, ec, [k for k in got if not k.endswith("_flat")], omega=1.0))


@pytest.mark.parametrize("name,maker", [CASES[0], CASES[2]])
def test_pressure_kernels_fp32_match_oracle(name, maker):
    prob = maker()
    print("pressure kernels FP32", name, prob.n, flush=True)
    e, r, ec, got = _run(prob, 1, OPS)
    _check(prob, 1, got, _oracle(prob, 1, e, r, ec, [k for k in got if not k.endswith("_flat")]))


def test_pressure_kernels_trilinear_prolongation():
    prob = W.config3()
    print("pressure kernels, trilinear prolongation", prob.n, flush=True)
    ops = [("sweep_ec", 0, True, True), ("sweep_ec_flat", 1, True, True)]
    e, r, ec, got = _run(prob, 0, ops, p_prolong=1)
    dim = prob.dim
    beta = M.betas(dim, prob.rho_faces[:dim])
    want = M.rb_gs_sweep(dim, prob.h, beta, e + M.prolong(dim, ec, lin=True), r, omega=OMEGA)
    _check(prob, 0, got, {"sweep_ec": want})


@pytest.mark.parametrize("name,maker", [("config4_1024x96x96", lambda: W.config4()),
                                        ("config5_256", lambda: W.config5())])
def test_pressure_kernels_full_size(name, maker):
    """The workloads' full sizes, in the launch configuration the solver uses there."""
    prob = maker()
    print("pressure kernels full size", name, prob.n, flush=True)
    ops = [o for o in OPS if o[0] in ("sweep", "sweep_flat", "sweep_ec", "sweep_ec_flat",
                                      "restrict", "restrict_flat")]
    e, r, ec, got = _run(prob, 0, ops)
    _check(prob, 0, got, _oracle(prob, 0, e, r, ec, [k for k in got if not k.endswith("_flat")]))


def test_pressure_op_argument_errors():
    import torch
    import paper_1901_07892_amd as S
    prob = W.config3(scale=8)
    s = solver_for(prob)
    z = torch.zeros(W.cell_shape(prob.n), dtype=torch.float64, device="cuda")
    try:
        for args in [(7, z, z, None, z), (2, None, z, None, z), (0, None, z, z, z), (0, z, None, None, z)]:
            with pytest.raises(S.StokesError) as ei:
                s.pressure_op(*args)
            assert ei.value.status == -1
    finally:
        s.close()


@pytest.mark.parametrize("name,maker", [
    ("config4_1024x96x96_open_top", lambda: W.config4()),
    ("config4_2d_512x48_open_top", lambda: W.config4_2d(512, 48)),
    ("rand_136x72x112_open_top", lambda: _rand_coeff_problem((136, 72, 112), 13)),
])
def test_pressure_kernels_open_top_match_oracle(name, maker):
    """With the wave tank's open top the pressure is zero on the top faces (a
    Dirichlet row in every kernel, carried by doubled top-face coefficients)."""
    prob = maker()
    print("pressure kernels, open top", name, prob.n, flush=True)
    e, r, ec, got = _run(prob, 0, OPS, open_top=1)
    _check(prob, 0, got, _oracle(prob, 0, e, r, ec, [k for k in got if not k.endswith("_flat")], open_top=True))
