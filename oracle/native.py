"""ctypes binding of the C oracle (``stokes_oracle.c`` -> ``liboracle.so``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "stokes_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP).  Always recompiles."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        pp = C.POINTER(dp)
        L.oracle_apply.argtypes = [C.c_int, ip, dp, C.c_double, C.c_double, pp, dp, pp, pp]
        L.oracle_apply.restype = C.c_int
        L.oracle_solve.argtypes = [C.c_int, ip, dp, C.c_double, C.c_double, pp, dp, pp,
                                   C.c_double, ip, C.c_double, pp, dp]
        L.oracle_solve.restype = C.c_int
        L.oracle_precond.argtypes = [C.c_int, ip, dp, C.c_double, C.c_double, pp, dp, ip, pp, pp]
        L.oracle_precond.restype = C.c_int
        L.oracle_auto_sigma.argtypes = [C.c_int, ip, dp, C.c_double, C.c_double, pp, dp, dp]
        L.oracle_auto_sigma.restype = C.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return C.cast(None, C.POINTER(C.c_double))
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _parr(arrs):
    t = (C.POINTER(C.c_double) * len(arrs))()
    for i, a in enumerate(arrs):
        t[i] = _dp(a)
    return t


def _grid_args(dim, n, h):
    ni = (C.c_int * 3)(*[int(v) for v in n])
    hd = (C.c_double * 3)(*[float(v) for v in h])
    return ni, hd


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def apply(dim, n, h, dt, theta, rho_faces, mu, xu, xp):
    """y = K x in the API layout; returns (yu list, yp)."""
    rho = [_c(r) for r in list(rho_faces) + [None] * (3 - len(rho_faces))][:3]
    mu = _c(mu)
    xs = [_c(a) for a in (list(xu) + [None] * 3)[:3]] + [_c(xp)]
    ys = [None if a is None else np.zeros_like(a) for a in xs]
    ni, hd = _grid_args(dim, n, h)
    rc = lib().oracle_apply(dim, ni, hd, dt, theta, _parr(rho), _dp(mu), _parr(xs), _parr(ys))
    if rc != 0:
        raise ValueError("oracle_apply failed")
    return ys[:3], ys[3]


DEFAULT_OPTS = dict(restart=30, max_iters=300, nu1=2, nu2=2, vel_cycles=1, p_cycles=1,
                    coarse_sweeps=400)


def solve(dim, n, h, dt, theta, rho_faces, mu, fu, fp, tol, x0u=None, x0p=None,
          cont_scale=0.0, **opts):
    """FGMRES solve; returns (xu list, xp, info dict).

    ``cont_scale`` weights the continuity rows in the residual norm (0: automatic
    balance, 1: the plain 2-norm).
    """
    o = dict(DEFAULT_OPTS)
    o.update(opts)
    rho = [_c(r) for r in (list(rho_faces) + [None] * 3)[:3]]
    mu = _c(mu)
    fs = [_c(a) for a in (list(fu) + [None] * 3)[:3]] + [_c(fp)]
    if x0u is None:
        xs = [None if a is None else np.zeros_like(a) for a in fs]
    else:
        xs = [_c(a).copy() if a is not None else None for a in (list(x0u) + [None] * 3)[:3]]
        xs.append(_c(x0p).copy())
    ni, hd = _grid_args(dim, n, h)
    oa = (C.c_int * 7)(o["restart"], o["max_iters"], o["nu1"], o["nu2"], o["vel_cycles"],
                       o["p_cycles"], o["coarse_sweeps"])
    out = np.zeros(10)
    rc = lib().oracle_solve(dim, ni, hd, dt, theta, _parr(rho), _dp(mu), _parr(fs), tol, oa,
                            float(cont_scale), _parr(xs), _dp(out))
    if rc != 0:
        raise ValueError("oracle_solve failed")
    info = dict(iters=int(out[0]), restarts=int(out[1]), status=int(out[2]),
                rel_res_est=out[3], rel_res_true=out[4], g_mean=out[5], levels=int(out[6]),
                sigma=out[7], setup_s=out[8], solve_s=out[9])
    return xs[:3], xs[3], info


def precond(dim, n, h, dt, theta, rho_faces, mu, ru, rp, **opts):
    o = dict(DEFAULT_OPTS)
    o.update(opts)
    rho = [_c(r) for r in (list(rho_faces) + [None] * 3)[:3]]
    rs = [_c(a) for a in (list(ru) + [None] * 3)[:3]] + [_c(rp)]
    zs = [None if a is None else np.zeros_like(a) for a in rs]
    ni, hd = _grid_args(dim, n, h)
    oa = (C.c_int * 7)(o["restart"], o["max_iters"], o["nu1"], o["nu2"], o["vel_cycles"],
                       o["p_cycles"], o["coarse_sweeps"])
    rc = lib().oracle_precond(dim, ni, hd, dt, theta, _parr(rho), _dp(_c(mu)), oa, _parr(rs), _parr(zs))
    if rc != 0:
        raise ValueError("oracle_precond failed")
    return zs[:3], zs[3]


def auto_sigma(prob, theta=1.0) -> float:
    """The oracle's continuity weight of the residual norm for a ``workloads.Problem``."""
    rho = [_c(r) for r in (list(prob.rho_faces[:prob.dim]) + [None] * 3)[:3]]
    ni, hd = _grid_args(prob.dim, prob.n, prob.h)
    out = C.c_double()
    rc = lib().oracle_auto_sigma(prob.dim, ni, hd, prob.dt, theta, _parr(rho), _dp(_c(prob.mu)), C.byref(out))
    if rc != 0:
        raise ValueError("oracle_auto_sigma failed")
    return out.value


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    lib().oracle_set_threads(int(n))


def solve_problem(prob, tol=None, theta=1.0, **opts):
    """Oracle FGMRES on a ``workloads.Problem``."""
    return solve(prob.dim, prob.n, prob.h, prob.dt, theta, prob.rho_faces, prob.mu,
                 prob.rhs_u[:prob.dim], prob.rhs_p, prob.tol if tol is None else tol, **opts)


def apply_problem(prob, xu, xp, theta=1.0):
    return apply(prob.dim, prob.n, prob.h, prob.dt, theta, prob.rho_faces, prob.mu, xu[:prob.dim], xp)
