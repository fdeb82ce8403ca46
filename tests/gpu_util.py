"""Helpers shared by the GPU tests: upload workloads, run the C-ABI, compare."""
from __future__ import annotations

import numpy as np


def to_dev(a):
    import torch
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def to_host(t):
    return None if t is None else t.detach().cpu().numpy()


def solver_for(prob, theta=1.0, **opts):
    import paper_1901_07892_amd as S
    rho = [to_dev(r) for r in prob.rho_faces[:prob.dim]]
    mu = to_dev(prob.mu)
    s = S.StokesSolver(prob.dim, prob.n, prob.h, rho, mu, prob.dt, visc_scale=theta, **opts)
    s._keep = (rho, mu)
    return s


def gpu_solve(prob, tol=None, theta=1.0, x0=None, **opts):
    import torch
    s = solver_for(prob, theta=theta, **opts)
    rhs_u = [to_dev(f) for f in prob.rhs_u[:prob.dim]]
    rhs_p = to_dev(prob.rhs_p)
    if x0 is None:
        xu = [torch.zeros_like(f) for f in rhs_u]
        xp = torch.zeros_like(rhs_p)
    else:
        xu = [to_dev(a) for a in x0[0]]
        xp = to_dev(x0[1])
    st, stats = s.solve(rhs_u, rhs_p, prob.tol if tol is None else tol, xu, xp)
    torch.cuda.synchronize()
    out = ([to_host(a) for a in xu], to_host(xp), st, stats)
    s.close()
    return out


def gpu_apply(prob, xu, xp, theta=1.0, **opts):
    import torch
    s = solver_for(prob, theta=theta, **opts)
    xd = [to_dev(a) for a in xu[:prob.dim]]
    pd = to_dev(xp)
    yd = [torch.full_like(a, np.nan) for a in xd]
    yp = torch.full_like(pd, np.nan)
    s.apply(xd, pd, yd, yp)
    torch.cuda.synchronize()
    s.close()
    return [to_host(a) for a in yd], to_host(yp)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
