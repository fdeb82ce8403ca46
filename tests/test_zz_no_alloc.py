"""The allocation-free rigid projection (stokes_rigid_projection_noalloc) against
the workspace entry point (stokes_rigid_projection), through the C-ABI.

Two calls in a row on one GPU, the second with fewer markers than the first (the
fixed scratch keeps the first call's contents, which the second must not read),
in 3D and 2D, free-body and prescribed motion; then a call with more markers
than the scratch holds, which is refused on the host before any GPU work.

Tolerance: both entry points run the same kernels; the spread adds its
contributions with atomics in an arbitrary order, so the corrected velocities
agree to a few units of rounding of the largest contribution (1e-12 for O(1)
velocities) and the body velocities to 1e-11 relative."""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _ball(center, radius, h, dim, L):
    rng = [np.arange(max(math.floor((center[d] - radius) / h[d]), 0),
                     min(math.ceil((center[d] + radius) / h[d]) + 1, int(round(L[d] / h[d]))))
           for d in range(dim)]
    pts = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, dim)
    X = (pts + 0.5) * np.asarray(h[:dim])
    return X[np.linalg.norm(X - np.asarray(center[:dim]), axis=1) <= radius]


def _velocity(dim, n, seed):
    rng = np.random.default_rng(seed)
    u = [rng.standard_normal(W.face_shape(n, k)) for k in range(dim)]
    for k in range(dim):
        sl = [slice(None)] * 3
        for end in (0, -1):
            sl[2 - k] = end
            u[k][tuple(sl)] = 0.0
    return u


def _both(dim, n, h, u, X, free, Ur, Wr):
    import torch
    import paper_1901_07892_amd as S
    grid = S._binding.make_grid(dim, n, h)
    dV = float(np.prod(h[:dim]))
    xc = X.mean(0)
    Xd = to_dev(np.ascontiguousarray(X))
    ua = [to_dev(a) for a in u]
    ub = [to_dev(a) for a in u]
    ws = torch.empty(S.stokes_rigid_workspace_size(dim, len(X)), dtype=torch.uint8, device="cuda")
    print("rigid projection dim=%d n=%s markers=%d free=%d: workspace, then no-alloc" % (dim, tuple(n), len(X), free),
          flush=True)
    ba = S.stokes_rigid_projection(grid, ua, Xd, dV, free, S.make_body(xc, Ur, Wr), ws)
    torch.cuda.synchronize()
    bb = S.stokes_rigid_projection_noalloc(grid, ub, Xd, dV, free, S.make_body(xc, Ur, Wr))
    torch.cuda.synchronize()
    return [to_host(a) for a in ua], [to_host(a) for a in ub], ba, bb


CASES = [
    # dim, cells, spacing, (first ball centre, radius), (second, smaller ball)
    (3, (48, 40, 44), (1 / 48,) * 3, ((0.45, 0.4, 0.5), 0.3), ((0.3, 0.25, 0.6), 0.12)),
    (2, (96, 80, 1), (1 / 96,) * 3, ((0.5, 0.45), 0.35), ((0.2, 0.7), 0.1)),
]


@pytest.mark.parametrize("free", [1, 0])
@pytest.mark.parametrize("case", CASES, ids=["3d", "2d"])
def test_noalloc_matches_workspace_entry_point(case, free):
    dim, n, h, big, small = case
    L = [n[d] * h[d] for d in range(dim)]
    rng = np.random.default_rng(5 + free)
    Ur, Wr = rng.standard_normal(3), rng.standard_normal(3)
    sizes = []
    for call, (c, r) in enumerate([big, small]):
        X = _ball(c, r, h, dim, L)
        sizes.append(len(X))
        u = _velocity(dim, n, 17 + call)
        ga, gb, ba, bb = _both(dim, n, h, u, X, free, Ur, Wr)
        for k in range(dim):
            assert np.all(np.isfinite(gb[k]))
            np.testing.assert_allclose(gb[k], ga[k], rtol=0, atol=1e-12)
        va = np.array(list(ba.u_r) + list(ba.w_r))
        vb = np.array(list(bb.u_r) + list(bb.w_r))
        np.testing.assert_allclose(vb, va, rtol=1e-11, atol=1e-14)
        moved = max(float(np.abs(ga[k] - u[k]).max()) for k in range(dim))
        print("  call %d: %d markers, largest correction %.3g, max |noalloc - workspace| %.2e" %
              (call, len(X), moved, max(float(np.abs(gb[k] - ga[k]).max()) for k in range(dim))), flush=True)
        assert moved > 1e-3                      # the projection did act
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_more_markers_than_its_scratch():
    import torch
    import paper_1901_07892_amd as S
    dim, n, h = 3, (8, 8, 8), (0.125,) * 3
    grid = S._binding.make_grid(dim, n, h)
    u = [to_dev(a) for a in _velocity(dim, n, 3)]
    before = [a.clone() for a in u]
    X = torch.full((S.RIGID_NOALLOC_MAX_MARKERS + 1, 3), 0.5, dtype=torch.float64, device="cuda")
    print("rigid projection no-alloc: %d markers (one beyond the scratch)" % X.shape[0], flush=True)
    with pytest.raises(S.StokesError) as ei:
        S.stokes_rigid_projection_noalloc(grid, u, X, 0.1, 1, S.make_body((0.5, 0.5, 0.5)))
    torch.cuda.synchronize()
    assert ei.value.status == -3
    assert "524288" in str(ei.value)
    for a, b in zip(u, before):
        assert torch.equal(a, b)
