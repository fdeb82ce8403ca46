"""GPU parity of the SSP-RK3 face-density transport (stokes_density_rk3) with the
oracle (oracle/transport.py), element by element, and its invariants at the
256^3 headline size.

Tolerance: both sides evaluate the same fluxes in FP64 with the same limiter
branches; they differ only in rounding order (and, at a limiter break point,
by the limiter's continuity), so |gpu - oracle| <= 1e-13 max|rho|."""
import numpy as np
import pytest

import workloads as W
from oracle import transport as OT
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _gpu(dim, n, h, dt, rho, stages):
    import torch
    import paper_1901_07892_amd as S
    grid = S._binding.make_grid(dim, n, h)
    rd = [to_dev(a) for a in rho]
    ud = [[to_dev(a) for a in st] for st in stages]
    out = [torch.full_like(a, np.nan) for a in rd]
    ws = torch.empty(S.stokes_density_workspace_size(grid), dtype=torch.uint8, device="cuda")
    print("stokes_density_rk3 dim=%d n=%s dt=%g" % (dim, tuple(n), dt), flush=True)
    S.stokes_density_rk3(grid, dt, rd, ud, out, ws)
    torch.cuda.synchronize()
    return [to_host(a) for a in out]


def _stages(dim, n, h, seed, margin=0):
    return [W.stream_velocity(n, h, dim, seed + s, margin=margin) for s in range(3)]


def _random_stages(dim, n, seed):
    """Arbitrary (not divergence-free) stage velocities with zero wall-normal entries."""
    out = []
    for s in range(3):
        xs, _ = W.random_vector(n, dim, seed + s)
        out.append(xs[:dim])
    return out


def _check(got, want, dim):
    scale = max(np.abs(w).max() for w in want)
    errs = [float(np.abs(got[c] - want[c]).max() / scale) for c in range(dim)]
    print("  max |gpu - oracle| / max|rho| per component", ["%.1e" % e for e in errs], flush=True)
    for c in range(dim):
        assert np.all(np.isfinite(got[c]))
    assert max(errs) <= 1e-13, errs


CASES = [
    # config 1's densities (air/water/solid, ratio 833) in a divergence-free flow, CFL 0.4
    ("config1_64", lambda: W.config1(), "stream", 0.4),
    # config 2's wavy interface and three discs at a quarter of its size
    ("config2_128", lambda: W.config2(scale=4), "stream", 0.4),
    # config 3's dam break at 32^3
    ("config3_32", lambda: W.config3(scale=4), "stream", 0.3),
    # the headline recipe at 48^3 with arbitrary (not divergence-free) stage velocities
    ("config5_48_random_u", lambda: W.config5(n_cells=48), "random", 0.2),
]


@pytest.mark.parametrize("name,maker,kind,cfl", CASES)
def test_density_transport_matches_oracle(name, maker, kind, cfl):
    prob = maker()
    dim, n, h = prob.dim, prob.n, prob.h
    rho = [prob.rho_faces[c] for c in range(dim)]
    stages = _stages(dim, n, h, 11) if kind == "stream" else _random_stages(dim, n, 21)
    umax = max(float(np.abs(a).max()) for st in stages for a in st)
    dt = cfl * min(h[:dim]) / umax
    got = _gpu(dim, n, h, dt, rho, stages)
    want = OT.ssp_rk3(dim, h, dt, rho, stages)
    _check(got, want, dim)
    moved = max(float(np.abs(want[c] - rho[c]).max()) for c in range(dim))
    assert moved > 1e-3 * max(float(np.abs(r).max()) for r in rho)     # the interface did move


@pytest.mark.parametrize("dim,n", [(2, (7, 5, 1)), (3, (5, 9, 6)), (3, (2, 2, 2)), (3, (3, 2, 4))])
def test_density_transport_ragged_and_minimal_grids(dim, n):
    rng = np.random.default_rng(sum(n))
    h = (0.2, 0.15, 0.1)
    rho = [rng.uniform(1.0, 1000.0, size=W.face_shape(n, c)) for c in range(dim)]
    stages = _random_stages(dim, n, 3)
    got = _gpu(dim, n, h, 0.01, rho, stages)
    _check(got, OT.ssp_rk3(dim, h, 0.01, rho, stages), dim)


def test_density_transport_full_size_headline():
    """The 256^3 headline densities (two solids, density ratio 1000): element by
    element against the oracle, and mass conserved to round-off by a flow that
    vanishes near the walls."""
    prob = W.config5()
    dim, n, h = 3, prob.n, prob.h
    rho = [prob.rho_faces[c] for c in range(3)]
    stages = _stages(dim, n, h, 31, margin=2)
    dt = 0.3 * h[0]                                       # max |u| = 1
    got = _gpu(dim, n, h, dt, rho, stages)
    print("  oracle at 256^3 ...", flush=True)
    want = OT.ssp_rk3(dim, h, dt, rho, stages)
    _check(got, want, dim)
    for c in range(3):
        m0, m1 = float(rho[c].sum()), float(got[c].sum())
        print("  component %d: mass %.15e -> %.15e" % (c, m0, m1), flush=True)
        assert abs(m1 - m0) <= 1e-12 * m0


def test_density_transport_argument_errors():
    import torch
    import paper_1901_07892_amd as S
    n, h = (4, 4, 4), (0.25,) * 3
    grid = S._binding.make_grid(3, n, h)
    rho = [torch.ones(W.face_shape(n, c), dtype=torch.float64, device="cuda") for c in range(3)]
    u = [[torch.zeros_like(a) for a in rho] for _ in range(3)]
    out = [torch.zeros_like(a) for a in rho]
    ws = torch.empty(S.stokes_density_workspace_size(grid), dtype=torch.uint8, device="cuda")
    with pytest.raises(S.StokesError) as e:
        S.stokes_density_rk3(grid, -1.0, rho, u, out, ws)
    assert e.value.status == -1
    with pytest.raises(S.StokesError) as e:
        S.stokes_density_rk3(grid, 0.1, rho, u, out, ws[:8])
    assert e.value.status == -3
    bad = S._binding.make_grid(3, (1, 4, 4), h)
    with pytest.raises(S.StokesError) as e:
        S.stokes_density_rk3(bad, 0.1, rho, u, out, ws)
    assert e.value.status == -2
