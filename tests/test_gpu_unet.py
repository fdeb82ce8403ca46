"""The learned form's network on the GPU against the numpy oracle network.

Forward: the BF16/MFMA U-Net equals the oracle forward (float64 arithmetic with
the same BF16 rounding of inputs, weights and activations) to a relative L2
error set by BF16 storage (2^-8 per rounding, a few roundings deep).
Backward: the gradient of one training step matches central finite differences
of the oracle loss (float64, no rounding) on sampled parameters.
"""
import numpy as np
import pytest

from oracle import unet as OU

pytestmark = pytest.mark.gpu


def _net(n, seed=3):
    import paper_1901_07892_amd as S
    net = S.UNet(n, seed=seed)
    rng = np.random.default_rng(seed)
    p = np.zeros(OU.param_count())
    ws, off = [], 0
    for _, ci, co, _ in OU.SPEC:
        cnt = co * 27 * ci
        fan = 27 * (3 if off == 0 else ci)
        p[off:off + cnt] = rng.uniform(-1, 1, cnt) * np.sqrt(6.0 / fan)
        off += cnt
    p[off:] = rng.uniform(-0.05, 0.05, p.size - off)
    p = OU.round_bf16(p).astype(np.float32)          # weights exactly representable in BF16
    net.set_params(p)
    return net, p.astype(np.float64)


def _feats(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    f = OU.round_bf16(rng.standard_normal((3, n, n, n)))
    dev = [torch.from_numpy(np.ascontiguousarray(f[c], dtype=np.float32)).cuda() for c in range(3)]
    return f, dev


@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_unet_forward_matches_oracle(n):
    import torch
    net, p = _net(n)
    f, dev = _feats(n, 11)
    out = torch.zeros((n, n, n), dtype=torch.float32, device="cuda")
    net.forward(dev[0], dev[1], dev[2], out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = OU.forward(p, f, bf16=True)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("unet forward n=%d rel L2 %.2e" % (n, err))
    assert err <= 2e-2
    net.close()


def test_unet_gradient_matches_finite_differences():
    import torch
    n = 8
    net, p = _net(n, seed=5)
    f, dev = _feats(n, 12)
    target = np.random.default_rng(13).standard_normal((n, n, n))
    tdev = torch.from_numpy(target.astype(np.float32)).cuda()
    net.train_step(dev[0], dev[1], dev[2], tdev, 0.0)      # lr 0: gradient only
    g = net.get_grads().astype(np.float64)
    rng = np.random.default_rng(14)
    # sample parameters from every layer, weights and biases
    idx = []
    off = 0
    for _, ci, co, _ in OU.SPEC:
        cnt = co * 27 * ci
        idx += list(off + rng.choice(cnt, 4, replace=False))
        off += cnt
    idx += list(off + rng.choice(p.size - off, 8, replace=False))
    fd = []
    for i in idx:
        h = 1e-3 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd.append((OU.loss(pp, f, target) - OU.loss(pm, f, target)) / (2 * h))
    fd = np.array(fd)
    gs = g[idx]
    cos = gs @ fd / (np.linalg.norm(gs) * np.linalg.norm(fd))
    big = np.abs(fd) > 0.05 * np.abs(fd).max()
    rel = np.abs(gs[big] - fd[big]) / np.abs(fd[big])
    print("grad cosine %.4f, median rel err %.3f on %d large components" % (cos, np.median(rel), big.sum()))
    assert cos >= 0.98
    assert np.median(rel) <= 0.1
    net.close()


def test_unet_training_reduces_loss():
    import torch
    n = 16
    net, p = _net(n, seed=7)
    f, dev = _feats(n, 21)
    # a smooth target the network can fit
    z, y, x = np.meshgrid(*(np.linspace(0, 1, n),) * 3, indexing="ij")
    target = torch.from_numpy((np.sin(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * z)).astype(np.float32)).cuda()
    losses = [net.train_step(dev[0], dev[1], dev[2], target, 2e-3) for _ in range(60)]
    print("loss %.4f -> %.4f" % (losses[0], losses[-1]))
    assert losses[-1] < 0.3 * losses[0]
    net.close()


@pytest.mark.parametrize("n", [16, 24])
def test_unet_training_is_deterministic(n):
    """Weight, bias and loss reductions go through per-block partial sums added in
    a fixed order: the same steps from the same start give bitwise-equal
    parameters and losses (n = 24 takes the ragged-grid kernels)."""
    import torch
    f, dev = _feats(n, 31)
    target = torch.from_numpy(np.random.default_rng(32).standard_normal((n, n, n)).astype(np.float32)).cuda()
    runs = []
    for _ in range(2):
        net, _p = _net(n, seed=9)
        losses = [net.train_step(dev[0], dev[1], dev[2], target, 1e-3) for _ in range(3)]
        runs.append((losses, net.get_params(), net.get_grads()))
        net.close()
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])


def test_unet_forward_ragged_grid_matches_oracle():
    """n = 24 (a multiple of 8, not of 16) takes the gather kernel on every level."""
    import torch
    n = 24
    net, p = _net(n)
    f, dev = _feats(n, 17)
    out = torch.zeros((n, n, n), dtype=torch.float32, device="cuda")
    net.forward(dev[0], dev[1], dev[2], out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = OU.forward(p, f, bf16=True)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("unet forward n=%d rel L2 %.2e" % (n, err))
    assert err <= 2e-2
    net.close()


def _learned_solver(prob, net, stall=0.9, **opts):
    import paper_1901_07892_amd as S
    from tests.gpu_util import solver_for
    s = solver_for(prob, **opts)
    S.stokes_attach_learned(s.ctx, net, stall)
    return s


def _solve_with(s, prob, tol):
    import torch
    from tests.gpu_util import to_dev, to_host
    rhs_u = [to_dev(f) for f in prob.rhs_u[:3]]
    rhs_p = to_dev(prob.rhs_p)
    xu = [torch.zeros_like(f) for f in rhs_u]
    xp = torch.zeros_like(rhs_p)
    st, stats = s.solve(rhs_u, rhs_p, tol, xu, xp)
    torch.cuda.synchronize()
    return [to_host(a) for a in xu], to_host(xp), st, stats


def test_learned_tuple_normalisation():
    """Tuples on the 32^3 level of a 64^3 headline-recipe instance."""
    import torch
    import workloads as W
    import paper_1901_07892_amd as S
    from tests.gpu_util import solver_for, to_dev
    prob = W.config5(n_cells=64, seed=7)
    s = solver_for(prob)
    out = [torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda") for _ in range(4)]
    S.stokes_learned_tuple(s.ctx, [to_dev(f) for f in prob.rhs_u[:3]], to_dev(prob.rhs_p), 32, 8, *out)
    f0, f1, sc, ph = [o.cpu().numpy() for o in out]
    assert abs(np.sqrt(np.mean(sc ** 2)) - 1) < 1e-4
    assert abs(ph.mean()) < 1e-4 and abs(np.sqrt(np.mean(ph ** 2)) - 1) < 1e-4
    assert f0.min() >= np.log10(0.99) / 3 - 0.5 and f0.max() <= np.log10(1001) / 3 - 0.5
    assert f1.min() >= np.log10(1.7e-5) / 2 + 2 and f1.max() <= np.log10(1.01e-3) / 2 + 2
    s.close()


@pytest.mark.parametrize("stall", [0.9, 0.0])
def test_learned_form_matches_oracle(oracle_lib, stall):
    """An untrained network attached as the learned stage: the FP64 residual check
    still decides convergence, the answer matches the oracle's FGMRES solution at
    tol 1e-13 (relative L2 <= 1e-9 per field), and with stall_ratio 0 the fallback
    to plain multigrid is taken and reported."""
    import workloads as W
    import paper_1901_07892_amd as S
    from tests.gpu_util import rel
    prob = W.config5(n_cells=64, seed=7)
    print("learned form vs oracle", prob.n, "stall", stall, flush=True)
    ou, op, info = oracle_lib.solve_problem(prob, tol=1e-13, max_iters=400)
    assert info["status"] == 0 or info["rel_res_true"] <= 1e-12, info
    net = S.UNet(32, seed=1)
    s = _learned_solver(prob, net, stall, max_iters=400)
    xu, xp, st, stats = _solve_with(s, prob, 1e-13)
    print("  learned(untrained) status %d iters %d res %.2e fell_back %d; oracle iters %d" %
          (st, stats.iters, stats.rel_res_true, stats.fell_back, info["iters"]), flush=True)
    assert st == 0 or (st == 1 and stats.rel_res_true <= 1e-12), stats.as_dict()
    if stall == 0.0:
        assert stats.fell_back == 1
    errs = [rel(xu[c], ou[c]) for c in range(3)] + [rel(xp - xp.mean(), op - op.mean())]
    print("  rel errors per field", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= 1e-9, errs
    s.close()
    net.close()


def test_trained_learned_form_on_headline_instance(oracle_lib):
    """With the committed trained weights, on the 256^3 headline instance at tol 1e-8:
    the learned form converges, and the oracle's operator with its own continuity
    weight confirms the residual in the weighted and the plain 2-norm."""
    import workloads as W
    import paper_1901_07892_amd as S
    from paper_1901_07892_amd import learned
    p, meta = learned.load_params()
    if p is None:
        pytest.skip("no trained weights in the package")
    prob = W.config5()
    print("trained learned form", prob.n, flush=True)
    net = S.UNet(32)
    net.set_params(p)
    s = _learned_solver(prob, net)
    xu, xp, st, stats = _solve_with(s, prob, prob.tol)
    print("  status %d iters %d res %.2e fell_back %d" % (st, stats.iters, stats.rel_res_true, stats.fell_back),
          flush=True)
    assert st == 0 and stats.rel_res_true <= prob.tol
    sigma = oracle_lib.auto_sigma(prob)
    yu, yp = oracle_lib.apply_problem(prob, xu, xp)
    r2 = sum(np.sum((prob.rhs_u[c] - yu[c]) ** 2) for c in range(3))
    b2 = sum(np.sum(prob.rhs_u[c] ** 2) for c in range(3))
    rp2 = np.sum(yp ** 2)                                   # rhs_p = 0
    plain, weighted = np.sqrt((r2 + rp2) / b2), np.sqrt((r2 + sigma ** 2 * rp2) / b2)
    print("  oracle residual plain %.2e weighted %.2e" % (plain, weighted), flush=True)
    assert plain <= prob.tol and weighted <= 1.01 * prob.tol
    s.close()
    net.close()
