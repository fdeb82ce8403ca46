"""Pins of the learned-stage network oracle (oracle/unet.py) against things other
than itself: brute-force loops for the 3x3x3 convolution, scipy's correlation,
explicit block means for pooling and nearest upsampling, torch's float32 ->
bfloat16 conversion (round to nearest, ties to even), and closed forms of the
whole network for kernels that are (signed) identities on channel 0, where the
output reduces to sums of block means of the input."""
import numpy as np
import pytest

from oracle import unet as U


def _conv_loops(x, w, b):
    """out[z,y,x,co] = b[co] + sum over taps (dz,dy,dx) in {-1,0,1}^3 and ci of
    w[co, 9(dz+1) + 3(dy+1) + (dx+1), ci] * x[z+dz, y+dy, x+dx, ci], zero outside."""
    n, _, _, ci_n = x.shape
    co_n = w.shape[0]
    out = np.zeros((n, n, n, co_n))
    for z in range(n):
        for y in range(n):
            for xx in range(n):
                for co in range(co_n):
                    acc = b[co]
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, yy, x2 = z + dz, y + dy, xx + dx
                                if not (0 <= zz < n and 0 <= yy < n and 0 <= x2 < n):
                                    continue
                                tap = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                                for ci in range(ci_n):
                                    acc += w[co, tap, ci] * x[zz, yy, x2, ci]
                    out[z, y, xx, co] = acc
    return out


def _block_mean(x, k):
    """Mean of a 3D array over aligned blocks of side 2^k, by explicit loops."""
    n = x.shape[0]
    s = 1 << k
    m = n // s
    out = np.zeros((m, m, m))
    for a in range(m):
        for b in range(m):
            for c in range(m):
                out[a, b, c] = x[a * s:(a + 1) * s, b * s:(b + 1) * s, c * s:(c + 1) * s].sum() / s ** 3
    return out


def _spread(c, k):
    """Nearest (piecewise-constant) upsampling of a coarse array by 2^k per axis."""
    return np.kron(c, np.ones((1 << k,) * 3))


def test_conv3_matches_brute_force_loops():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 4, 4, 2))
    w = rng.standard_normal((3, 27, 2))
    b = rng.standard_normal(3)
    np.testing.assert_allclose(U.conv3(x, w, b), _conv_loops(x, w, b), rtol=0, atol=1e-12)


def test_conv3_matches_scipy_correlate():
    from scipy import ndimage
    rng = np.random.default_rng(4)
    n, ci_n, co_n = 8, 3, 2
    x = rng.standard_normal((n, n, n, ci_n))
    w = rng.standard_normal((co_n, 27, ci_n))
    b = np.zeros(co_n)
    ref = np.zeros((n, n, n, co_n))
    for co in range(co_n):
        for ci in range(ci_n):
            k = w[co, :, ci].reshape(3, 3, 3)       # [dz][dy][dx] with offsets -1..1
            ref[..., co] += ndimage.correlate(x[..., ci], k, mode="constant", cval=0.0)
    np.testing.assert_allclose(U.conv3(x, w, b), ref, rtol=0, atol=1e-11)


def test_pool_and_up_are_block_mean_and_nearest_spread():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((8, 8, 8, 1))
    np.testing.assert_allclose(U.pool(x)[..., 0], _block_mean(x[..., 0], 1), atol=1e-14)
    c = rng.standard_normal((4, 4, 4, 1))
    np.testing.assert_array_equal(U.up(c)[..., 0], _spread(c[..., 0], 1))


def test_round_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    vals = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-6, 6, 4000),
                           # exact ties between two bfloat16 neighbours: both parities of the kept bit
                           np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2 ** -126 * (1 + 2 ** -8),
                                     0.0, -0.0, 65504.0, 3.0e38])])
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(U.round_bf16(vals), ref)
    assert U.round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0                  # tie -> even mantissa
    assert U.round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6      # tie -> even mantissa


def _identity_params(signs=None):
    """Every layer maps input channel 0 to output channel 0 through the centre tap
    only (weight +1, or signs[layer]); all other weights and all biases zero."""
    ws, bs = [], []
    for i, (_, ci, co, _) in enumerate(U.SPEC):
        w = np.zeros((co, 27, ci))
        w[0, 13, 0] = 1.0 if signs is None else signs.get(i, 1.0)
        ws.append(w)
        bs.append(np.zeros(co))
    return np.concatenate([w.ravel() for w in ws] + bs)


def test_param_count_and_layout():
    p = _identity_params()
    assert p.size == U.param_count() == 594960
    ws, bs = U.split_params(p)
    assert len(ws) == len(bs) == 15
    assert all(w[0, 13, 0] == 1.0 and np.count_nonzero(w) == 1 for w in ws)


def test_identity_network_is_sum_of_block_means():
    """With identity kernels and non-negative input, every ReLU is inactive and the
    output is x + B1 x + B2 x + B3 x (B_k: mean over aligned 2^k blocks, spread back):
    three poolings on the way down, and on the way up each level adds its skip."""
    rng = np.random.default_rng(7)
    n = 8
    x = rng.random((n, n, n))
    feats = np.stack([x, rng.standard_normal((n, n, n)), rng.standard_normal((n, n, n))])
    y = U.forward(_identity_params(), feats, bf16=False)
    ref = x + sum(_spread(_block_mean(x, k), k) for k in (1, 2, 3))
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13)


def test_skip_is_added_before_the_relu():
    """Layer 8 (the first decoder convolution, on the level coarsened twice) with
    weight -1: that level computes relu(B2 x - spread(B3 x)); a skip added after
    the ReLU would give B2 x instead."""
    rng = np.random.default_rng(8)
    n = 8
    x = rng.random((n, n, n)) ** 3              # skewed so that the difference changes sign
    feats = np.stack([x, np.zeros((n, n, n)), np.zeros((n, n, n))])
    y = U.forward(_identity_params({8: -1.0}), feats, bf16=False)
    p1, p2, p3 = (_block_mean(x, k) for k in (1, 2, 3))
    x2 = np.maximum(p2 - _spread(p3, 1), 0.0)
    assert (p2 - _spread(p3, 1) < 0).any() and (p2 - _spread(p3, 1) > 0).any()
    ref = x + _spread(p1 + _spread(x2, 1), 1)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13)


def test_first_relu_clamps_negative_input_and_output_bias_adds():
    rng = np.random.default_rng(9)
    n = 8
    x = rng.standard_normal((n, n, n))
    feats = np.stack([x, np.zeros((n, n, n)), np.zeros((n, n, n))])
    p = _identity_params()
    p[-U.SPEC[-1][2]] = 0.25                    # bias of output channel 0 of the last layer
    y = U.forward(p, feats, bf16=False)
    xp = np.maximum(x, 0.0)
    ref = xp + sum(_spread(_block_mean(xp, k), k) for k in (1, 2, 3)) + 0.25
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13)
