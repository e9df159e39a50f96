"""Pins of the FP64 network-layer oracle (learned warm start): exact
special cases and identities that a transposed operand, a flipped tap or a
wrong index would break.  CPU only."""
import numpy as np

import oracle


def rng(seed):
    return np.random.default_rng(seed)


def test_conv3_delta_and_shift_kernels():
    """Centre-tap identity reproduces the input; a single off-centre tap
    (tz, ty, tx) reads the input at offset (tz-1, ty-1, tx-1) with zero fill."""
    x = rng(1).standard_normal((5, 6, 7, 3))
    w = np.zeros((27, 3, 3))
    w[13] = np.eye(3)
    assert np.array_equal(oracle.conv3(x, w), x)
    w = np.zeros((27, 3, 2))
    t = (2 * 3 + 0) * 3 + 1          # tz = 2, ty = 0, tx = 1
    w[t, 1, 0] = 1.0
    out = oracle.conv3(x, w)
    ref = np.zeros((5, 6, 7))
    ref[:-1, 1:, :] = x[1:, :-1, :, 1]
    assert np.array_equal(out[..., 0], ref)
    assert not out[..., 1].any()


def test_conv3_bias_and_constant_interior():
    x = np.full((6, 6, 6, 2), 0.5)
    w = rng(2).standard_normal((27, 2, 4))
    b = rng(3).standard_normal(4)
    out = oracle.conv3(x, w, b)
    ref = b + 0.5 * w.sum(axis=(0, 1))
    assert np.allclose(out[1:-1, 1:-1, 1:-1], ref, atol=1e-13)


def test_conv3_transpose_is_adjoint():
    x = rng(4).standard_normal((4, 5, 6, 3))
    y = rng(5).standard_normal((4, 5, 6, 5))
    w = rng(6).standard_normal((27, 3, 5))
    lhs = np.sum(oracle.conv3(x, w) * y)
    rhs = np.sum(x * oracle.conv3_t(y, w))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_conv3_weight_gradient_matches_finite_difference():
    """<conv3(x; w, b), y> is linear in (w, b): its directional derivative
    equals the central difference exactly up to round-off."""
    x = rng(7).standard_normal((4, 4, 5, 2))
    y = rng(8).standard_normal((4, 4, 5, 3))
    w = rng(9).standard_normal((27, 2, 3))
    b = rng(10).standard_normal(3)
    gw, gb = oracle.conv3_dw(x, y)
    dw = rng(11).standard_normal(w.shape)
    db = rng(12).standard_normal(b.shape)
    eps = 1e-3
    f = lambda ww, bb: np.sum(oracle.conv3(x, ww, bb) * y)
    fd = (f(w + eps * dw, b + eps * db) - f(w - eps * dw, b - eps * db)) / (2 * eps)
    assert abs(fd - (np.sum(gw * dw) + np.sum(gb * db))) < 1e-9 * abs(fd)


def test_pool_upsample_head_lrelu():
    z, y, x = np.meshgrid(np.arange(4.0), np.arange(6.0), np.arange(8.0), indexing="ij")
    f = (1.0 + 2 * z - 3 * y + 0.5 * x)[..., None]
    p = oracle.pool2(f)
    zc, yc, xc = np.meshgrid(np.arange(2.0), np.arange(3.0), np.arange(4.0), indexing="ij")
    assert np.allclose(p[..., 0], 1.0 + 2 * (2 * zc + 0.5) - 3 * (2 * yc + 0.5) + 0.5 * (2 * xc + 0.5))
    a = rng(13).standard_normal((2, 3, 4, 2))
    b = rng(14).standard_normal((4, 6, 8, 3))
    u = oracle.up2cat(a, b)
    assert np.array_equal(u[..., 2:], b)
    assert np.array_equal(u[1::2, 0::2, 1::2, :2], a)
    hw = rng(15).standard_normal((3, 2))
    hb = rng(16).standard_normal(2)
    assert np.allclose(oracle.head(b, hw, hb), b @ hw + hb)
    v = np.array([-2.0, -0.0, 0.0, 3.0])
    assert np.array_equal(oracle.lrelu(v, 0.2), np.array([-0.4, 0.0, 0.0, 3.0]))


def test_reference_network_gradient_matches_finite_difference():
    """The composed FP64 network (forward + hand-written backward through
    every layer: conv, LeakyReLU, pooling, upsample-concat, head, MSE) has a
    parameter gradient equal to central differences of its loss."""
    from oracle.net_oracle import RefNet, init_params
    n = 8
    p = init_params(3, scale_head=0.5)
    r = rng(21)
    m0, m1 = r.random((n, n, n)), r.random((n, n, n))
    label = 0.1 * r.standard_normal((3, n, n, n))
    L, g = RefNet(p).loss_grad(m0, m1, label)
    for k in range(3):
        d = rng(30 + k).standard_normal(p.size)
        eps = 1e-8          # small enough that no LeakyReLU kink is crossed
        Lp = RefNet(p + eps * d).loss_grad(m0, m1, label)[0]
        Lm = RefNet(p - eps * d).loss_grad(m0, m1, label)[0]
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g @ d) < 1e-6 * max(1.0, abs(fd)), (fd, g @ d)


def test_bf16_round_is_nearest_even():
    from oracle.net_oracle import bf16_round
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 -> ties to even (1.0)
    assert bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert bf16_round(np.array([-2.5]))[0] == -2.5
