"""Pins of the CPU reference U-Net: hand-written backward against central
finite differences in FP64 (mini-net), layer identities, and Adam."""
import numpy as np
import pytest

from oracle import unet as U


def _mini(seed=0):
    ch = (8, 16)
    cin = 5
    theta = U.init_params(ch, seed, cin=cin, dtype=np.float64)
    rng = np.random.default_rng(seed + 1)
    x = rng.standard_normal((16, 16, cin))
    target = rng.standard_normal((16, 16))
    mask = rng.uniform(size=(16, 16)) > 0.2
    return ch, cin, theta, x, target, mask


def _loss(theta, ch, cin, x, target, mask):
    out, _ = U.forward(theta, x, ch, cin)
    return U.loss_and_grad_out(out, target, mask)[0]


def test_backward_matches_finite_differences():
    ch, cin, theta, x, target, mask = _mini()
    out, cache = U.forward(theta, x, ch, cin)
    loss, dout = U.loss_and_grad_out(out, target, mask)
    g = U.backward(theta, cache, dout, ch, cin)
    assert g.shape == theta.shape
    rng = np.random.default_rng(7)
    idx = rng.choice(len(theta), 60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (_loss(tp, ch, cin, x, target, mask) - _loss(tm, ch, cin, x, target, mask)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9)
    # directional derivative over all parameters at once
    d = rng.standard_normal(len(theta))
    fd = (_loss(theta + h * d, ch, cin, x, target, mask) - _loss(theta - h * d, ch, cin, x, target, mask)) / (2 * h)
    assert fd == pytest.approx(g @ d, rel=1e-6)


def test_layer_identities():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((8, 8, 3))
    # identity kernel (centre tap) reproduces the input
    W = np.zeros((9, 3, 3))
    W[4] = np.eye(3)
    assert np.allclose(U.conv3x3(x, W, np.zeros(3)), x)
    # a shift kernel moves the image by one pixel with zero fill
    W = np.zeros((9, 3, 3))
    W[5] = np.eye(3)               # offset (+1, 0): out[y, x] = in[y, x+1]
    y = U.conv3x3(x, W, np.zeros(3))
    assert np.allclose(y[:, :-1], x[:, 1:]) and np.allclose(y[:, -1], 0)
    # pooling is the adjoint of (upsampling / 4)
    a = rng.standard_normal((8, 8, 2))
    b = rng.standard_normal((4, 4, 2))
    assert np.sum(U.pool2(a) * b) == pytest.approx(np.sum(a * U.up2(b) / 4))
    assert np.allclose(U.pool2_backward(b), U.up2(b) / 4)


def test_zero_head_predicts_no_correction():
    """The head output is the correction to the warm start: a zero head gives 0."""
    ch = (16, 32)
    theta = U.init_params(ch, 0)
    P = U.unpack(theta, ch)
    P["head"][0][:] = 0.0
    rng = np.random.default_rng(0)
    x = rng.standard_normal((16, 16, U.IN_CHANNELS)).astype(np.float32)
    out, _ = U.forward(theta, x, ch)
    assert np.all(out == 0.0)


def test_pack_input_scales_each_field_by_its_own_rms():
    rng = np.random.default_rng(4)
    n = (8, 4)
    role = np.full(32, -1, dtype=np.int8)
    role[:3] = 0
    role[3:5] = 2
    role[5:8] = 1
    unknown = (role == -1) | (role == 2)
    r = rng.standard_normal(32) * 1e3
    p = rng.standard_normal(32) * 1e-2
    x, rr = U.pack_input(r, p, role, unknown, n)
    assert x.shape == (4, 8, U.IN_CHANNELS)
    c0 = x[:, :, 0].reshape(-1)[unknown]
    c1 = x[:, :, 1].reshape(-1)[unknown]
    assert np.sqrt(np.mean(c0 ** 2)) == pytest.approx(1.0) and np.sqrt(np.mean(c1 ** 2)) == pytest.approx(1.0)
    assert rr == pytest.approx(np.sqrt(np.mean(r[unknown] ** 2)))
    assert np.all(x[:, :, :2].reshape(-1, 2)[~unknown] == 0.0)
    assert np.array_equal(x[:, :, 2].reshape(-1), (role == -1).astype(float))
    assert np.array_equal(x[:, :, 3].reshape(-1), (role == 2).astype(float))
    assert np.array_equal(x[:, :, 4].reshape(-1), (role == 1).astype(float))
    # the correction target undoes the guess formula p_prev + s rms(r) h
    pt = p + 0.3 * rng.standard_normal(32)
    t = U.correction_target(pt, p, rr, 2.5, n).reshape(-1)
    assert np.allclose(p + 2.5 * rr * t, pt)


def test_adam_first_step_moves_by_lr():
    theta = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    t, m, v = U.adam_update(theta, np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    assert np.allclose(t[:3], -0.01 * np.sign(g[:3]), rtol=1e-6) and t[3] == 0.0


# ---------------------------------------------------------------------------
# 3D network (27-tap convolutions, 2x2x2 pooling), same code path
# ---------------------------------------------------------------------------

def test_backward_matches_finite_differences_3d():
    ch, cin = (8, 16), 5
    theta = U.init_params(ch, 3, cin=cin, dtype=np.float64, dim=3)
    assert len(theta) == U.n_params(ch, cin, dim=3) == sum(27 * a * b + b for _, a, b in U.layer_shapes(ch, cin))
    rng = np.random.default_rng(8)
    x = rng.standard_normal((4, 8, 6, cin))          # (z, y, x): unequal axes catch transpositions
    target = rng.standard_normal((4, 8, 6))
    mask = rng.uniform(size=(4, 8, 6)) > 0.2
    out, cache = U.forward(theta, x, ch, cin)
    assert out.shape == (4, 8, 6)
    loss, dout = U.loss_and_grad_out(out, target, mask)
    g = U.backward(theta, cache, dout, ch, cin)

    def f(th):
        return U.loss_and_grad_out(U.forward(th, x, ch, cin)[0], target, mask)[0]

    h = 1e-6
    for i in rng.choice(len(theta), 40, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        assert (f(tp) - f(tm)) / (2 * h) == pytest.approx(g[i], rel=1e-5, abs=1e-9)
    d = rng.standard_normal(len(theta))
    assert (f(theta + h * d) - f(theta - h * d)) / (2 * h) == pytest.approx(g @ d, rel=1e-6)


def test_3d_conv_of_a_z_constant_image_is_the_2d_conv():
    """With an input constant along z, an interior plane of the 27-tap
    convolution is the 9-tap convolution with the three z-planes of taps
    summed; the first plane sees only the taps dz = 0, +1 (zero padding)."""
    rng = np.random.default_rng(5)
    x2 = rng.standard_normal((7, 5, 3))
    x3 = np.repeat(x2[None], 6, axis=0)
    W3 = rng.standard_normal((27, 3, 4))
    b = rng.standard_normal(4)
    y3 = U.conv3x3(x3, W3, b)
    W2_all = W3[0:9] + W3[9:18] + W3[18:27]
    for z in range(1, 5):
        assert np.allclose(y3[z], U.conv3x3(x2, W2_all, b))
    assert np.allclose(y3[0], U.conv3x3(x2, W3[9:18] + W3[18:27], b))
    assert np.allclose(y3[5], U.conv3x3(x2, W3[0:9] + W3[9:18], b))
    # the centre tap alone is the identity map
    W = np.zeros((27, 3, 3))
    W[13] = np.eye(3)
    assert np.allclose(U.conv3x3(x3, W, np.zeros(3)), x3)
    # tap 22 = (dz, dy, dx) = (2, 1, 1): out[z] = in[z + 1]
    W = np.zeros((27, 3, 3))
    W[22] = np.eye(3)
    xr = rng.standard_normal((4, 3, 3, 3))
    y = U.conv3x3(xr, W, np.zeros(3))
    assert np.allclose(y[:-1], xr[1:]) and np.allclose(y[-1], 0)


def test_3d_pool_and_upsample():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((4, 6, 8, 2))
    b = rng.standard_normal((2, 3, 4, 2))
    assert np.sum(U.pool2(a) * b) == pytest.approx(np.sum(a * U.up2(b) / 8))
    assert np.allclose(U.pool2(U.up2(b)), b)
    assert U.pool2(a)[1, 2, 3, 1] == pytest.approx(a[2:4, 4:6, 6:8, 1].mean())
    assert np.allclose(U.up2_backward(U.up2(b)), 8 * b)
