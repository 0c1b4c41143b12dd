"""Pins for the CNN oracle: scipy's correlate on single channels, a delta
kernel that shifts, finite differences of the loss, and Adam's first step."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import cnn

RNG = np.random.default_rng(21)


def test_conv_matches_scipy_correlate():
    x = RNG.standard_normal((5, 6, 7, 1))
    W = RNG.standard_normal((27, 1, 1))
    y = cnn.conv3d(x, W, np.zeros(1))
    kern = np.zeros((3, 3, 3))
    for k, (dx, dy, dz) in enumerate(cnn.offsets()):
        kern[dz + 1, dy + 1, dx + 1] = W[k, 0, 0]
    ref = correlate(x[..., 0], kern, mode="same", method="direct")
    assert np.allclose(y[..., 0], ref, atol=1e-13)


def test_delta_kernel_is_a_shift_and_channels_mix_linearly():
    x = RNG.standard_normal((4, 4, 4, 3))
    W = np.zeros((27, 3, 2))
    k = cnn.offsets().index((1, 0, -1))
    M = RNG.standard_normal((3, 2))
    W[k] = M
    y = cnn.conv3d(x, W, np.array([0.5, -1.0]))
    ref = np.zeros((4, 4, 4, 2)) + np.array([0.5, -1.0])
    ref[1:, :, :3] += x[:3, :, 1:] @ M          # y[z, y, x] = x[z - 1, y, x + 1] M
    assert np.allclose(y, ref, atol=1e-14)


def test_loss_gradients_finite_differences():
    params = cnn.init_params(3, channels=(8, 4, 4))
    x = RNG.standard_normal((5, 5, 5, 8))
    target = RNG.standard_normal((5, 5, 5, 4))
    win = (slice(1, 4), slice(1, 4), slice(1, 4))
    loss, grads = cnn.loss_and_grads(params, x, target, win)
    eps = 1e-6
    for l, (W, b) in enumerate(params):
        for idx in [(0, 0, 0), (13, 5, 2), (26, 7, 3)]:
            if idx[1] >= W.shape[1]:
                continue
            Wp = [(w.copy(), bb.copy()) for w, bb in params]
            Wm = [(w.copy(), bb.copy()) for w, bb in params]
            Wp[l][0][idx] += eps
            Wm[l][0][idx] -= eps
            fd = (cnn.loss_and_grads(Wp, x, target, win)[0] - cnn.loss_and_grads(Wm, x, target, win)[0]) / (2 * eps)
            assert grads[l][0][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
        Bp = [(w.copy(), bb.copy()) for w, bb in params]
        Bm = [(w.copy(), bb.copy()) for w, bb in params]
        Bp[l][1][1] += eps
        Bm[l][1][1] -= eps
        fd = (cnn.loss_and_grads(Bp, x, target, win)[0] - cnn.loss_and_grads(Bm, x, target, win)[0]) / (2 * eps)
        assert grads[l][1][1] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_input_gradient_finite_differences():
    W = RNG.standard_normal((27, 2, 3))
    x = RNG.standard_normal((4, 5, 6, 2))
    dy = RNG.standard_normal((4, 5, 6, 3))
    dx, dW, db = cnn.conv3d_backward(x, W, dy)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (2, 3, 4, 1), (3, 4, 5, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (np.sum(dy * cnn.conv3d(xp, W, np.zeros(3))) - np.sum(dy * cnn.conv3d(xm, W, np.zeros(3)))) / (2 * eps)
        assert dx[idx] == pytest.approx(fd, rel=1e-7)
    assert np.allclose(db, dy.reshape(-1, 3).sum(0))


def test_parameter_count_of_the_proposal_network():
    params = cnn.init_params(0)
    assert sum(W.size + b.size for W, b in params) == 121124


def test_adam_first_step_moves_by_lr_times_sign():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -3.0, 1e-3])
    q, m, v = cnn.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 1e-2)
    assert np.allclose(q, p - 1e-2 * np.sign(g), atol=1e-7)


def test_bf16_round_pins():
    """Round-to-nearest-even on the bfloat16 grid (8 significand bits)."""
    from oracle import cnn
    # exact values stay; halfway cases go to the even neighbour
    assert cnn.bf16_round(np.array([1.0, 3.0, -2.5]))[0] == 1.0
    one_ulp = 2.0 ** -7                       # bf16 spacing in [1, 2)
    v = np.array([1.0 + one_ulp / 2, 1.0 + 1.5 * one_ulp, 1.0 + one_ulp / 4, 1.0 + 0.75 * one_ulp])
    assert np.array_equal(cnn.bf16_round(v), [1.0, 1.0 + 2 * one_ulp, 1.0, 1.0 + one_ulp])
    x = np.random.default_rng(0).standard_normal(1000)
    r = cnn.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-12))
