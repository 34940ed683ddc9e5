"""Pins of the seed-network oracle: convolution against scipy's correlate2d,
identity kernels, strides as subsampling, gradients against central finite
differences, the loss gradient, Adam's first step, bfloat16 rounding, and
the seeded key-frame fit on constructed tiles."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import seednet as sn


def test_param_count():
    assert sn.n_params() == 15552 + 84


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 9, 13))
    W = rng.normal(size=(1, 1, 3, 3))
    out = sn.conv2d(x, W, np.zeros(1), (1, 1))
    ref = correlate2d(x[0], W[0, 0], mode="same", boundary="fill", fillvalue=0.0)
    assert np.allclose(out[0], ref, rtol=0, atol=1e-12)


def test_conv_multichannel_is_sum_of_correlations():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 7, 10))
    W = rng.normal(size=(2, 3, 3, 3))
    b = rng.normal(size=2)
    out = sn.conv2d(x, W, b, (1, 1))
    for o in range(2):
        ref = b[o] + sum(correlate2d(x[c], W[o, c], mode="same") for c in range(3))
        assert np.allclose(out[o], ref, atol=1e-12)


@pytest.mark.parametrize("stride", [(2, 2), (1, 2), (2, 1)])
def test_strided_conv_is_subsampled(stride):
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 8, 12))
    W = rng.normal(size=(3, 2, 3, 3))
    full = sn.conv2d(x, W, np.zeros(3), (1, 1))
    st = sn.conv2d(x, W, np.zeros(3), stride)
    assert np.allclose(st, full[:, ::stride[0], ::stride[1]], atol=1e-12)


def test_identity_kernel():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(4, 6, 8))
    W = np.zeros((4, 4, 3, 3))
    for c in range(4):
        W[c, c, 1, 1] = 1.0
    assert np.allclose(sn.conv2d(x, W, np.zeros(4), (1, 1)), x, atol=0)


def test_output_grid_matches_4x8_tiles():
    p = sn.init_params(0)
    x0 = np.zeros((4, 64, 256), np.float32)
    out, _ = sn.forward(p, x0)
    assert out.shape == (4, 16, 32)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 1e-3], np.float32)
    r = sn.bf16(vals)
    # ties to even at the 8-bit mantissa boundary, exact values unchanged
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0 + 2 ** -7)
    assert r[3] == np.float32(1.0 + 2 ** -6) and r[4] == -2.5
    assert abs(r[5] - 1e-3) <= 1e-3 * 2 ** -8


def _fd_check(f, x, idx, h=1e-6):
    g = np.zeros(len(idx))
    for q, i in enumerate(idx):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        g[q] = (f(xp) - f(xm)) / (2 * h)
    return g


def test_backward_against_finite_differences():
    rng = np.random.default_rng(5)
    p = rng.normal(0, 0.3, sn.n_params())
    x0 = rng.normal(size=(4, 8, 16))
    dout = rng.normal(size=(4, 2, 2))

    def f(pp):
        out, _ = sn.forward(pp, x0, rounding=False)
        return float((out * dout).sum())
    out, cache = sn.forward(p, x0, rounding=False)
    g = sn.backward(p, cache, dout)
    idx = rng.choice(sn.n_params(), 60, replace=False)
    idx = np.concatenate([idx, np.arange(sn.n_params() - 84, sn.n_params())[:20]])   # some biases
    fd = _fd_check(f, p.astype(np.float64), idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-7)


def test_loss_gradient_against_finite_differences():
    rng = np.random.default_rng(6)
    s = rng.normal(size=(4, 3, 5))
    planar = (rng.random((3, 5)) < 0.6).astype(float)
    nrm = rng.normal(size=(3, 5, 3))
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    valid = (rng.random((3, 5)) < 0.8).astype(float)
    L, g = sn.loss(s, planar, nrm, valid)
    fd = _fd_check(lambda v: sn.loss(v.reshape(s.shape), planar, nrm, valid)[0], s.ravel().copy(),
                   np.arange(s.size))
    assert np.allclose(g.ravel(), fd, rtol=1e-5, atol=1e-8)


def test_loss_special_cases():
    s = np.zeros((4, 1, 1))
    s[:3, 0, 0] = [0, 0, 2.0]
    nrm = np.zeros((1, 1, 3))
    nrm[0, 0] = [0, 0, -1.0]
    # normal sign does not matter; logit 0 costs log 2
    L, _ = sn.loss(s, np.ones((1, 1)), nrm, np.ones((1, 1)))
    assert abs(L - np.log(2.0)) < 1e-12


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = sn.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-4)


def test_adam_steps_two_and_three_hand_worked():
    """Gradients g, -g, g (Kingma and Ba's update, beta1 0.9, beta2 0.999),
    worked by hand.  Second moments: v_t = (1 - beta2^t) g^2 whatever the
    signs, so the bias-corrected v is g^2 at every step.  First moments:
    m1 = 0.1 g; m2 = 0.09 g - 0.1 g = -0.01 g, corrected by 1 - 0.81 = 0.19
    to -g/19; m3 = -0.009 g + 0.1 g = 0.091 g, corrected by 1 - 0.729 = 0.271
    to (91/271) g.  So the steps are -lr sign(g), +lr sign(g)/19 and
    -lr (91/271) sign(g), for any |g| well above the epsilon 1e-8.  A wrong
    beta in either moment, a missing bias correction or swapped betas moves
    the second or third step."""
    lr = 0.01
    g = np.array([3.0, -0.5, 1e-3, 250.0])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    want = np.zeros(4)
    for t, (sg, step) in enumerate(((1, -1.0), (-1, 1.0 / 19.0), (1, -91.0 / 271.0)), start=1):
        p, m, v = sn.adam(p, sg * g, m, v, t, lr=lr)
        want = want + lr * step * np.sign(g)
        assert np.allclose(p, want, rtol=1e-4, atol=0), (t, p, want)
    # constant gradients: every bias-corrected step is lr sign(g)
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 6):
        p, m, v = sn.adam(p, g, m, v, t, lr=lr)
        assert np.allclose(p, -lr * t * np.sign(g), rtol=1e-4, atol=0), t


def test_labels_from_stored_planes():
    # ground plane z = -1.7 stored on axis 2 with a = b = 0
    planar, n, valid = sn.labels_from_tiles(np.array([5, 3, 0]), np.array([2, 0, 0]),
                                            np.array([[0, 0, -1.7], [0.5, 0, 1], [0, 0, 0]]))
    assert list(planar) == [1, 0, 0] and list(valid) == [1, 1, 0]
    assert np.allclose(n[0], [0, 0, 1])
    assert np.allclose(n[1], np.array([1, 0.5, 0]) / np.linalg.norm([1, 0.5, 0]))


def _plane_tile_range(tb, tr, tc, th, tw, normal, c):
    d = tb.directions()[tr * th:(tr + 1) * th, tc * tw:(tc + 1) * tw].astype(np.float64)
    t = c / (d @ np.asarray(normal, np.float64))
    return t.astype(np.float32)


def test_seeded_fit_accepts_good_seed_and_falls_back_on_bad(orc):
    """A noiseless ground tile: a seed near the true normal is accepted after one
    refit; a wrong seed falls back to the plain fit, which is accepted too."""
    from paper_2008_06972_amd import synth
    s = synth.SENSORS["c1"]
    tb = orc.Tables.of(s)
    prm = orc.Params(eps=0.02, th=4, tw=4)
    rng = np.zeros((s.H, s.W), np.float32)
    tr, tc = 3, 40
    rng[tr * 4:(tr + 1) * 4, tc * 4:(tc + 1) * 4] = _plane_tile_range(tb, tr, tc, 4, 4, [0, 0, 1.0], -1.7)
    T = (s.H // 4) * (s.W // 4)
    t = tr * (s.W // 4) + tc
    plain = orc.encode_key(rng, tb, prm)
    seed = np.zeros((T, 4), np.float32)
    seed[t] = [0.0005, -0.001, 1.0, 3.0]     # within a milliradian of the true normal
    good = orc.encode_key(rng, tb, prm, seed)
    assert good.seeded[t] == 1 and good.own_status[t] == orc.ACCEPTED and good.own_iters[t] == 1
    assert good.own_axis[t] == plain.own_axis[t] == 2
    assert np.allclose(good.own_abc[t], plain.own_abc[t], atol=1e-5)
    seed[t] = [1.0, 0.0, 0.05, 3.0]          # a wall normal on the ground: nothing reproduced
    bad = orc.encode_key(rng, tb, prm, seed)
    assert bad.seeded[t] == 2 and bad.own_status[t] == orc.ACCEPTED
    assert np.array_equal(bad.own_abc[t], plain.own_abc[t])
    seed[t] = [0.0, 0.0, 1.0, -1.0]          # negative logit: no seed
    off = orc.encode_key(rng, tb, prm, seed)
    assert off.seeded[t] == 0 and np.array_equal(off.own_abc[t], plain.own_abc[t])
    assert off.size_bytes == plain.size_bytes
