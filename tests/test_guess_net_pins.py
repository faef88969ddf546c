"""Pins of the guess-network oracle (CPU): BF16 rounding against torch's own
conversion, the convolution against scipy on the reflect-padded grid, adjoint
identities of padding and convolution, derivatives against central
differences, Adam against its closed form for a constant gradient, and the
algebra of features, targets and guesses."""
import numpy as np
import pytest

import synthetic as S
from oracle import guess_net as G


def rand_params(seed=3, bias=0.1):
    return S.net_init(seed=seed, zero_last=False, bias_scale=bias)


# ---------------------------------------------------------------- BF16
def test_bf16_matches_torch_round_to_nearest_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))).astype(np.float32)
    # exact ties: low 16 bits 0x8000 with odd and even upper halves
    ties = (rng.integers(0x3F000000, 0x41000000, 5000, dtype=np.uint32) & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32), -ties.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(G.bf16(x).view(np.uint32), ref.view(np.uint32))


def test_bf16_hand_cases():
    one = np.float32(1.0)
    # 7 fraction bits: ulp(1) = 2^-7; 1 + 2^-8 is a tie -> even (1.0)
    assert G.bf16(np.float32(1 + 2.0 ** -8)) == one
    # 1 + 2^-7 + 2^-8 is a tie between odd 1 + 2^-7 and even 1 + 2^-6
    assert G.bf16(np.float32(1 + 2.0 ** -7 + 2.0 ** -8)) == np.float32(1 + 2.0 ** -6)
    assert G.bf16(np.float32(1 + 2.0 ** -8 + 2.0 ** -20)) == np.float32(1 + 2.0 ** -7)
    assert G.bf16(np.float32(3.0)) == np.float32(3.0)


# ---------------------------------------------------------------- convolution
def test_conv_matches_scipy_correlation_on_reflected_grid():
    from scipy.signal import correlate2d
    rng = np.random.default_rng(1)
    a = rng.standard_normal((2, 7, 5, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    out = G.conv(a, w, b)
    for n in range(2):
        for o in range(4):
            ref = np.full((7, 5), b[o])
            for c in range(3):
                ref += correlate2d(np.pad(a[n, :, :, c], 1, mode="reflect"), w[:, :, c, o], mode="valid")
            assert np.allclose(out[n, :, :, o], ref, rtol=0, atol=1e-12)


def test_reflective_padding_mirrors_the_first_interior_line():
    a = np.arange(12.0).reshape(1, 3, 4, 1)
    p = G.pad_reflect(a)[0, :, :, 0]
    assert np.array_equal(p[0, 1:-1], a[0, 1, :, 0]) and np.array_equal(p[-1, 1:-1], a[0, 1, :, 0])
    assert np.array_equal(p[1:-1, 0], a[0, :, 1, 0]) and np.array_equal(p[1:-1, -1], a[0, :, 2, 0])
    assert p[0, 0] == a[0, 1, 1, 0]


@pytest.mark.parametrize("shape", [(1, 2, 2, 3), (2, 5, 4, 2), (1, 9, 3, 1)])
def test_fold_is_the_adjoint_of_pad(shape):
    rng = np.random.default_rng(2)
    a = rng.standard_normal(shape)
    g = rng.standard_normal((shape[0], shape[1] + 2, shape[2] + 2, shape[3]))
    assert np.isclose(np.vdot(G.pad_reflect(a), g), np.vdot(a, G.fold_reflect(g)), rtol=1e-13)


def test_conv_gradients_are_adjoints():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2, 6, 5, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    g = rng.standard_normal((2, 6, 5, 4))
    y = G.conv(a, w, np.zeros(4))
    dw, db = G.conv_grad_weights(a, g)
    assert np.isclose(np.vdot(y, g), np.vdot(a, G.conv_grad_input(g, w)), rtol=1e-12)
    assert np.isclose(np.vdot(y, g), np.vdot(w, dw), rtol=1e-12)
    assert np.allclose(db, g.sum(axis=(0, 1, 2)), rtol=1e-13)


def test_backward_matches_central_differences_fp64():
    rng = np.random.default_rng(5)
    params = [(w.astype(np.float64), b.astype(np.float64)) for w, b in rand_params()]
    feats = rng.standard_normal((2, 6, 7, 8))
    t = rng.standard_normal((2, 6, 7, 4))
    mask = np.ones((2, 6, 7))
    mask[:, :1, :] = 0

    def loss(ps):
        _, y = G.forward(ps, feats, quantize=False)
        return G.loss_and_grad_output(y, t, mask, [1.5, 0.5], quantize=False)[0]

    acts, y = G.forward(params, feats, quantize=False)
    _, gy = G.loss_and_grad_output(y, t, mask, [1.5, 0.5], quantize=False)
    grads = G.backward(params, acts, gy, quantize=False)
    h = 1e-6
    for k in range(4):
        for which in (0, 1):
            arr = params[k][which]
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(4)]:
                def bumped(delta):
                    ps = [(w.copy(), b.copy()) for w, b in params]
                    ps[k][which][idx] += delta
                    return loss(ps)
                fd = (bumped(h) - bumped(-h)) / (2 * h)
                an = grads[k][which][idx]
                assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)), (k, which, idx, fd, an)


def test_output_gradient_matches_central_differences():
    rng = np.random.default_rng(6)
    y = rng.standard_normal((1, 3, 4, 4))
    t = rng.standard_normal((1, 3, 4, 4))
    mask = rng.integers(0, 2, (1, 3, 4)).astype(float)
    mask[0, 0, 0] = 1
    # a constant error c on the masked pixels is a mean square of c^2
    assert np.isclose(G.loss_and_grad_output(t + 0.5, t, mask, quantize=False)[0], 0.25, rtol=1e-14)
    _, g = G.loss_and_grad_output(y, t, mask, quantize=False)
    for idx in [(0, 0, 0, 1), (0, 2, 3, 3), (0, 1, 2, 0)]:
        yp, ym = y.copy(), y.copy()
        yp[idx] += 1e-6
        ym[idx] -= 1e-6
        fd = (G.loss_and_grad_output(yp, t, mask, quantize=False)[0]
              - G.loss_and_grad_output(ym, t, mask, quantize=False)[0]) / 2e-6
        assert abs(fd - g[idx]) <= 1e-7


def test_weighted_loss_is_the_mean_of_per_sample_means():
    rng = np.random.default_rng(16)
    y = rng.standard_normal((3, 4, 5, 4))
    t = rng.standard_normal((3, 4, 5, 4))
    mask = np.ones((3, 4, 5))
    mask[1, :2] = 0
    mask[2, :, :4] = 0
    w = np.array([2.0, 0.5, 3.0])
    per = [float(np.sum(mask[s][..., None] * (y[s] - t[s]) ** 2) / (4 * mask[s].sum())) for s in range(3)]
    loss, g = G.loss_and_grad_output(y, t, mask, w, quantize=False)
    assert np.isclose(loss, np.dot(w, per) / 3, rtol=1e-13)
    # the pair penalty on a constant error is zero; on an error alternating in
    # sign along rows it adds smooth * (2c)^2 per masked horizontal pair
    c = 0.3
    assert np.isclose(G.loss_and_grad_output(t + c, t, mask, w, smooth=5.0, quantize=False)[0],
                      np.dot(w, [c * c] * 3) / 3, rtol=1e-13)
    alt = t + c * (-1.0) ** np.arange(5)[None, None, :, None]
    pairs = [float((mask[s][:, 1:] * mask[s][:, :-1]).sum()) for s in range(3)]
    ref = sum(w[s] * (4 * mask[s].sum() * c * c + 5.0 * 4 * pairs[s] * 4 * c * c) / (4 * mask[s].sum())
              for s in range(3)) / 3
    assert np.isclose(G.loss_and_grad_output(alt, t, mask, w, smooth=5.0, quantize=False)[0], ref,
                      rtol=1e-12)
    loss_s, g_s = G.loss_and_grad_output(y, t, mask, w, smooth=2.5, quantize=False)
    for idx in [(2, 1, 4, 2), (1, 3, 0, 1), (0, 0, 0, 0)]:
        yp, ym = y.copy(), y.copy()
        yp[idx] += 1e-6
        ym[idx] -= 1e-6
        fd = (G.loss_and_grad_output(yp, t, mask, w, 2.5, quantize=False)[0]
              - G.loss_and_grad_output(ym, t, mask, w, 2.5, quantize=False)[0]) / 2e-6
        assert abs(fd - g_s[idx]) <= 1e-7
    idx = (2, 1, 4, 2)
    yp, ym = y.copy(), y.copy()
    yp[idx] += 1e-6
    ym[idx] -= 1e-6
    fd = (G.loss_and_grad_output(yp, t, mask, w, quantize=False)[0]
          - G.loss_and_grad_output(ym, t, mask, w, quantize=False)[0]) / 2e-6
    assert abs(fd - g[idx]) <= 1e-7


def test_sample_weight_is_inverse_mean_square_target():
    x2, x1, x0 = states()
    _, sigma = G.features(x2, x1)
    t = G.target(x2, x1, x0, sigma).astype(np.float64)
    assert np.isclose(G.sample_weight(x2, x1, x0, sigma), 1.0 / (np.mean(t * t) + 1e-4), rtol=1e-6)
    # a pure linear extrapolation step has a zero target: the weight is the floor's inverse
    assert G.sample_weight(x2, x1, 2 * x1 - x2, sigma) == pytest.approx(1e4, rel=1e-9)


def test_quantized_forward_rounds_at_the_stated_boundaries():
    rng = np.random.default_rng(7)
    params = rand_params()
    feats = rng.standard_normal((1, 5, 6, 8)).astype(np.float32)
    acts, y = G.forward(params, feats)
    for a in acts:   # every stored activation is a BF16 value
        assert np.array_equal(G.bf16(a), a)
    assert y.dtype == np.float32
    # the first hidden layer by hand: BF16 weights, FP32 sum, bias, ReLU, BF16
    w, b = params[0]
    ref = G.bf16(np.maximum(G.conv(G.bf16(feats), G.bf16(w), b).astype(np.float32), 0))
    assert np.array_equal(acts[1], ref)


# ---------------------------------------------------------------- Adam
def test_adam_constant_gradient_closed_form():
    # constant g: m_hat = g and v_hat = g^2 at every step, so each step moves
    # w by lr * g / (|g| + eps)
    w0 = np.array([0.5, -1.0, 2.0], dtype=np.float32)
    g = np.array([0.3, -2e-3, 4.0], dtype=np.float32)
    params = [(w0.copy(),)]
    m = [(np.zeros(3, np.float32),)]
    v = [(np.zeros(3, np.float32),)]
    lr = 1e-2
    for t in range(1, 6):
        params, m, v = G.adam(params, [(g,)], m, v, t, lr)
    expect = w0.astype(np.float64) - 5 * lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(params[0][0], expect, rtol=2e-6, atol=1e-7)
    assert np.allclose(m[0][0], g * (1 - 0.9 ** 5), rtol=1e-5)
    # 1 - beta2 in FP32 is 0.0010000467: 5e-5 relative from 1e-3
    assert np.allclose(v[0][0], g * g * (1 - 0.999 ** 5), rtol=1e-4)


# ---------------------------------------------------------------- features, guesses
def states(seed=8, H=6, W=7):
    rng = np.random.default_rng(seed)
    x2 = rng.standard_normal((4, H, W))
    x1 = x2 + 1e-3 * rng.standard_normal((4, H, W))
    x0 = x1 + 1e-3 * rng.standard_normal((4, H, W))
    return x2, x1, x0


def test_zero_last_layer_gives_linear_extrapolation():
    x2, x1, _ = states()
    feats, sigma = G.features(x2, x1)
    _, y = G.forward(S.net_init(zero_last=True), feats[None])
    assert np.array_equal(G.guess(x2, x1, y[0], sigma), x1 + (x1 - x2))


def test_target_and_guess_invert_each_other():
    x2, x1, x0 = states()
    _, sigma = G.features(x2, x1)
    t = G.target(x2, x1, x0, sigma).astype(np.float64)
    assert np.allclose(G.guess(x2, x1, t, sigma), x0, rtol=0, atol=1e-9)


def test_features_are_scale_free_in_the_increment_and_the_state():
    x2, x1, _ = states()
    f, s = G.features(x2, x1, quantize=False)
    c = np.array([3.0, 0.5, 7.0, 2.0])[:, None, None]
    f2, s2 = G.features(x1 - c * (x1 - x2), x1, quantize=False)
    assert np.allclose(f2, f, atol=1e-12) and np.allclose(s2, s * c[:, 0, 0], rtol=1e-12)
    f3, _ = G.features(5 * x2 + 1, 5 * x1 + 1, quantize=False)
    assert np.allclose(f3, f, atol=1e-12)
    assert np.allclose(np.sqrt(np.mean(f ** 2, axis=(0, 1))), 1.0)
    zero, sz = G.features(x1, x1)
    assert np.all(zero[..., :4] == 0) and np.all(sz == 0)


def test_crop_interior_equals_full_grid():
    rng = np.random.default_rng(9)
    params = rand_params()
    feats = rng.standard_normal((1, 20, 23, 8))
    _, yf = G.forward(params, feats, quantize=False)
    oy, ox, h, w = 3, 5, 12, 14
    _, yc = G.forward(params, feats[:, oy:oy + h, ox:ox + w], quantize=False)
    m = G.crop_mask(20, 23, oy, ox, h, w).astype(bool)
    assert m.sum() == (h - 8) * (w - 8)
    assert np.allclose(yc[0][m], yf[0, oy:oy + h, ox:ox + w][m], rtol=0, atol=1e-12)
    # a crop at the domain corner keeps its outer rows and columns
    m2 = G.crop_mask(20, 23, 0, 0, 12, 14)
    assert m2[0, 0] == 1 and m2[-1, -1] == 0 and m2.sum() == 8 * 10
    _, yc2 = G.forward(params, feats[:, :12, :14], quantize=False)
    assert np.allclose(yc2[0][m2.astype(bool)], yf[0, :12, :14][m2.astype(bool)], atol=1e-12)
