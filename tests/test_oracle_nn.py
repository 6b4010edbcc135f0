"""Pins of the oracle's network reference (convolution, its gradients, pooling,
rounding, Adam) against facts that do not depend on its code."""
import numpy as np

from oracle import nn

RNG = np.random.default_rng(21)


def test_bf16_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                       # bfloat16 spacing on [1, 2)
    assert nn.bf16_round(one) == one
    assert nn.bf16_round(one + ulp / 2) == one                 # tie -> even (mantissa 0)
    assert nn.bf16_round(one + 3 * ulp / 2) == one + 2 * ulp   # tie -> even (mantissa 2)
    assert nn.bf16_round(one + 0.6 * ulp) == one + ulp
    assert nn.bf16_round(-3.0) == -3.0
    x = RNG.standard_normal(1000)
    r = nn.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-6))


def test_one_tap_convolution_is_a_matrix_product():
    X = RNG.standard_normal((3, 4, 5, 6))
    W = RNG.standard_normal((1, 7, 6))
    Y = nn.conv3d(X, W, round_inputs=False)
    assert np.allclose(Y, np.einsum("dhwi,oi->dhwo", X, W[0]), atol=1e-13)


def test_delta_kernel_is_a_zero_padded_shift():
    X = RNG.standard_normal((4, 5, 6, 2))
    for ti, (dz, dy, dx) in enumerate(nn.TAPS):
        W = np.zeros((27, 2, 2))
        W[ti] = np.eye(2)
        Y = nn.conv3d(X, W, round_inputs=False)
        for z in range(4):
            for y in range(5):
                for x in range(6):
                    zz, yy, xx = z + dz, y + dy, x + dx
                    inside = 0 <= zz < 4 and 0 <= yy < 5 and 0 <= xx < 6
                    want = X[zz, yy, xx] if inside else np.zeros(2)
                    assert np.array_equal(Y[z, y, x], want)


def test_gradients_are_adjoints():
    X = RNG.standard_normal((4, 3, 5, 3))
    W = RNG.standard_normal((27, 4, 3))
    dY = RNG.standard_normal((4, 3, 5, 4))
    Y = nn.conv3d(X, W, round_inputs=False)
    dX = nn.conv3d_dgrad(dY, W, round_inputs=False)
    dW = nn.conv3d_wgrad(X, dY, round_inputs=False)
    assert abs(np.sum(Y * dY) - np.sum(X * dX)) < 1e-10 * np.abs(Y * dY).sum()
    assert abs(np.sum(Y * dY) - np.sum(W * dW)) < 1e-10 * np.abs(Y * dY).sum()


def test_gradients_match_central_differences():
    X = RNG.standard_normal((3, 3, 4, 2))
    W = RNG.standard_normal((27, 3, 2))
    T = RNG.standard_normal((3, 3, 4, 3))

    def loss(X_, W_):
        return 0.5 * np.sum((nn.conv3d(X_, W_, relu=True, round_inputs=False) - T) ** 2)

    Y = nn.conv3d(X, W, relu=True, round_inputs=False)
    dY = (Y - T) * (Y > 0)
    dX = nn.conv3d_dgrad(dY, W, round_inputs=False)
    dW = nn.conv3d_wgrad(X, dY, round_inputs=False)
    eps = 1e-6
    for _ in range(10):
        idx = tuple(RNG.integers(0, s) for s in X.shape)
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += eps
        Xm[idx] -= eps
        fd = (loss(Xp, W) - loss(Xm, W)) / (2 * eps)
        assert abs(fd - dX[idx]) < 1e-6 * max(1, abs(fd))
        jdx = tuple(RNG.integers(0, s) for s in W.shape)
        Wp, Wm = W.copy(), W.copy()
        Wp[jdx] += eps
        Wm[jdx] -= eps
        fd = (loss(X, Wp) - loss(X, Wm)) / (2 * eps)
        assert abs(fd - dW[jdx]) < 1e-6 * max(1, abs(fd))


def test_pool_and_upsample_adjoints():
    X = RNG.standard_normal((4, 6, 8, 3))
    Yp = RNG.standard_normal((2, 3, 4, 3))
    assert abs(np.sum(nn.avgpool2(X) * Yp) - np.sum(X * nn.avgpool2_grad(Yp))) < 1e-12
    Xs = RNG.standard_normal((2, 3, 4, 3))
    Yu = RNG.standard_normal((4, 6, 8, 3))
    assert abs(np.sum(nn.upsample2(Xs) * Yu) - np.sum(Xs * nn.upsample2_grad(Yu))) < 1e-12
    assert np.allclose(nn.avgpool2(nn.upsample2(Xs)), Xs)


def test_adam_first_step_is_a_sign_step():
    w = RNG.standard_normal(20)
    g = RNG.standard_normal(20)
    w1, m, v = nn.adam_step(w, g, np.zeros(20), np.zeros(20), 1, lr=1e-3)
    assert np.allclose(w1, w - 1e-3 * np.sign(g), atol=1e-9)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the moments are m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected moments equal g and g^2 at every step t
    and each step moves w by exactly lr g / (|g| + eps) (Kingma & Ba, Algorithm 1).
    A bias-correction exponent off by one fails here from the second step on."""
    w0 = RNG.standard_normal(16)
    g = RNG.standard_normal(16) * 10.0 ** RNG.uniform(-3, 2, 16)
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    w, m, v = w0.copy(), np.zeros(16), np.zeros(16)
    for t in range(1, 41):
        w, m, v = nn.adam_step(w, g, m, v, t, lr, b1, b2, eps)
        assert np.allclose(m, (1 - b1 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12, atol=0)
        want = w0 - t * lr * g / (np.abs(g) + eps)
        assert np.allclose(w, want, rtol=0, atol=1e-12 * t), t


def test_adam_two_gradients_closed_form():
    """Two steps with gradients g1 then g2: m_2 = b1 (1 - b1) g1 + (1 - b1) g2 and
    v_2 = b2 (1 - b2) g1^2 + (1 - b2) g2^2, corrected by 1 - b1^2 and 1 - b2^2."""
    w0 = RNG.standard_normal(8)
    g1, g2 = RNG.standard_normal(8), RNG.standard_normal(8)
    lr, b1, b2, eps = 1e-2, 0.8, 0.99, 1e-8
    w1, m, v = nn.adam_step(w0, g1, np.zeros(8), np.zeros(8), 1, lr, b1, b2, eps)
    w2, m, v = nn.adam_step(w1, g2, m, v, 2, lr, b1, b2, eps)
    m2 = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    v2 = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    want = w0 - lr * g1 / (np.abs(g1) + eps) - lr * m2 / (np.sqrt(v2) + eps)
    assert np.allclose(w2, want, rtol=0, atol=1e-13)


def _unet_case(seed, n=(8, 8, 8)):
    rng = np.random.default_rng(seed)
    flat = np.concatenate([rng.standard_normal(t * ci * co) * np.sqrt(2.0 / (t * cr))
                           for (t, ci, co, cr) in nn.LAYERS])
    W = nn.split_params(flat)
    r = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
    chi = (rng.uniform(0, 1, n) > 0.4) * (0.8 + 0.05j)
    tgt = r + 0.5 * (rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n))
    return W, r, chi, tgt


def test_unet_gradient_matches_central_differences():
    """The composed backward pass equals the derivative of the composed loss (exact FP64
    mode, no bfloat16 rounding) for weights of every kind of layer: the first and last
    convolutions, encoder layers whose outputs feed both a skip and a pooling path,
    the bottom, a decoder layer on a concatenation and the 1x1x1 output layer."""
    W, r, chi, tgt = _unet_case(3)
    samples = [(r, chi, tgt)]
    loss, grads = nn.unet_loss_grads(W, samples, bf16=False)
    assert abs(loss - nn.unet_loss(W, samples, bf16=False)) < 1e-12 * loss
    rng = np.random.default_rng(4)
    eps = 1e-5
    for layer in (0, 1, 3, 5, 7, 8, 10, 12, 14):
        gmax = np.abs(grads[layer]).max()
        assert gmax > 0, layer
        # the largest-gradient entry and two random ones
        picks = [np.unravel_index(np.argmax(np.abs(grads[layer])), W[layer].shape)]
        picks += [tuple(rng.integers(0, s) for s in W[layer].shape) for _ in range(2)]
        for idx in picks:
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += eps
            Wm[layer][idx] -= eps
            fd = (nn.unet_loss(Wp, samples, bf16=False) - nn.unet_loss(Wm, samples, bf16=False)) / (2 * eps)
            assert abs(fd - grads[layer][idx]) <= 1e-5 * gmax, (layer, idx, fd, grads[layer][idx])


def test_unet_with_zero_weights_is_the_identity_and_rounding_is_exact_on_integers():
    W, r, chi, _ = _unet_case(5)
    zero = [np.zeros_like(w) for w in W]
    assert np.array_equal(nn.unet_apply(zero, r, chi), r)
    # integer weights and inputs: the rounded and the exact composition agree while
    # every stored value is representable in bfloat16
    rng = np.random.default_rng(6)
    Wi = [np.where(rng.uniform(0, 1, w.shape) < 1.0 / w[0].size, 1.0, 0.0) for w in W]
    ri = np.where(rng.uniform(0, 1, r.shape) < 0.5, 1.0, -1.0).astype(complex)
    ci = (chi != 0).astype(float)
    a = nn.unet_forward(Wi, nn.pack_input(ri, ci, True)[0], True)
    b = nn.unet_forward(Wi, nn.pack_input(ri, ci, False)[0], False)
    for k in a:
        if np.abs(b[k]).max() < 256:
            assert np.array_equal(a[k], b[k]), k
