"""Pins for the oracle's HDR-NIF (Sec. 3.2): Fourier features, dense ReLU
layers, fixed YUV->RGB output matrix, log compression; Huber loss and Adam
of Sec. 3.2.1.  Forward pass pinned by closed forms (zero network, a
single-neuron path, positive homogeneity), the colour matrix by the BT.601
forward transform, the backward pass by FP64 central differences."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import synth

SHAPE = O.nif_shape(16, 96, 5)


def _layout(shape):
    """(offset_W, offset_b, out, in) of each layer in the flat vector."""
    dims = [4 * shape.n_freq] + [shape.hidden] * shape.layers + [3]
    out, off = [], 0
    for i in range(len(dims) - 1):
        fi, fo = dims[i], dims[i + 1]
        out.append((off, off + fo * fi, fo, fi))
        off += fo * fi + fo
    return out


def test_param_count():
    assert O.nif_param_count(SHAPE) == 43779 == synth.nif_param_count()
    assert O.nif_param_count(O.nif_shape(16, 128, 5)) == synth.nif_param_count(16, 128, 5)


def test_frequencies():
    assert [O.nif_frequency(k) for k in range(16)] == [1, 2, 3, 4, 6, 8, 11, 16, 23, 32, 45, 64,
                                                       91, 128, 181, 256]


def test_features_orthogonal_on_grid():
    # distinct integer frequencies below N/2 are orthogonal on N uniform
    # points: sum sin_a sin_b = sum cos_a cos_b = N/2 delta_ab, sum sin_a cos_b = 0
    N = 1024
    v0 = 0.3125
    F = np.array([O.nif_features(SHAPE, j / N, v0) for j in range(N)])
    G = F[:, :32].T @ F[:, :32]
    assert np.allclose(G, np.eye(32) * N / 2, atol=1e-9)
    # v block is constant along u
    assert np.allclose(F[:, 32:], F[0, 32:], atol=0)
    Fv = np.array([O.nif_features(SHAPE, 0.7, j / N) for j in range(N)])
    Gv = Fv[:, 32:].T @ Fv[:, 32:]
    assert np.allclose(Gv, np.eye(32) * N / 2, atol=1e-9)


def test_features_periodic_in_u():
    for u in (0.0, 0.123, 0.5):
        a = O.nif_features(SHAPE, u, 0.4)
        b = O.nif_features(SHAPE, u + 1.0, 0.4)
        assert np.allclose(a, b, atol=1e-12)


def test_yuv_matrix_inverts_bt601():
    M = O.yuv_to_rgb_matrix()
    # BT.601 RGB -> YUV (Y = .299R + .587G + .114B, U = .492(B - Y), V = .877(R - Y))
    Y = np.array([0.299, 0.587, 0.114])
    F = np.stack([Y, 0.492 * (np.array([0, 0, 1]) - Y), 0.877 * (np.array([1, 0, 0]) - Y)])
    assert np.abs(M @ F - np.eye(3)).max() < 2e-3
    assert np.allclose(M @ [1, 0, 0], [1, 1, 1])  # pure luma is grey


def test_ycocg_matrix_inverts_the_forward_transform():
    # YCoCg (Malvar & Sullivan 2003): Y = R/4 + G/2 + B/4, Co = (R - B)/2,
    # Cg = -R/4 + G/2 - B/4; every coefficient is dyadic, so M F = I exactly
    F = np.array([[0.25, 0.5, 0.25], [0.5, 0.0, -0.5], [-0.25, 0.5, -0.25]])
    M = O.colour_to_rgb_matrix(O.COLOUR_YCOCG)
    assert np.array_equal(M @ F, np.eye(3))
    assert np.array_equal(M @ [1, 0, 0], [1, 1, 1])  # pure luma is grey


def test_colour_matrix_selection():
    assert np.array_equal(O.colour_to_rgb_matrix(O.COLOUR_RGB), np.eye(3))
    assert np.array_equal(O.colour_to_rgb_matrix(O.COLOUR_YUV), O.yuv_to_rgb_matrix())


@pytest.mark.parametrize("colour", [O.COLOUR_YUV, O.COLOUR_RGB, O.COLOUR_YCOCG])
def test_zero_network_outputs_folded_bias(colour):
    shape = O.nif_shape(16, 96, 5, colour)
    p = np.zeros(O.nif_param_count(shape))
    b = np.array([0.3, -0.2, 0.1])
    p[-3:] = b
    z = O.nif_forward(shape, p, 0.37, 0.61)
    assert np.allclose(z, O.colour_to_rgb_matrix(colour) @ b, atol=1e-15)
    rad = O.nif_radiance(shape, p, 0.37, 0.61)
    assert np.allclose(rad, np.maximum(0, np.expm1(z)), atol=1e-15)


@pytest.mark.parametrize("feat", [0, 3, 16 + 5, 32 + 9, 48 + 15])
def test_single_neuron_path_closed_form(feat):
    # W1 routes one feature into neuron 0 with bias 2 (always positive), the
    # hidden layers pass neuron 0 on, the output layer reads it as Y
    p = np.zeros(O.nif_param_count(SHAPE))
    lay = _layout(SHAPE)
    oW, ob, fo, fi = lay[0]
    p[oW + 0 * fi + feat] = 1.0
    p[ob + 0] = 2.0
    for oW, ob, fo, fi in lay[1:-1]:
        p[oW + 0 * fi + 0] = 1.0
    oW, ob, fo, fi = lay[-1]
    p[oW + 0 * fi + 0] = 0.5  # Y = 0.5 * neuron0
    k = feat % 16
    f = O.nif_frequency(k)
    blk = feat // 16
    for u, v in ((0.1, 0.2), (0.77, 0.05), (0.5, 0.9)):
        arg = u if blk < 2 else v
        val = (np.sin if blk % 2 == 0 else np.cos)(2 * np.pi * f * arg)
        z = O.nif_forward(SHAPE, p, u, v)
        assert np.allclose(z, 0.5 * (val + 2.0), atol=1e-12)


def test_positive_homogeneity():
    rng = np.random.default_rng(0)
    p = synth.nif_init(5).astype(np.float64)
    lay = _layout(SHAPE)
    for oW, ob, fo, fi in lay:
        p[ob:ob + fo] = 0.0
    q = p.copy()
    oW, ob, fo, fi = lay[0]
    q[oW:ob] *= 3.0
    for u, v in rng.random((5, 2)):
        assert np.allclose(O.nif_forward(SHAPE, q, u, v), 3.0 * O.nif_forward(SHAPE, p, u, v),
                           rtol=1e-12, atol=1e-14)


def test_huber_closed_form():
    d = 1e-3
    assert O.huber(0.0, d) == 0.0
    assert O.huber(0.5e-3, d) == pytest.approx(0.5 * 0.25e-6)
    assert O.huber(1e-3, d) == pytest.approx(0.5e-6)
    assert O.huber(3e-3, d) == pytest.approx(1e-3 * (3e-3 - 0.5e-3))
    assert O.huber(-3e-3, d) == O.huber(3e-3, d)
    for e in np.linspace(-5e-3, 5e-3, 101):
        h = 1e-9
        fd = (O.huber(e + h, d) - O.huber(e - h, d)) / (2 * h)
        assert abs(fd - O.huber_grad(e, d)) < 1e-6


@pytest.mark.parametrize("colour", [O.COLOUR_YUV, O.COLOUR_RGB, O.COLOUR_YCOCG])
def test_backward_matches_central_differences(colour):
    SHAPE = O.nif_shape(16, 96, 5, colour)
    rng = np.random.default_rng(1)
    p = synth.nif_init(9).astype(np.float64)
    p += rng.normal(size=p.size) * 0.01  # non-zero biases
    n = 6
    uv = rng.random((n, 2))
    target = rng.normal(size=(n, 3)) * 0.5
    # Huber in the quadratic region everywhere keeps the loss smooth
    delta = 1e3
    loss, g = O.nif_loss_grad(SHAPE, p, uv, target, delta)
    idx = np.concatenate([rng.choice(p.size, 300, replace=False), np.arange(p.size - 291, p.size)])
    # step 1e-5: the roundoff of the loss difference (~eps * loss / h) stays
    # below 1e-6 relative for the smallest gradients sampled, the truncation
    # (~h^2) far below that
    h = 1e-5
    worst = 0.0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (O.nif_loss_grad(SHAPE, pp, uv, target, delta, False)[0] -
              O.nif_loss_grad(SHAPE, pm, uv, target, delta, False)[0]) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(1e-6, abs(g[i]), abs(fd)))
    assert worst < 1e-5, worst


@pytest.mark.parametrize("colour", [O.COLOUR_YUV, O.COLOUR_RGB, O.COLOUR_YCOCG])
def test_backward_linear_region_huber(colour):
    # with errors far beyond delta the gradient w.r.t. the last bias is
    # M^T sign(e) delta / (3n), independent of the network
    SHAPE = O.nif_shape(16, 96, 5, colour)
    rng = np.random.default_rng(2)
    p = synth.nif_init(4).astype(np.float64)
    n = 5
    uv = rng.random((n, 2))
    target = np.full((n, 3), 50.0)  # far above any output: e < 0 everywhere
    _, g = O.nif_loss_grad(SHAPE, p, uv, target, 1e-3)
    M = {O.COLOUR_YUV: np.array([[1, 0, 1.13983], [1, -0.39465, -0.58060], [1, 2.03211, 0]]),
         O.COLOUR_RGB: np.eye(3),
         O.COLOUR_YCOCG: np.array([[1, 1, -1], [1, 0, 1], [1, -1, -1]])}[colour]
    expect = M.T @ np.full(3, -1e-3 / 3)
    assert np.allclose(g[-3:], expect, atol=1e-15)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient, bias correction makes every step -lr*g/(|g|+eps)
    g = np.array([1e-3, -2.0, 5e-8, 0.0])
    p = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    for t in range(1, 6):
        before = p.copy()
        O.adam_step(p, g, m, v, t, 1e-3, 0.9, 0.999, 1e-7)
        assert np.allclose(p - before, -1e-3 * g / (np.abs(g) + 1e-7), rtol=1e-9, atol=1e-18)


def test_adam_first_step_sign_update():
    g = np.array([3.0, -0.25])
    p, m, v = np.array([1.0, 1.0]), np.zeros(2), np.zeros(2)
    O.adam_step(p, g, m, v, 1, 0.01, 0.9, 0.999, 0.0)
    assert np.allclose(p, [0.99, 1.01], atol=1e-15)


def test_train_batch_follows_philox_and_log1p(small_sky):
    uv, tg = O.nif_train_batch(small_sky, seed=7, step=3, n=64)
    for i in range(64):
        r = O.philox([i, 3, 0, O.RNG_TRAIN], [7, 0])
        assert uv[i, 0] == O.u01(int(r[0])) and uv[i, 1] == O.u01(int(r[1]))
        assert np.allclose(tg[i], np.log1p(O.env_bilinear(small_sky, *uv[i])), atol=0)


def test_training_reduces_loss(small_sky):
    p = synth.nif_init(3).astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    losses = [O.nif_train_step(SHAPE, p, m, v, small_sky, seed=1, step=s, batch=256, lr=3e-3)
              for s in range(30)]
    assert np.mean(losses[-5:]) < 0.6 * np.mean(losses[:5])


# ---- skip-concat (Sec. 3.2: the features enter again at a middle layer, and
# the layer before it is narrowed so that the concatenation stays H wide)
SKIP = O.nif_shape(4, 32, 4, O.COLOUR_YUV, 2)  # 16 features; layer 1 is 32 - 16 = 16 wide


def _skip_layout():
    """(offset_W, offset_b, out, in) per layer of SKIP: layer 1 has 16
    outputs, layer 2 reads them followed by the 16 features (32 inputs)."""
    fans = [(16, 32), (32, 16), (16 + 16, 32), (32, 32), (32, 3)]
    out, off = [], 0
    for fi, fo in fans:
        out.append((off, off + fo * fi, fo, fi))
        off += fo * fi + fo
    return out


def test_skip_param_count():
    n = sum(fo * fi + fo for _, _, fo, fi in _skip_layout())
    assert O.nif_param_count(SKIP) == n == synth.nif_param_count(4, 32, 4, 2) == synth.nif_init(1, 4, 32, 4, 2).size
    # the plain network minus the 16 rows (weights and biases) the narrowed layer drops
    assert n == O.nif_param_count(O.nif_shape(4, 32, 4)) - 16 * (32 + 1)
    # the paper's shape: 40-d features, H128, four dense-ReLU layers,
    # concatenation at hidden layer 2
    paper = O.nif_shape(10, 128, 4, O.COLOUR_YUV, 2)
    assert O.nif_param_count(paper) == (40 * 128 + 128) + (128 * 88 + 88) + 2 * (128 * 128 + 128) + (3 * 128 + 3)


@pytest.mark.parametrize("feat", [0, 5, 15])
def test_skip_path_closed_form(feat):
    # every weight zero except the skip layer reading one feature into neuron
    # 0 (bias 2), the next layer passing it on, the output reading it as Y:
    # the features appear after the 16 outputs of the narrowed layer
    p = np.zeros(O.nif_param_count(SKIP))
    lay = _skip_layout()
    oW, ob, fo, fi = lay[2]
    p[oW + 0 * fi + 16 + feat] = 1.0
    p[ob + 0] = 2.0
    oW, ob, fo, fi = lay[3]
    p[oW + 0] = 1.0
    oW, ob, fo, fi = lay[4]
    p[oW + 0] = 0.5
    k, blk = feat % 4, feat // 4
    f = O.nif_frequency(k)
    for u, v in ((0.1, 0.2), (0.77, 0.05)):
        val = (np.sin if blk % 2 == 0 else np.cos)(2 * np.pi * f * (u if blk < 2 else v))
        assert np.allclose(O.nif_forward(SKIP, p, u, v), 0.5 * (val + 2.0), atol=1e-12)
        # the quantised forward in FP32 mode is the same function
        assert np.allclose(O.nif_forward_q(SKIP, p, O.PREC_FP32, u, v), 0.5 * (val + 2.0), atol=1e-12)


def test_skip_narrowed_layer_feeds_the_hidden_columns():
    # a path through neuron 15 of the narrowed layer (its last output) and
    # column 15 of the skip layer: ReLU(u-feature sin) passes through, and
    # column 16 (the first feature) is not fed by the narrowed layer
    p = np.zeros(O.nif_param_count(SKIP))
    lay = _skip_layout()
    oW, ob, fo, fi = lay[0]
    p[oW + 15 * fi + 0] = 1.0  # neuron 15 of layer 0 reads feature 0: sin(2 pi u)
    p[ob + 15] = 1.5
    oW, ob, fo, fi = lay[1]
    p[oW + 15 * fi + 15] = 1.0  # narrowed layer 1, output 15 (its last), reads it
    oW, ob, fo, fi = lay[2]
    p[oW + 3 * fi + 15] = 2.0  # skip layer: hidden column 15 into neuron 3
    oW, ob, fo, fi = lay[3]
    p[oW + 0 * fi + 3] = 1.0
    oW, ob, fo, fi = lay[4]
    p[oW + 0] = 1.0
    for u, v in ((0.1, 0.2), (0.6, 0.9)):
        assert np.allclose(O.nif_forward(SKIP, p, u, v), 2.0 * (np.sin(2 * np.pi * u) + 1.5), atol=1e-12)


def test_skip_backward_matches_central_differences():
    rng = np.random.default_rng(7)
    p = synth.nif_init(9, 4, 32, 4, 2).astype(np.float64) + rng.normal(size=O.nif_param_count(SKIP)) * 0.01
    uv = rng.random((5, 2))
    target = rng.normal(size=(5, 3)) * 0.5
    _, g = O.nif_loss_grad(SKIP, p, uv, target, 1e3)
    lay = _skip_layout()
    # every weight of the skip layer's feature columns, every weight of the
    # narrowed layer, plus a random sample
    oW, ob, fo, fi = lay[2]
    skip_cols = [oW + j * fi + 16 + c for j in range(0, fo, 5) for c in range(16)]
    oW1, ob1, fo1, fi1 = lay[1]
    idx = np.concatenate([skip_cols, np.arange(oW1, ob1 + fo1, 7), rng.choice(p.size, 200, replace=False)])
    h = 1e-5
    worst = 0.0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (O.nif_loss_grad(SKIP, pp, uv, target, 1e3, False)[0] - O.nif_loss_grad(SKIP, pm, uv, target, 1e3,
                                                                                      False)[0]) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(1e-6, abs(g[i]), abs(fd)))
    assert worst < 1e-5, worst


def test_fewer_frequencies_keep_the_feature_layout():
    # 10 frequencies (the paper's 40-d features): the first 10 of each block of
    # the 16-frequency features, blocks [sin u | cos u | sin v | cos v]
    s10 = O.nif_shape(10, 32, 2)
    for u, v in ((0.13, 0.71), (0.5, 0.25)):
        f16 = O.nif_features(SHAPE, u, v).reshape(4, 16)
        f10 = O.nif_features(s10, u, v).reshape(4, 10)
        assert np.array_equal(f10, f16[:, :10])
    assert O.nif_param_count(s10) == 40 * 32 + 32 + (32 * 32 + 32) + 3 * 32 + 3
