"""Pins for the oracle's reduced-precision training gradient
(or_nif_loss_grad_q; Sec. 3.2.1 trains in low precision with a loss scale):
FP32 mode is the FP64 gradient of or_nif_loss_grad; FP16 / BF16 equal a
batched NumPy layer loop that rounds with library casts; the loss scale
cancels exactly where nothing underflows (BF16) and, in FP16, the paper's
scale of 16384 keeps the gradient closer to the FP64 one than no scale."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2305_20061_amd import synth

DELTA = 1e-3


def _batch(env, n, seed=5, step=2):
    return O.nif_train_batch(env, seed, step, n)


def _dims(shape):
    return synth.nif_layer_dims(shape.n_freq, shape.hidden, shape.layers, shape.skip)


def _rounder(prec):
    if prec == O.PREC_FP16:
        return lambda x: np.asarray(x, np.float64).astype(np.float16).astype(np.float64)
    if prec == O.PREC_BF16:  # via FP32 (torch's cast); FP32-exact inputs round once
        return lambda x: torch.from_numpy(np.asarray(x, np.float64)).to(torch.bfloat16).to(torch.float64).numpy()
    return lambda x: np.asarray(x, np.float64)


def _numpy_loss_grad_q(shape, p, prec, S, uv, target):
    """Whole-batch matrix form of the rounded-operand backward."""
    rnd = _rounder(prec)
    dims = _dims(shape)
    L = shape.layers
    Ws, bs, off = [], [], 0
    for fi, fo in dims:
        Ws.append(p[off:off + fo * fi].reshape(fo, fi))
        bs.append(p[off + fo * fi:off + fo * fi + fo])
        off += fo * fi + fo
    Wq = [rnd(W) for W in Ws[:L]] + [Ws[L]]
    X0 = rnd(np.array([O.nif_features(shape, u, v) for u, v in uv]))
    xs = [X0]
    for l in range(L):
        a = rnd(np.maximum(xs[-1] @ Wq[l].T + bs[l], 0.0))
        if shape.skip and l + 1 == shape.skip:
            a = np.concatenate([a, X0], axis=1)
        xs.append(a)
    M = O.colour_to_rgb_matrix(shape.colour)
    Z = (xs[L] @ Ws[L].T + bs[L]) @ M.T
    E = Z - target
    A = np.abs(E)
    loss = np.mean(np.where(A <= DELTA, 0.5 * E * E, DELTA * (A - 0.5 * DELTA)))
    dY = (np.where(A <= DELTA, E, np.sign(E) * DELTA) * S) @ M
    gW = [None] * (L + 1)
    gb = [None] * (L + 1)
    gW[L], gb[L] = dY.T @ xs[L], dY.sum(0)
    G = rnd(np.where(xs[L] > 0, dY @ Ws[L], 0.0))
    for l in range(L - 1, -1, -1):
        gW[l], gb[l] = G.T @ xs[l], G.sum(0)
        if l > 0:
            nprev = dims[l - 1][1]
            G = rnd(np.where(xs[l][:, :nprev] > 0, G @ Wq[l][:, :nprev], 0.0))
    n = uv.shape[0]
    g = np.concatenate([np.concatenate([gW[l].ravel(), gb[l]]) for l in range(L + 1)])
    return loss, g / (3.0 * n * S)


SHAPES = [O.nif_shape(16, 32, 3), O.nif_shape(4, 32, 4, O.COLOUR_YUV, 2), O.nif_shape(16, 96, 5, O.COLOUR_RGB)]


def _params(shape, seed=11):
    return synth.nif_init(seed, shape.n_freq, shape.hidden, shape.layers, shape.skip).astype(np.float64)


@pytest.mark.parametrize("shape", SHAPES[:2])
@pytest.mark.parametrize("S", [1.0, 1024.0, 16384.0])
def test_fp32_mode_is_the_fp64_gradient(shape, S, small_sky):
    p = _params(shape)
    uv, tg = _batch(small_sky, 40)
    l0, g0 = O.nif_loss_grad(shape, p, uv, tg, DELTA)
    l1, g1 = O.nif_loss_grad_q(shape, p, O.PREC_FP32, S, uv, tg, DELTA)
    assert abs(l1 - l0) <= 1e-14 * abs(l0)
    assert np.allclose(g1, g0, rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", [O.PREC_FP16, O.PREC_BF16])
def test_rounded_backward_matches_batched_numpy_loop(shape, prec, small_sky):
    p = _params(shape)
    uv, tg = _batch(small_sky, 48)
    S = 16384.0 if prec == O.PREC_FP16 else 1.0
    lc, gc = O.nif_loss_grad_q(shape, p, prec, S, uv, tg, DELTA)
    ln, gn = _numpy_loss_grad_q(shape, p, prec, S, uv, tg)
    r = np.sqrt(np.sum((gc - gn) ** 2) / np.sum(gn ** 2))
    assert abs(lc - ln) <= 1e-12 * abs(ln)
    # FP16: numpy rounds binary64 -> binary16 once, as the oracle does.  BF16
    # goes through FP32 in torch: a value within an FP32 rounding of a BF16
    # tie can round the other way (rare; one activation, one ulp)
    assert r <= (1e-12 if prec == O.PREC_FP16 else 1e-5), r
    # a dropped or mis-signed term would show far above rounding level
    l0, g0 = O.nif_loss_grad(shape, p, uv, tg, DELTA)
    assert np.sqrt(np.sum((gc - g0) ** 2) / np.sum(g0 ** 2)) < 0.1


def test_bf16_gradient_does_not_depend_on_the_loss_scale(small_sky):
    # BF16 has FP32's exponent range: a power-of-two scale commutes with every
    # rounding and cancels exactly
    shape = SHAPES[0]
    p = _params(shape)
    uv, tg = _batch(small_sky, 64)
    g = [O.nif_loss_grad_q(shape, p, O.PREC_BF16, S, uv, tg, DELTA)[1] for S in (1.0, 1024.0, 16384.0)]
    assert np.array_equal(g[0], g[1]) and np.array_equal(g[0], g[2])


def test_fp16_loss_scale_keeps_small_gradients(small_sky):
    # a network close to its targets (output weights scaled by 1e-3, targets
    # 1e-4 off its output): the back-propagated gradients are of order 1e-7,
    # inside binary16's subnormal range (spacing 2^-24 = 6e-8), and lose
    # their digits without a scale; the paper's 16384 lifts them into the
    # normal range
    shape = O.nif_shape(16, 96, 5)
    p = _params(shape)
    dims = _dims(shape)
    off = sum(fo * fi + fo for fi, fo in dims[:-1])
    p[off:off + 3 * 96] *= 1e-3
    rng = np.random.default_rng(3)
    uv = rng.random((96, 2))
    tg = np.array([O.nif_forward(shape, p, u, v) for u, v in uv]) + 1e-4 * rng.choice([-1.0, 1.0], (96, 3))
    _, g0 = O.nif_loss_grad(shape, p, uv, tg, DELTA)
    err = {}
    for S in (1.0, 16384.0):
        _, g = O.nif_loss_grad_q(shape, p, O.PREC_FP16, S, uv, tg, DELTA)
        # the hidden layers' gradients (the output layer's gradient is formed
        # before any rounding of a back-propagated value)
        err[S] = np.sqrt(np.sum((g[:off] - g0[:off]) ** 2) / np.sum(g0[:off] ** 2))
    assert err[16384.0] < 0.1 * err[1.0], err


def test_threaded_batch_chunks_give_the_same_mean(small_sky):
    shape = SHAPES[1]
    p = _params(shape)
    uv, tg = _batch(small_sky, 203)
    l1, g1 = O.nif_loss_grad_q(shape, p, O.PREC_FP16, 16384.0, uv, tg, DELTA)
    l4, g4 = O.nif_loss_grad_q(shape, p, O.PREC_FP16, 16384.0, uv, tg, DELTA, threads=4)
    assert abs(l4 - l1) <= 1e-13 * l1
    assert np.allclose(g4, g1, rtol=1e-11, atol=1e-20)
    l0, g0 = O.nif_loss_grad(shape, p, uv, tg, DELTA)
    l3, g3 = O.nif_loss_grad(shape, p, uv, tg, DELTA, threads=3)
    assert abs(l3 - l0) <= 1e-13 * l0 and np.allclose(g3, g0, rtol=1e-11, atol=1e-20)
