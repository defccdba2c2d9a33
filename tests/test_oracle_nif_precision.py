"""Pins for the oracle's reduced-precision NIF inference: the rounding
functions against library conversions and brute force over the E4M3 code
table, the FP8 weight scale rule, the dequantised weights, and the quantised
forward pass (FP32 mode is the FP64 forward; the others insert the rounding
at each layer input, checked against a NumPy layer loop using the library
conversions)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2305_20061_amd import synth

SHAPE = O.nif_shape(16, 96, 5)


def _e4m3_table():
    """Value of every finite OCP E4M3 code (sign, 4 exponent bits with bias 7,
    3 fraction bits; exponent field 0 is subnormal; S.1111.111 is NaN)."""
    codes, vals = [], []
    for c in range(256):
        e, m = (c >> 3) & 15, c & 7
        if e == 15 and m == 7:
            continue
        mag = m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
        codes.append(c)
        vals.append(-mag if c & 0x80 else mag)
    return np.array(codes), np.array(vals)


def _e4m3_brute(x):
    codes, vals = _e4m3_table()
    out = np.empty_like(x)
    for i, xv in enumerate(x):
        if abs(xv) >= 448:
            out[i] = np.sign(xv) * 448.0
            continue
        d = np.abs(vals - xv)
        best = np.nonzero(d == d.min())[0]
        # a tie goes to the code with an even fraction field
        k = best[0] if len(best) == 1 else [b for b in best if codes[b] % 2 == 0][0]
        out[i] = vals[k]
    return out


def _probe_values(seed=0):
    rng = np.random.default_rng(seed)
    _, vals = _e4m3_table()
    pos = np.unique(np.abs(vals))
    mids = (pos[:-1] + pos[1:]) / 2  # exact ties of E4M3
    return np.concatenate([mids, -mids[::3], vals, rng.uniform(-460, 460, 500), rng.normal(0, 0.02, 500),
                           rng.lognormal(-3, 3, 500), [0.0, 2.0 ** -10, 2.0 ** -11, 449.0, 463.9, 1e6]])


def test_e4m3_rounding_brute_force():
    x = _probe_values()
    assert np.array_equal(O.round_to(x, O.FMT_E4M3), _e4m3_brute(x))


def test_e4m3_rounding_matches_torch_in_range():
    x = _probe_values(1)
    x = x[np.abs(x) <= 448].astype(np.float32).astype(np.float64)
    t = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(O.round_to(x, O.FMT_E4M3), t)


def test_fp16_rounding_matches_numpy():
    rng = np.random.default_rng(2)
    h = rng.integers(0, 0x7C00, 4000).astype(np.uint16).view(np.float16).astype(np.float64)
    nxt = np.nextafter(h.astype(np.float16), np.float16(np.inf)).astype(np.float64)
    x = np.concatenate([h, (h + nxt) / 2, -(h + nxt) / 2, rng.normal(0, 1e3, 2000), rng.normal(0, 1e-6, 2000),
                        [65504.0, 65519.0, 65520.0, 1e9]])
    x = x[np.isfinite(x)]
    with np.errstate(over="ignore"):  # beyond 65520 the cast is infinite, as is the rounding
        ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(O.round_to(x, O.FMT_F16), ref)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 3000), rng.lognormal(0, 20, 3000), -rng.lognormal(0, 20, 1000)])
    x = x.astype(np.float32)
    b = x.view(np.uint32) & np.uint32(0xFFFF0000)
    ties = (b.view(np.float32).astype(np.float64) + (b + np.uint32(0x10000)).view(np.float32).astype(np.float64)) / 2
    x = np.concatenate([x.astype(np.float64), ties[np.isfinite(ties)]])
    x = x[np.abs(x) < 3e38].astype(np.float32)  # float32 inputs, as the device converts
    t = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.round_to(x.astype(np.float64), O.FMT_BF16), t)


@pytest.mark.parametrize("m", [1e-9, 0.013, 0.3, 1.0, 1.75, 1.7500001, 2.0, 447.9, 448.0, 449.0, 1e6])
def test_fp8_scale_rule(m):
    s = O.nif_fp8_scale_exp(m)
    assert m * 2.0 ** s <= 448.0 < m * 2.0 ** (s + 1)


def test_fp8_scale_of_zero_layer():
    assert O.nif_fp8_scale_exp(0.0) == 0


def _params(seed=3):
    p = synth.nif_init(seed).astype(np.float32).astype(np.float64)
    p[-3:] = (0.6, 0.05, -0.05)
    return p


def _layers(shape):
    dims = [4 * shape.n_freq] + [shape.hidden] * shape.layers + [3]
    off = 0
    for l in range(len(dims) - 1):
        fi, fo = dims[l], dims[l + 1]
        yield l, off, off + fo * fi, fo, fi
        off += fo * fi + fo


def test_dequantized_weights():
    p = _params()
    assert np.array_equal(O.nif_dequantize(SHAPE, p, O.PREC_FP32), p)
    f16 = O.nif_dequantize(SHAPE, p, O.PREC_FP16)
    f8 = O.nif_dequantize(SHAPE, p, O.PREC_FP8)
    _, table = _e4m3_table()
    for l, ow, ob, fo, fi in _layers(SHAPE):
        w = p[ow:ob]
        assert np.array_equal(f16[ow:ob], w.astype(np.float16).astype(np.float64))
        assert np.array_equal(f16[ob:ob + fo], p[ob:ob + fo]) and np.array_equal(f8[ob:ob + fo], p[ob:ob + fo])
        if l in (0, SHAPE.layers):
            assert np.array_equal(f8[ow:ob], f16[ow:ob])
        else:
            s = O.nif_fp8_scale_exp(np.abs(w).max())
            q = f8[ow:ob] * 2.0 ** s
            assert np.all(np.isin(q, table))  # every weight is an E4M3 value times 2^-s
            assert np.array_equal(q, _e4m3_brute(w * 2.0 ** s))


def test_fp32_mode_is_the_fp64_forward():
    p = _params()
    for u, v in [(0.1, 0.7), (0.93, 0.02), (0.5, 0.5)]:
        assert np.array_equal(O.nif_forward_q(SHAPE, p, O.PREC_FP32, u, v), O.nif_forward(SHAPE, p, u, v))


def _numpy_forward_q(p_deq, prec, u, v):
    """Layer loop in NumPy; inputs rounded by library conversions."""
    def rnd(x, l):
        last = l == SHAPE.layers
        if prec == O.PREC_FP16 or (prec == O.PREC_FP8 and (l == 0 or last)):
            return x.astype(np.float16).astype(np.float64)
        if prec == O.PREC_BF16:
            return torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
        if prec == O.PREC_FP8:
            return torch.from_numpy(np.minimum(x, 448).astype(np.float32)).to(torch.float8_e4m3fn).to(
                torch.float64).numpy()
        return x
    x = O.nif_features(SHAPE, u, v)
    for l, ow, ob, fo, fi in _layers(SHAPE):
        W = p_deq[ow:ob].reshape(fo, fi)
        y = W @ rnd(x, l) + p_deq[ob:ob + fo]
        x = np.maximum(y, 0.0) if l < SHAPE.layers else y
    return O.yuv_to_rgb_matrix() @ x


def test_skip_quantised_forward_matches_numpy_layer_loop():
    # skip-concat network (features again at hidden layer 2, layer 1 narrowed
    # to 96 - 64 = 32 outputs), FP16 operands: the concatenated input is
    # rounded as one vector
    shape = O.nif_shape(16, 96, 4, O.COLOUR_YUV, 2)
    p = synth.nif_init(4, 16, 96, 4, 2).astype(np.float64)
    p[-3:] = (0.6, 0.05, -0.05)
    q = O.nif_dequantize(shape, p, O.PREC_FP16)
    fans = [(64, 96), (96, 32), (32 + 64, 96), (96, 96), (96, 3)]
    rnd = lambda x: x.astype(np.float16).astype(np.float64)
    for u, v in np.random.default_rng(8).uniform(0, 1, (10, 2)):
        feat = O.nif_features(shape, u, v)
        x, off = feat, 0
        for l, (fi, fo) in enumerate(fans):
            if l == 2:
                x = np.concatenate([x, feat])
            W = q[off:off + fo * fi].reshape(fo, fi)
            y = W @ rnd(x) + q[off + fo * fi:off + fo * fi + fo]
            off += fo * fi + fo
            x = np.maximum(y, 0.0) if l < 4 else y
        assert np.allclose(O.nif_forward_q(shape, q, O.PREC_FP16, u, v), O.yuv_to_rgb_matrix() @ x,
                           rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("prec", [O.PREC_FP16, O.PREC_BF16, O.PREC_FP8])
def test_quantised_forward_matches_numpy_layer_loop(prec):
    # BF16 via torch needs float32-exact inputs: features and activations are
    # rounded from FP64 here, so compare with a tolerance far below one BF16 ulp
    p = O.nif_dequantize(SHAPE, _params(), prec)
    rng = np.random.default_rng(5)
    for u, v in rng.uniform(0, 1, (20, 2)):
        a = O.nif_forward_q(SHAPE, p, prec, u, v)
        b = _numpy_forward_q(p, prec, u, v)
        assert np.allclose(a, b, rtol=1e-6, atol=1e-9), (prec, u, v, a, b)


def test_fp8_inference_stays_close_to_fp64():
    p = _params()
    q = O.nif_dequantize(SHAPE, p, O.PREC_FP8)
    rng = np.random.default_rng(6)
    z64, z8 = [], []
    for u, v in rng.uniform(0, 1, (200, 2)):
        z64.append(O.nif_forward(SHAPE, p, u, v))
        z8.append(O.nif_forward_q(SHAPE, q, O.PREC_FP8, u, v))
    z64, z8 = np.array(z64), np.array(z8)
    r = np.sqrt(np.mean((z8 - z64) ** 2)) / np.sqrt(np.mean(z64 ** 2))
    # 3 fraction bits: per-value relative rounding error up to 2^-4
    assert 1e-4 < r < 0.1
