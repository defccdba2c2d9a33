"""Pins for the oracle's environment side (Sec. 3.3 direction -> equirect
(u,v); Sec. 3.2.1 bilinear sub-pixel samples)."""
import numpy as np

import oracle as O


def test_equirect_round_trip():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        u, v = O.dir_to_uv(d)
        assert 0 <= u <= 1 and 0 <= v <= 1
        assert np.abs(O.uv_to_dir(u, v) - d).max() < 1e-12


def test_equirect_poles_and_axes():
    assert O.dir_to_uv([0, 1, 0])[1] == 0.0
    assert O.dir_to_uv([0, -1, 0])[1] == 1.0
    u, v = O.dir_to_uv([1, 0, 0])
    assert abs(u - 0.5) < 1e-15 and abs(v - 0.5) < 1e-15
    u, _ = O.dir_to_uv([0, 0, 1])
    assert abs(u - 0.75) < 1e-15


def test_bilinear_texel_centres_exact():
    rng = np.random.default_rng(1)
    env = rng.random((16, 32, 3)).astype(np.float32)
    for j in range(16):
        for i in range(32):
            out = O.env_bilinear(env, (i + 0.5) / 32, (j + 0.5) / 16)
            assert out.tolist() == env[j, i].astype(np.float64).tolist()


def test_bilinear_midpoints_wrap_and_clamp():
    rng = np.random.default_rng(2)
    env = rng.random((8, 16, 3)).astype(np.float32)
    e = env.astype(np.float64)
    # midpoint between two horizontal neighbours
    assert np.allclose(O.env_bilinear(env, 3.0 / 16, 2.5 / 8), 0.5 * (e[2, 2] + e[2, 3]), atol=1e-15)
    # u = 0 is half-way between the last and the first column (wrap)
    assert np.allclose(O.env_bilinear(env, 0.0, 4.5 / 8), 0.5 * (e[4, 15] + e[4, 0]), atol=1e-15)
    # v = 0 clamps to the first row
    assert np.allclose(O.env_bilinear(env, 5.5 / 16, 0.0), e[0, 5], atol=1e-15)
    assert np.allclose(O.env_bilinear(env, 5.5 / 16, 1.0), e[7, 5], atol=1e-15)
    # centre of four texels: their mean
    assert np.allclose(O.env_bilinear(env, 6.0 / 16, 3.0 / 8), e[2:4, 5:7].mean(axis=(0, 1)), atol=1e-15)


def test_bilinear_reproduces_linear_ramps():
    # bilinear interpolation is exact on a field linear in texel coordinates
    W, H = 32, 16
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    env = np.stack([ii * 1.0, jj * 2.0, ii + jj], -1).astype(np.float32)
    rng = np.random.default_rng(3)
    for _ in range(500):
        x, y = rng.uniform(0.5, W - 1.5), rng.uniform(0.5, H - 1.5)
        out = O.env_bilinear(env, (x + 0.5) / W, (y + 0.5) / H)
        assert np.allclose(out, [x, 2 * y, x + y], atol=1e-9)
