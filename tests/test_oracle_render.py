"""Pins for the oracle's path-tracing estimator (Sec. 3.1, Sec. 4): furnace
closed forms, roulette unbiasedness, depth semantics, energy bound,
BVH/brute-force identity.  The estimator adds beta*Le only on front-face
emitter hits and beta*Env on escape; roulette from depth rr_start."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import synth


def _closed_furnace_scene(rho, emission=1.0):
    sc = synth.box_scene(open_front=False)
    nt = len(sc["tris"]) - 2  # drop the light quad
    return {"verts": sc["verts"], "tris": sc["tris"][:nt], "tri_mat": np.zeros(nt, np.uint32),
            "materials": [{"type": O.LAMBERT, "albedo": rho, "emission": (emission,) * 3}],
            "camera": sc["camera"]}


@pytest.mark.parametrize("depth", [1, 2, 5, 9])
def test_closed_box_furnace_zero_variance(depth):
    rho = (0.5, 0.25, 0.75)
    sc = _closed_furnace_scene(rho)
    S = O.Scene(sc)
    cam = O.make_camera(**sc["camera"])
    rd = O.render_desc(24, 20, 2, depth, seed=3, rr_start=100, env_const=(0, 0, 0))
    img = O.render(S, cam, rd)
    expect = [sum(r ** k for k in range(depth)) for r in rho]
    assert np.abs(img - np.array(expect)).max() < 1e-12


def test_closed_box_furnace_with_roulette_is_unbiased():
    rho = (0.5, 0.6, 0.7)
    sc = _closed_furnace_scene(rho)
    S = O.Scene(sc)
    cam = O.make_camera(**sc["camera"])
    D = 8
    rd = O.render_desc(96, 96, 1, D, seed=11, rr_start=3, env_const=(0, 0, 0))
    img = O.render(S, cam, rd).reshape(-1, 3)
    expect = np.array([sum(r ** k for k in range(D)) for r in rho])
    mean, sem = img.mean(0), img.std(0, ddof=1) / np.sqrt(len(img))
    assert np.all(np.abs(mean - expect) < 5 * sem + 1e-12), (mean, expect, sem)
    assert img.std(0).min() > 0  # roulette really ran


def _sphere_scene(mtype, albedo=(1, 1, 1)):
    return {"verts": np.zeros((0, 3), np.float32), "tris": np.zeros((0, 3), np.uint32),
            "spheres": np.array([[0, 0, 0, 1]], np.float32), "sph_mat": np.array([0], np.uint32),
            "materials": [{"type": mtype, "albedo": albedo, "ior": 1.5}]}


def test_convex_lambertian_furnace_exact():
    rho = (0.3, 0.55, 0.8)
    S = O.Scene(_sphere_scene(O.LAMBERT, rho))
    cam = O.make_camera((0, 0, 4), (0, 0, 0), (0, 1, 0), 40)
    prim, _, _, _ = O.trace_primary(S, cam, 40, 40, 0, 5)
    rd = O.render_desc(40, 40, 1, 4, seed=5, rr_start=100, env_const=(1, 1, 1))
    img = O.render(S, cam, rd).reshape(-1, 3)
    hit = prim != O.MISS
    assert hit.sum() > 200 and (~hit).sum() > 200
    assert np.all(img[hit] == np.array(rho, np.float32).astype(np.float64))
    assert np.all(img[~hit] == 1.0)


def test_convex_mirror_furnace_exact():
    S = O.Scene(_sphere_scene(O.MIRROR))
    cam = O.make_camera((0, 0, 4), (0, 0, 0), (0, 1, 0), 40)
    rd = O.render_desc(32, 32, 2, 3, seed=5, rr_start=100, env_const=(1, 1, 1))
    assert np.all(O.render(S, cam, rd) == 1.0)


def test_dielectric_sphere_conserves_energy():
    S = O.Scene(_sphere_scene(O.DIELECTRIC))
    cam = O.make_camera((0, 0, 4), (0, 0, 0), (0, 1, 0), 30)
    rd = O.render_desc(32, 32, 4, 64, seed=5, rr_start=1000, env_const=(1, 1, 1))
    img = O.render(S, cam, rd)
    assert img.max() <= 1.0
    assert img.mean() > 0.995  # only paths truncated after 64 segments lose energy


def test_depth_one_sees_only_direct_emission_and_env():
    sc = synth.box_scene(open_front=True)
    S = O.Scene(sc)
    cam = O.make_camera(**sc["camera"])
    W = H = 48
    prim, _, _, _ = O.trace_primary(S, cam, W, H, 0, 9)
    rd = O.render_desc(W, H, 1, 1, seed=9, env_const=(0.25, 0.5, 1.0))
    img = O.render(S, cam, rd).reshape(-1, 3)
    nt = len(sc["tris"])
    light = (prim == nt - 1) | (prim == nt - 2)
    miss = prim == O.MISS
    assert np.all(img[light] == 15.0)
    assert np.all(img[miss] == [0.25, 0.5, 1.0])
    assert np.all(img[~light & ~miss] == 0.0)


def test_emitter_back_face_is_dark():
    # the light quad faces down; seen from above it emits nothing
    sc = synth.box_scene(open_front=True)
    nt = len(sc["tris"])
    only_light = {"verts": sc["verts"], "tris": sc["tris"][nt - 2:], "tri_mat": sc["tri_mat"][nt - 2:],
                  "materials": sc["materials"]}
    S = O.Scene(only_light)
    above = O.make_camera((0, 3, -0.35), (0, 0, -0.35), (0, 0, -1), 10)
    below = O.make_camera((0, 1, -0.35), (0, 3, -0.35), (0, 0, -1), 10)
    rd = O.render_desc(8, 8, 1, 3, seed=1, env_const=(0, 0, 0))
    assert np.all(O.render(S, above, rd) == 0.0)
    assert np.all(O.render(S, below, rd) == 15.0)


def test_energy_bounded_by_brightest_env(small_sky):
    sc = synth.box_scene(open_front=True, light_radiance=0.0)
    S = O.Scene(sc)
    cam = O.make_camera(**sc["camera"])
    rd = O.render_desc(32, 32, 2, 6, seed=2, env=small_sky)
    img = O.render(S, cam, rd)
    assert img.max() <= small_sky.max() * (1 + 1e-12)
    assert img.min() >= 0.0


@pytest.mark.parametrize("cfg", [0, 2])
def test_bvh_render_identical_to_brute_force(cfg, small_sky):
    sc = synth.scene_for(cfg)
    cam = O.make_camera(**sc["camera"])
    env = None if cfg == 0 else small_sky
    kw = {"env_const": (0, 0, 0)} if env is None else {"env": env}
    rd = O.render_desc(24, 24, 2, 5, seed=1, **kw)
    a = O.render(O.Scene(sc, accel=1), cam, rd)
    b = O.render(O.Scene(sc, accel=0), cam, rd)
    assert np.array_equal(a, b)


def test_row_subset_equals_full_render():
    sc = synth.box_scene()
    S = O.Scene(sc)
    cam = O.make_camera(**sc["camera"])
    rd = O.render_desc(32, 32, 2, 5, seed=1, env_const=(0, 0, 0))
    full = O.render(S, cam, rd)
    sub = O.render(S, cam, rd, y0=3, ystep=8)
    assert np.array_equal(full[3::8], sub[3::8])
    assert np.isnan(sub[4]).all()


def test_pixel_list_equals_full_primary_trace():
    sc = synth.large_bvh_scene(grid=33, n_inst=6, ico_level=2, size=20.0, amp=2.0)
    S = O.Scene(sc)
    cam = O.make_camera(**sc["camera"])
    full = O.trace_primary(S, cam, 48, 32, 2, 9)
    px = np.array([0, 5, 47, 48, 700, 1535, 5], np.uint32)
    part = O.trace_pixels(S, cam, 48, 32, 2, 9, px)
    for a, b in zip(full, part):
        assert np.array_equal(a[px], b)
    assert np.any(full[1][full[0] != O.MISS] > 0)  # some instance hits
