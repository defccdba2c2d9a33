"""Pins for the oracle's ray operations (Sec. 3.1.3-3.1.4): camera, watertight
triangle test, sphere test, BVH closest hit, spawned-ray offset.  Each is
checked against FP64 closed forms, brute force or geometric invariants."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import synth


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


# ------------------------------------------------------------------- camera
def test_camera_matches_fp64_pinhole():
    cam = O.make_camera((0.5, 1.0, 3.0), (0.0, 0.8, -1.0), (0, 1, 0), 50.0)
    W, H = 64, 48
    eye = np.array([0.5, 1.0, 3.0])
    fwd = _unit(np.array([0.0, 0.8, -1.0]) - eye)
    right = _unit(np.cross(fwd, [0, 1, 0]))
    up = np.cross(right, fwd)
    th = np.tan(np.radians(25.0))
    rng = np.random.default_rng(2)
    for _ in range(300):
        x, y = int(rng.integers(W)), int(rng.integers(H))
        jx, jy = np.float32(rng.random()), np.float32(rng.random())
        o, d = O.camera_ray(cam, W, H, x, y, jx, jy)
        sx = 2 * (x + float(jx)) / W - 1
        sy = 1 - 2 * (y + float(jy)) / H
        ref = _unit(fwd + sx * th * (W / H) * right + sy * th * up)
        assert np.allclose(o, eye, atol=0)
        assert np.abs(d - ref).max() < 3e-7


def test_camera_centre_ray_is_forward():
    cam = O.make_camera((0, 0, 0), (0, 0, -5), (0, 1, 0), 60.0)
    o, d = O.camera_ray(cam, 2, 2, 1, 1, 0.0, 0.0)  # ndc (0,0)
    assert d.tolist() == [0.0, 0.0, -1.0]


# ----------------------------------------------------------------- triangle
def test_triangle_t_matches_fp64_plane():
    rng = np.random.default_rng(3)
    n_hit = 0
    for _ in range(2000):
        v = rng.normal(size=(3, 3)).astype(np.float32)
        o = (rng.normal(size=3) * 4).astype(np.float32)
        w = rng.dirichlet([1, 1, 1])
        target = w @ v.astype(np.float64)
        d = _unit(target - o).astype(np.float32)
        t = O.intersect_triangle(o, d, *v)
        # FP64 plane intersection of the FP32 ray
        n = np.cross(v[1].astype(np.float64) - v[0], v[2].astype(np.float64) - v[0])
        dn = np.dot(n, d.astype(np.float64))
        if abs(dn) < 1e-3 * np.linalg.norm(n) or w.min() < 1e-3:
            continue  # grazing or near an edge: FP32 inside/outside not decided by FP64
        tref = np.dot(n, v[0].astype(np.float64) - o) / dn
        assert t is not None, "interior hit missed"
        assert abs(t - tref) <= 1e-5 * max(1.0, abs(tref)), (t, tref)
        n_hit += 1
    assert n_hit > 1000


def test_triangle_misses_outside_and_behind():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    assert O.intersect_triangle([0.6, 0.6, 1], [0, 0, -1], *v) is None  # outside the hypotenuse
    assert O.intersect_triangle([0.2, 0.2, -1], [0, 0, -1], *v) is None  # behind the origin
    assert O.intersect_triangle([0.2, 0.2, 1], [0, 0, -1], *v, tmax=0.5) is None  # beyond tmax
    assert O.intersect_triangle([0.2, 0.2, 1], [0, 0, -1], *v) == 1.0
    assert O.intersect_triangle([0.2, 0.2, -1], [0, 0, 1], *v) == 1.0  # back face is hit
    assert O.intersect_triangle([0, 0, 1], [1, 0, 0], *v) is None  # parallel: det == 0


def test_triangle_watertight_on_shared_edges():
    # a 16x16 grid of quads split into triangles; rays aimed at grid vertices
    # and edge midpoints (exactly representable) must hit at least one triangle
    N = 16
    xs = np.arange(N + 1, dtype=np.float32) / 4
    tris = []
    for i in range(N):
        for j in range(N):
            a = (xs[i], xs[j], 0)
            b = (xs[i + 1], xs[j], 0)
            c = (xs[i + 1], xs[j + 1], 0)
            d = (xs[i], xs[j + 1], 0)
            tris += [(a, b, c), (a, c, d)]
    tris = np.array(tris, np.float32)
    rng = np.random.default_rng(4)
    for k in range(400):
        i, j = rng.integers(1, N, size=2)
        px, py = xs[i], xs[j]
        if k % 2:
            px = np.float32((xs[i] + xs[i + 1]) / 2)
        o = np.array([px, py, 0], np.float32) + (rng.normal(size=3) * [1, 1, 0] + [0, 0, 3]).astype(np.float32)
        d = (np.array([px, py, 0], np.float64) - o)
        d = (d / np.linalg.norm(d)).astype(np.float32)
        hits = [O.intersect_triangle(o, d, *t) for t in tris]
        assert any(h is not None for h in hits), (px, py, o, d)


def test_triangle_closed_mesh_always_hit_from_inside():
    v, f = synth.icosphere(2)
    v = v.astype(np.float32)
    sc = {"verts": v, "tris": f.astype(np.uint32), "materials": [{"type": 0, "albedo": (1, 1, 1)}]}
    S = O.Scene(sc, accel=0)
    rng = np.random.default_rng(5)
    for _ in range(2000):
        o = (rng.normal(size=3) * 0.2).astype(np.float32)
        d = _unit(rng.normal(size=3)).astype(np.float32)
        assert S.closest_hit(o, d) is not None


# ------------------------------------------------------------------- sphere
def test_sphere_t_matches_fp64_quadratic():
    rng = np.random.default_rng(6)
    n = 0
    for _ in range(3000):
        c = (rng.normal(size=3) * 3).astype(np.float32)
        r = np.float32(rng.uniform(0.2, 2.0))
        o = (rng.normal(size=3) * 6).astype(np.float32)
        d = _unit(c + rng.normal(size=3) * r * 0.7 - o).astype(np.float32)
        t = O.intersect_sphere(o, d, c, r)
        oo, dd, cc = o.astype(np.float64), d.astype(np.float64), c.astype(np.float64)
        dd = dd  # FP32-unit direction, solved exactly in FP64 with its own length
        a = dd @ dd
        b = 2 * dd @ (oo - cc)
        k = (oo - cc) @ (oo - cc) - float(r) ** 2
        disc = b * b - 4 * a * k
        if disc <= 1e-6 * b * b:
            continue
        roots = sorted([(-b - np.sqrt(disc)) / (2 * a), (-b + np.sqrt(disc)) / (2 * a)])
        pos = [x for x in roots if x > 1e-4]
        if not pos:
            assert t is None
            continue
        assert t is not None
        assert abs(t - pos[0]) <= 2e-6 * max(1.0, pos[0]) + 1e-6 * np.linalg.norm(oo - cc), (t, pos[0])
        n += 1
    assert n > 1500


def test_sphere_through_centre():
    rng = np.random.default_rng(7)
    for _ in range(200):
        c = (rng.normal(size=3) * 2).astype(np.float32)
        r = np.float32(rng.uniform(0.3, 1.5))
        o = (c + _unit(rng.normal(size=3)) * rng.uniform(3, 9)).astype(np.float32)
        d = _unit(c.astype(np.float64) - o).astype(np.float32)
        t = O.intersect_sphere(o, d, c, r)
        ref = np.linalg.norm(c.astype(np.float64) - o) - r
        assert abs(t - ref) < 2e-6 * ref


def test_sphere_from_inside_hits_far_side():
    t = O.intersect_sphere([0, 0, 0], [0, 0, 1], [0, 0, 0], 2.0)
    assert t == 2.0
    assert O.intersect_sphere([0, 0, 5], [0, 0, 1], [0, 0, 0], 2.0) is None  # behind


# ---------------------------------------------------- BVH vs brute force
def _random_soup(rng, nt, ns):
    centres = rng.uniform(-5, 5, size=(nt, 1, 3))
    verts = (centres + rng.normal(size=(nt, 3, 3)) * 0.6).reshape(-1, 3).astype(np.float32)
    tris = np.arange(3 * nt, dtype=np.uint32).reshape(nt, 3)
    sph = np.concatenate([rng.uniform(-5, 5, size=(ns, 3)), rng.uniform(0.1, 0.8, size=(ns, 1))], 1)
    return {"verts": verts, "tris": tris, "spheres": sph.astype(np.float32),
            "materials": [{"type": 0, "albedo": (1, 1, 1)}]}


@pytest.mark.parametrize("seed", [0, 1])
def test_bvh_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    sc = _random_soup(rng, 300, 30)
    A, B = O.Scene(sc, accel=1), O.Scene(sc, accel=0)
    for _ in range(3000):
        o = rng.uniform(-8, 8, size=3).astype(np.float32)
        d = _unit(rng.normal(size=3)).astype(np.float32)
        ha, hb = A.closest_hit(o, d), B.closest_hit(o, d)
        assert (ha is None) == (hb is None)
        if ha:
            assert ha[0] == hb[0] and ha[1] == hb[1] and ha[2] == hb[2]


def test_ties_go_to_lowest_primitive():
    # two coincident triangles: the lower index wins, whichever the BVH visits first
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]] * 2, np.float32)
    sc = {"verts": v, "tris": np.array([[3, 4, 5], [0, 1, 2]], np.uint32),
          "materials": [{"type": 0}]}
    for accel in (0, 1):
        h = O.Scene(sc, accel=accel).closest_hit([0.2, 0.2, 1], [0, 0, -1])
        assert h[1] == 0 and h[0] == 1.0


def test_instances_equal_flattened_copies():
    # translate + uniform scale instances of a mesh hit exactly the primitives
    # that a flattened copy would (up to the documented FP32 transform)
    v, f = synth.icosphere(1)
    blas = {"verts": v.astype(np.float32), "tris": f.astype(np.uint32)}
    inst = [{"blas": 0, "translate": (3.0, 0.0, 0.0), "scale": 2.0},
            {"blas": 0, "translate": (-3.0, 1.0, 0.0), "scale": 0.5}]
    sc = {"verts": np.zeros((0, 3), np.float32), "tris": np.zeros((0, 3), np.uint32),
          "blas": [blas], "instances": inst, "materials": [{"type": 0}]}
    S = O.Scene(sc, accel=1)
    rng = np.random.default_rng(8)
    nhit = 0
    for _ in range(1000):
        k = rng.integers(2)
        tr, s = np.array(inst[k]["translate"]), inst[k]["scale"]
        o = np.array([0, 0, 8], np.float32)
        target = tr + _unit(rng.normal(size=3)) * s * 0.5
        d = _unit(target - o).astype(np.float32)
        h = S.closest_hit(o, d)
        assert h is not None and h[2] in (1, 2)
        # the hit point lies on the scaled sphere surface (radius s, icosphere
        # level 1 is within 10 % of the sphere)
        p = o + h[0] * d
        r = np.linalg.norm(p - np.array(inst[h[2] - 1]["translate"]))
        assert 0.85 * inst[h[2] - 1]["scale"] <= r <= 1.0001 * inst[h[2] - 1]["scale"]
        nhit += 1
    assert nhit == 1000


# ---------------------------------------------------------------- offset
def test_offset_origin_side_and_no_self_hit():
    rng = np.random.default_rng(9)
    for _ in range(2000):
        v = (rng.normal(size=(3, 3)) * rng.choice([0.01, 1, 100])).astype(np.float32)
        n = np.cross(v[1].astype(np.float64) - v[0], v[2].astype(np.float64) - v[0])
        n = (n / np.linalg.norm(n)).astype(np.float32)
        w = rng.dirichlet([2, 2, 2])
        p = (w @ v.astype(np.float64)).astype(np.float32)
        q = O.offset_origin(p, n)
        assert np.dot(q.astype(np.float64) - p, n) > 0
        assert np.abs(q.astype(np.float64) - p).max() <= 1e-3 * max(1.0, np.abs(p).max())
        # leaving into the upper hemisphere never re-hits the surface it left
        d = _unit(rng.normal(size=3))
        if np.dot(d, n) < 0:
            d = -d
        assert O.intersect_triangle(q, d.astype(np.float32), *v) is None
