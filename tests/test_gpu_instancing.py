"""Two-level (instanced) traversal vs the oracle: terrain plus instanced
copies of the displaced icosphere (the large-BVH scene of Fig. 1, reduced
here so the oracle finishes in seconds), first hits bit-exact in
(primitive, instance, t, normal), and a rendered image at equal seeds.  The
full-size scene is checked on a sample of pixels the oracle traces one by
one, in the configuration the benchmark uses."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import npt, synth

from gpu_util import gpu_primary, gpu_render, make_ctx, oracle_scene, rel_rmse

pytestmark = pytest.mark.gpu


def small_instanced_scene():
    return synth.large_bvh_scene(grid=193, n_inst=40, ico_level=4, size=60.0, amp=8.0)


def check_primary(scene, ctx, W, H, sample, seed):
    gp, gi, gt, gn = gpu_primary(ctx, W, H, sample, seed)
    osc, cam = oracle_scene(scene)
    op, oi, ot, on = O.trace_primary(osc, cam, W, H, sample, seed)
    same = (gp == op) & (gi == oi)
    agree = float(np.mean(same))
    hit = op != O.MISS
    print(f"sample {sample}: id agreement {agree:.6f}, instance hits {np.mean(oi[hit] > 0):.3f}")
    assert agree >= 0.9999
    assert np.array_equal(gt[same & hit], ot[same & hit])
    assert np.array_equal(gn[same & hit], on[same & hit])
    return oi


@pytest.mark.parametrize("max_leaf", [1, 2, 4])
def test_instanced_primary_hits_match_oracle(max_leaf):
    scene = small_instanced_scene()
    ctx = make_ctx(scene, max_leaf=max_leaf)
    try:
        for sample in (0, 5):
            oi = check_primary(scene, ctx, 192, 108, sample, 3)
            assert np.any(oi > 0) and np.any(oi == 0)  # both levels are exercised
    finally:
        npt.npt_destroy(ctx)


def test_instanced_env_render_matches_oracle(sky_map):
    scene = small_instanced_scene()
    ctx = make_ctx(scene, env=sky_map, max_leaf=2)
    try:
        npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        g = gpu_render(ctx, 96, 54, 2, 5, 11)
    finally:
        npt.npt_destroy(ctx)
    osc, cam = oracle_scene(scene)
    o = O.render(osc, cam, O.render_desc(96, 54, 2, 5, 11, env=sky_map))
    r = rel_rmse(g, o)
    print(f"instanced env-map relRMSE {r:.3e}")
    assert r <= 1e-3


def test_base_mesh_as_identity_instance_hits_the_same():
    # the icosphere as base geometry, and as one instance with translate 0 and
    # scale 1: the object ray equals the world ray, so every hit is identical
    # except the instance id (0 vs 1)
    bv, bt = synth.displaced_icosphere(4, seed=11)
    cam = {"eye": (0.3, 0.4, 3.0), "look_at": (0.0, 0.0, 0.0), "up": (0.0, 1.0, 0.0), "vfov_deg": 45.0}
    mats = [{"type": 0, "albedo": (0.5, 0.5, 0.5)}]
    base = {"verts": bv, "tris": bt, "materials": mats, "camera": cam}
    inst = {"blas": [{"verts": bv, "tris": bt}], "instances": [{"blas": 0, "translate": (0, 0, 0), "scale": 1.0}],
            "materials": mats, "camera": cam}
    outs = []
    for sc in (base, inst):
        ctx = make_ctx(sc, max_leaf=2)
        try:
            outs.append(gpu_primary(ctx, 128, 96, 0, 1))
        finally:
            npt.npt_destroy(ctx)
    (p0, i0, t0, n0), (p1, i1, t1, n1) = outs
    hit = p0 != O.MISS
    assert hit.mean() > 0.2
    assert np.array_equal(p0, p1) and np.array_equal(t0, t1) and np.array_equal(n0, n1)
    assert np.all(i0[hit] == 0) and np.all(i1[hit] == 1)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("node_format", [npt.NODES_FP16_EXTENT, npt.NODES_FP32, npt.NODES_Q8, npt.NODES_FP16_CORNER])
def test_large_bvh_full_size_sampled_hits_match_oracle(node_format):
    # the large-BVH workload itself (2048^2 terrain, 256 instances, leaf size
    # 2 and FP16-extent nodes as benchmarked) at 1920x1080: the GPU traces
    # every pixel, the oracle a seeded sample of 4096 of them
    scene = synth.scene_for(4)
    W, H = 1920, 1080
    ctx = make_ctx(scene, max_leaf=2, lds_levels=0, node_format=node_format)
    try:
        gp, gi, gt, gn = gpu_primary(ctx, W, H, 0, 1)
    finally:
        npt.npt_destroy(ctx)
    px = np.random.default_rng(4).choice(W * H, 4096, replace=False).astype(np.uint32)
    osc, cam = oracle_scene(scene)
    op, oi, ot, on = O.trace_pixels(osc, cam, W, H, 0, 1, px)
    same = (gp[px] == op) & (gi[px] == oi)
    hit = op != O.MISS
    print(f"full-size sample: agreement {same.mean():.6f}, hits {hit.mean():.3f}, "
          f"instance hits {np.mean(oi[hit] > 0):.3f}")
    assert same.mean() >= 0.9999
    assert np.array_equal(gt[px][same & hit], ot[same & hit])
    assert np.array_equal(gn[px][same & hit], on[same & hit])
    assert np.any(oi > 0)


def _stats_arrays(st):
    return (np.array(st["rays"], np.int64), np.array(st["node_visits"], np.int64),
            np.array(st["prim_tests"], np.int64))


@pytest.mark.parametrize("node_format", [npt.NODES_FP16_EXTENT, npt.NODES_FP32, npt.NODES_FP16_CORNER])
def test_visit_counting_build_leaves_the_image_unchanged(sky_map, node_format):
    # the counting build of the extend kernel (count_visits) traces the same
    # rays as the timed one: the image is bit-identical, every ray fetches at
    # least the root, and a node visit opens at most four leaves of at most
    # max_leaf primitives
    scene = small_instanced_scene()
    ctx = make_ctx(scene, env=sky_map, max_leaf=2, lds_levels=0, node_format=node_format)
    try:
        npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        a = gpu_render(ctx, 96, 54, 4, 6, 17)
        npt.npt_set_render_options(ctx, count_visits=1)
        b = gpu_render(ctx, 96, 54, 4, 6, 17)
        rays, nv, pt = _stats_arrays(npt.npt_get_stats(ctx))
    finally:
        npt.npt_destroy(ctx)
    assert np.array_equal(a, b)
    assert rays[0] == 96 * 54 * 4
    live = rays > 0
    assert np.all(nv[live] >= rays[live]) and np.all(pt[live] <= 4 * 2 * nv[live])
    assert np.all(nv[~live] == 0) and np.all(pt[~live] == 0)
    print("node visits per ray", nv[live] / rays[live], "primitive tests per ray", pt[live] / rays[live])


def test_visit_counts_of_a_one_triangle_scene_are_exact():
    # one triangle under the whole view: the tree is a root with one leaf
    # child, so every primary ray fetches exactly one node and tests exactly
    # one primitive
    v = np.array([[-100.0, 0.0, -100.0], [100.0, 0.0, -100.0], [0.0, 0.0, 200.0]], np.float32)
    scene = {"verts": v, "tris": np.array([[0, 2, 1]], np.uint32), "tri_mat": np.zeros(1, np.uint32),
             "materials": [synth._mat(synth.LAMBERT, (0.5, 0.5, 0.5))],
             "camera": {"eye": (0.0, 2.0, 0.0), "look_at": (0.0, 0.0, 1.0), "up": (0.0, 1.0, 0.0),
                        "vfov_deg": 40.0}}
    for fmt in (npt.NODES_FP16_EXTENT, npt.NODES_FP32, npt.NODES_FP16_CORNER):
        ctx = make_ctx(scene, max_leaf=2, lds_levels=0, node_format=fmt)
        try:
            npt.npt_set_render_options(ctx, count_visits=1)
            gpu_render(ctx, 64, 48, 2, 1, 5)
            rays, nv, pt = _stats_arrays(npt.npt_get_stats(ctx))
            gp, gi, _, _ = gpu_primary(ctx, 64, 48, 0, 5)
        finally:
            npt.npt_destroy(ctx)
        assert np.all(gp == 0)  # every primary ray hits the triangle
        assert rays[0] == 64 * 48 * 2 and nv[0] == rays[0] and pt[0] == rays[0]
        assert np.all(rays[1:] == 0)
