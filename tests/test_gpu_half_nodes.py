"""Compressed BVH4 nodes: binary16 extents (Sec. 3.1.4's FP16-extent
proposal), 8-bit child planes on a power-of-two step, and binary16 planes on
an FP32 node corner.  Every way the
decoded planes are FP32 values the builder keeps outside the true boxes, so
the traversal may visit more but never drops a primitive.  The closest hit
is defined over all primitives (ties to the lowest id), so first hits match
the oracle bit for bit and renders are identical to those of the FP32-node
tree, one- and two-level."""
import numpy as np
import pytest

import oracle as O
from paper_2305_20061_amd import npt, synth

from gpu_util import gpu_primary, gpu_render, make_ctx, oracle_scene, rel_rmse
from test_gpu_instancing import check_primary, small_instanced_scene

pytestmark = pytest.mark.gpu
FORMATS = [npt.NODES_FP16_EXTENT, npt.NODES_Q8, npt.NODES_FP16_CORNER]


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("cfg,W,H", [(0, 128, 128), (1, 96, 96), (2, 160, 120), (3, 192, 108)])
def test_half_node_primary_hits_match_oracle(cfg, W, H, fmt):
    scene = synth.scene_for(cfg)
    ctx = make_ctx(scene, lds_levels=0, node_format=fmt)
    try:
        for sample in (0, 3):
            gp, gi, gt, gn = gpu_primary(ctx, W, H, sample, seed=1)
            osc, cam = oracle_scene(scene)
            op, oi, ot, on = O.trace_primary(osc, cam, W, H, sample, 1)
            agree = np.mean(gp == op)
            print(f"node format {fmt}, cfg {cfg} sample {sample}: id agreement {agree:.6f}")
            assert agree >= 0.9999
            same = (gp == op) & (op != O.MISS)
            assert np.array_equal(gt[same], ot[same])
            assert np.array_equal(gn[same], on[same])
    finally:
        npt.npt_destroy(ctx)


@pytest.mark.parametrize("fmt", FORMATS)
def test_half_node_instanced_primary_hits_match_oracle(fmt):
    scene = small_instanced_scene()
    ctx = make_ctx(scene, max_leaf=2, node_format=fmt)
    try:
        for sample in (0, 5):
            oi = check_primary(scene, ctx, 192, 108, sample, 3)
            assert np.any(oi > 0) and np.any(oi == 0)
    finally:
        npt.npt_destroy(ctx)


@pytest.mark.parametrize("cfg", [2, 3, "instanced"])
def test_half_node_renders_equal_fp32_node_renders(cfg, sky_map):
    scene = small_instanced_scene() if cfg == "instanced" else synth.scene_for(cfg)
    imgs = []
    for fmt in [npt.NODES_FP32] + FORMATS:
        ctx = make_ctx(scene, env=sky_map, lds_levels=0, max_leaf=2, node_format=fmt)
        try:
            npt.npt_set_env_mode(ctx, npt.ENV_MAP)
            imgs.append(gpu_render(ctx, 96, 64, 2, 6, 5))
        finally:
            npt.npt_destroy(ctx)
    for k, fmt in enumerate(FORMATS):
        print(f"cfg {cfg}: node format {fmt} vs FP32 nodes max |diff| {np.abs(imgs[0] - imgs[k + 1]).max():.3e}")
        assert np.array_equal(imgs[0], imgs[k + 1])


@pytest.mark.parametrize("fmt", FORMATS)
def test_half_node_env_render_matches_oracle(fmt, sky_map):
    scene = synth.scene_for(2)
    ctx = make_ctx(scene, env=sky_map, lds_levels=0, node_format=fmt)
    try:
        npt.npt_set_env_mode(ctx, npt.ENV_MAP)
        g = gpu_render(ctx, 96, 72, 4, 8, 2)
    finally:
        npt.npt_destroy(ctx)
    osc, cam = oracle_scene(scene)
    o = O.render(osc, cam, O.render_desc(96, 72, 4, 8, 2, env=sky_map))
    r = rel_rmse(g, o)
    print(f"FP16-extent nodes env-map relRMSE {r:.3e}")
    assert r <= 1e-3


@pytest.mark.parametrize("cfg", [3, "instanced"])
def test_lds_staged_half_nodes_match_oracle_and_unstaged(cfg, sky_map):
    # the first levels of the tree (of an instanced scene: of its top tree),
    # binary16-extent nodes, read from the workgroup's LDS copy: first hits
    # bit for bit as the oracle's, and the image of the unstaged tree
    scene = small_instanced_scene() if cfg == "instanced" else synth.scene_for(cfg)
    imgs = []
    for lds in (0, 2):
        ctx = make_ctx(scene, env=sky_map, lds_levels=lds, max_leaf=2, node_format=npt.NODES_FP16_EXTENT)
        try:
            if lds:
                if cfg == "instanced":
                    oi = check_primary(scene, ctx, 192, 108, 1, 3)
                    assert np.any(oi > 0)
                else:
                    gp, gi, gt, gn = gpu_primary(ctx, 192, 108, 1, seed=3)
                    osc, cam = oracle_scene(scene)
                    op, oi, ot, on = O.trace_primary(osc, cam, 192, 108, 1, 3)
                    same = (gp == op) & (op != O.MISS)
                    print(f"cfg {cfg} staged: id agreement {np.mean(gp == op):.6f}")
                    assert np.mean(gp == op) >= 0.9999
                    assert np.array_equal(gt[same], ot[same])
            npt.npt_set_env_mode(ctx, npt.ENV_MAP)
            imgs.append(gpu_render(ctx, 96, 64, 2, 6, 5))
        finally:
            npt.npt_destroy(ctx)
    assert np.array_equal(imgs[0], imgs[1])
