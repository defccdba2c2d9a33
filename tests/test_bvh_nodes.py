"""Compressed BVH4 node encodings against the FP32 nodes of the same build,
decoded here in numpy float32 arithmetic exactly as the traversal forms the
planes: every encoded child box contains the FP32 box (the conservative
rounding the closest-hit parity rests on), empty children stay empty, refs
are unchanged, and the boxes are not looser than the binary16 steps allow.
Host-only contexts: no GPU."""
import numpy as np
import pytest

from paper_2305_20061_amd import npt, synth

EMPTY = 0x7FFFFFFF


def _export(scene_fn, **kw):
    c = npt.npt_create(-1)
    try:
        scene_fn(c)
        with pytest.raises(npt.NptError) as e:  # built on the host; no device to upload to
            npt.npt_build_bvh(c, **kw)
        assert e.value.name == "NO_DEVICE"
        return npt.npt_bvh_export(c)
    finally:
        npt.npt_destroy(c)


def _soup_scene(c):
    rng = np.random.default_rng(21)
    nt = 20_000
    centre = rng.random((nt, 1, 3)) * np.array([400.0, 40.0, 400.0]) - 200.0
    size = 10.0 ** rng.uniform(-3, 1, size=(nt, 1, 1))
    v = (centre + size * (rng.random((nt, 3, 3)) - 0.5)).reshape(-1, 3).astype(np.float32)
    npt.npt_scene_materials(c, [{"type": npt.LAMBERT, "albedo": (0.5, 0.5, 0.5)}])
    npt.npt_scene_triangles(c, v, np.arange(3 * nt, dtype=np.uint32).reshape(nt, 3))


def _instanced_scene(c):
    sc = synth.large_bvh_scene(grid=129, n_inst=24, ico_level=4, size=60.0, amp=8.0)
    npt.npt_scene_materials(c, sc["materials"])
    npt.npt_scene_triangles(c, sc["verts"], sc["tris"], sc["tri_mat"])
    b = sc["blas"][0]
    npt.npt_scene_blas_triangles(c, 0, b["verts"], b["tris"], b["tri_mat"])
    npt.npt_scene_instances(c, sc["instances"])


def _fp32_boxes(nodes):
    n = nodes.view(np.float32).reshape(-1, 7, 4)
    lo = np.stack([n[:, 0], n[:, 2], n[:, 4]], 1)  # [node, axis, child]
    hi = np.stack([n[:, 1], n[:, 3], n[:, 5]], 1)
    return lo, hi, n[:, 6].view(np.uint32)


def _corner_boxes(nodes):
    raw = nodes.view(np.uint32).reshape(-1, 5, 4)
    corner = raw[:, 0, :3].view(np.float32)  # [node, axis]
    words = raw[:, 1:4]  # [node, axis, word]
    halves = np.stack([words & 0xFFFF, words >> 16], -1).astype(np.uint16)  # [node, axis, word, half]
    q = halves.view(np.float16).astype(np.float32)
    qlo = np.concatenate([q[:, :, 0], q[:, :, 1]], -1)  # children 0..3
    qhi = np.concatenate([q[:, :, 2], q[:, :, 3]], -1)
    with np.errstate(over="ignore", invalid="ignore"):
        lo = corner[:, :, None] + qlo  # one float32 rounding, as the traversal's FMA by 1
        hi = corner[:, :, None] + qhi
    return lo, hi, raw[:, 4], corner


@pytest.mark.parametrize("scene", [_soup_scene, _instanced_scene])
def test_corner_nodes_contain_the_fp32_boxes(scene):
    ref = _export(scene, max_leaf=2, lds_levels=0, width=4, node_format=npt.NODES_FP32)
    enc = _export(scene, max_leaf=2, lds_levels=0, width=4, node_format=npt.NODES_FP16_CORNER)
    assert np.array_equal(ref[1], enc[1]) and np.array_equal(ref[2], enc[2])  # slots and records
    lo32, hi32, refs32 = _fp32_boxes(ref[0])
    lo, hi, refs, corner = _corner_boxes(enc[0])
    assert lo.shape == lo32.shape and np.array_equal(refs, refs32)
    live = np.broadcast_to((refs32 != EMPTY)[:, None, :], lo32.shape)
    assert np.all(lo[live] <= lo32[live]) and np.all(hi[live] >= hi32[live])
    # empty children: a lower plane at +inf, so no ray enters them
    assert np.all(np.isinf(lo[~live]) & (lo[~live] > 0))
    # at most a few binary16 steps of the offset (plus the FP32 sum's rounding) looser
    off_lo = (lo32 - corner[:, :, None])[live]
    off_hi = (hi32 - corner[:, :, None])[live]
    slack_lo = 2.0 ** -9 * off_lo + 2 * np.spacing(np.abs(lo32[live])) + 2.0 ** -23
    slack_hi = 2.0 ** -9 * off_hi + 2 * np.spacing(np.abs(hi32[live])) + 2.0 ** -23
    assert np.all(lo32[live] - lo[live] <= slack_lo) and np.all(hi[live] - hi32[live] <= slack_hi)
    # the corner is the smallest lower plane of the node's children
    lo32_live = np.where(live, lo32, np.inf)
    assert np.array_equal(corner, lo32_live.min(-1))


def test_corner_nodes_guard_wide_nodes_and_lds_levels():
    c = npt.npt_create(-1)
    try:
        npt.npt_scene_materials(c, [{"type": npt.LAMBERT, "albedo": (0.5, 0.5, 0.5)}])
        v = np.array([[0, 0, 0], [1e5, 0, 0], [0, 1, 0]], np.float32)
        npt.npt_scene_triangles(c, v, np.array([[0, 1, 2]], np.uint32))
        for kw, code in ((dict(lds_levels=0), "UNSUPPORTED"), (dict(lds_levels=2), "INVALID_ARG")):
            with pytest.raises(npt.NptError) as e:
                npt.npt_build_bvh(c, width=4, node_format=npt.NODES_FP16_CORNER, **kw)
            assert e.value.name == code
    finally:
        npt.npt_destroy(c)
