"""The host BVH build through the C ABI on one thread and on all of them:
the exported node, slot and instance-record bytes are identical (the
threaded build splits work over subtrees and ranges but takes every
decision the single-threaded build takes).  Host-only contexts: no GPU."""
import numpy as np
import pytest

from paper_2305_20061_amd import npt, synth


def _soup(nt, seed=7):
    rng = np.random.default_rng(seed)
    c = rng.random((nt, 1, 3)) * np.array([100.0, 20.0, 100.0])
    v = (c + 0.2 * (rng.random((nt, 3, 3)) - 0.5)).reshape(-1, 3).astype(np.float32)
    return v, np.arange(3 * nt, dtype=np.uint32).reshape(nt, 3)


def _export(scene_fn, threads, **kw):
    c = npt.npt_create(-1)
    try:
        scene_fn(c)
        with pytest.raises(npt.NptError) as e:  # built on the host; no device to upload to
            npt.npt_build_bvh(c, threads=threads, **kw)
        assert e.value.name == "NO_DEVICE"
        return npt.npt_bvh_export(c)
    finally:
        npt.npt_destroy(c)


@pytest.mark.parametrize("width,fmt", [(4, npt.NODES_FP32), (4, npt.NODES_FP16_EXTENT), (4, npt.NODES_FP16_CORNER),
                                       (2, npt.NODES_FP32)])
def test_threaded_build_equals_single_threaded(width, fmt):
    v, t = _soup(300_000)  # subtrees of >= 100k primitives get their own threads

    def scene(c):
        npt.npt_scene_materials(c, [{"type": npt.LAMBERT, "albedo": (0.5, 0.5, 0.5)}])
        npt.npt_scene_triangles(c, v, t)

    one = _export(scene, 1, max_leaf=2, lds_levels=0, width=width, node_format=fmt)
    for threads in (0, 3):
        other = _export(scene, threads, max_leaf=2, lds_levels=0, width=width, node_format=fmt)
        for a, b in zip(one, other):
            assert a.size == b.size and np.array_equal(a, b)
    assert one[0].size > 0 and one[1].size == 300_000 * 48 and one[2].size == 0


def test_threaded_two_level_build_equals_single_threaded():
    # the large-BVH generator at a smaller size: a 385^2 terrain (294,912
    # triangles) and 48 instances of a level-5 displaced icosphere
    sc = synth.large_bvh_scene(grid=385, n_inst=48, ico_level=5)

    def scene(c):
        npt.npt_scene_materials(c, sc["materials"])
        npt.npt_scene_triangles(c, sc["verts"], sc["tris"], sc.get("tri_mat"))
        for i, b in enumerate(sc["blas"]):
            npt.npt_scene_blas_triangles(c, i, b["verts"], b["tris"], b.get("tri_mat"))
        npt.npt_scene_instances(c, sc["instances"])

    one = _export(scene, 1, max_leaf=2, lds_levels=0, width=4)
    all_ = _export(scene, 0, max_leaf=2, lds_levels=0, width=4)
    assert one[2].size > 0
    for a, b in zip(one, all_):
        assert np.array_equal(a, b)
