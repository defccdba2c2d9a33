"""The C-ABI library loads and exports every function include/npt.h declares;
host-only contexts validate arguments and build BVHs without a GPU (no
compute calls here)."""
import ctypes as C

import numpy as np
import pytest

from paper_2305_20061_amd import npt, synth


@pytest.fixture(scope="module")
def L():
    return npt.lib()


def test_every_declared_function_is_exported(L):
    names = npt.header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(npt._SIGS), set(names) ^ set(npt._SIGS)


def test_header_is_plain_c():
    import re
    txt = open(npt.HEADER).read()
    code = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    assert 'extern "C"' in code
    for bad in ("torch", "hip_runtime", "std::", "template", "hipStream_t"):
        assert bad not in code


@pytest.fixture
def host_ctx():
    h = npt.npt_create(-1)
    yield h
    npt.npt_destroy(h)


def _code(fn, *a, **k):
    with pytest.raises(npt.NptError) as e:
        fn(*a, **k)
    return e.value.name


def test_host_only_validation(host_ctx):
    c = host_ctx
    v = np.zeros((3, 3), np.float32)
    v[1, 0] = 1
    v[2, 1] = 1
    assert _code(npt.npt_scene_triangles, c, v, np.array([[0, 1, 3]])) == "INVALID_ARG"
    bad = v.copy()
    bad[0, 0] = np.nan
    assert _code(npt.npt_scene_triangles, c, bad, np.array([[0, 1, 2]])) == "NAN_INPUT"
    assert _code(npt.npt_scene_spheres, c, np.array([[0, 0, 0, -1.0]])) == "INVALID_ARG"
    assert _code(npt.npt_scene_materials, c, [{"type": 9}]) == "INVALID_ARG"
    assert _code(npt.npt_build_bvh, c) == "NO_SCENE"
    assert _code(npt.npt_set_camera, c, (0, 0, 0), (0, 0, 0), (0, 1, 0), 40) == "INVALID_ARG"
    assert _code(npt.npt_set_camera, c, (0, 0, 0), (0, 0, -1), (0, 0, 1), 40) == "INVALID_ARG"
    assert _code(npt.npt_set_camera, c, (0, 0, 0), (0, 0, -1), (0, 1, 0), 180) == "INVALID_ARG"
    assert _code(npt.npt_set_env_mode, c, 5) == "INVALID_ARG"
    assert _code(npt.npt_nif_set_precision, c, 7) == "INVALID_ARG"
    assert _code(npt.npt_nif_set_precision, c, npt.FP8) == "UNSUPPORTED"
    assert _code(npt.npt_nif_upload, c, np.zeros(10)) == "INVALID_ARG"
    assert _code(npt.npt_nif_upload, c, np.zeros(43779), hidden=100) == "UNSUPPORTED"  # not a multiple of 32
    assert _code(npt.npt_nif_upload, c, np.zeros(43779), layers=9) == "UNSUPPORTED"
    assert _code(npt.npt_nif_upload, c, np.zeros(43779), hidden=128) == "INVALID_ARG"  # count of another shape
    assert npt.nif_param_count(128, 3) == 64 * 128 + 128 + 2 * (128 * 128 + 128) + 3 * 128 + 3
    assert npt.nif_param_count() == 43779
    # skip-concat: the layer before it has 128 - 64 outputs (64 fewer rows of 129)
    assert npt.nif_param_count(128, 4, 2) == npt.nif_param_count(128, 4) - 64 * 129
    assert _code(npt.npt_nif_upload, c, np.zeros(43779), skip=5) == "UNSUPPORTED"  # skip must be < layers
    assert _code(npt.npt_nif_upload, c, np.zeros(43779), n_freq=17) == "UNSUPPORTED"
    assert npt.nif_param_count(128, 4, 2, 10) == (40 * 128 + 128) + (128 * 88 + 88) + 2 * (128 * 128 + 128) + 3 * 128 + 3
    assert _code(npt.npt_nif_upload, c, np.zeros(43779), colour=3) == "INVALID_ARG"
    # training state: nothing uploaded yet
    assert _code(npt.npt_nif_get_state, c) == "STATE"
    z = np.zeros(43779, np.float32)
    assert _code(npt.npt_nif_set_state, c, z, z, z, 0) == "STATE"
    assert _code(npt.npt_env_upload, c, np.zeros((4, 8, 3))) == "NO_DEVICE"
    assert _code(npt.npt_env_upload, c, -np.ones((4, 8, 3))) == "NAN_INPUT"
    # render argument checks come before any device work
    lib = npt.lib()
    assert lib.npt_render(c, 0, 4, 1, 1, 0, C.c_void_p(1), None) == npt.NPT_E["INVALID_ARG"]
    assert lib.npt_render(c, 4, 4, 0, 1, 0, C.c_void_p(1), None) == npt.NPT_E["INVALID_ARG"]
    assert lib.npt_render(c, 4, 4, 1, 0, 0, C.c_void_p(1), None) == npt.NPT_E["INVALID_ARG"]
    assert lib.npt_render(c, 4, 4, 1, 65, 0, C.c_void_p(1), None) == npt.NPT_E["INVALID_ARG"]
    assert lib.npt_render(c, 1 << 20, 1 << 20, 1 << 20, 1, 0, C.c_void_p(1), None) == npt.NPT_E["INVALID_ARG"]
    assert lib.npt_render(c, 4, 4, 1, 1, 0, None, None) == npt.NPT_E["INVALID_ARG"]
    assert lib.npt_render(c, 4, 4, 1, 1, 0, C.c_void_p(1), None) == npt.NPT_E["NO_DEVICE"]
    assert "host-only" in npt.npt_last_error(c)
    assert lib.npt_render(None, 4, 4, 1, 1, 0, C.c_void_p(1), None) == npt.NPT_E["INVALID_ARG"]
    # progressive render: running sums required and 16-byte aligned, sample
    # indices below 2^32, then npt_render's own checks
    rs = lib.npt_render_samples
    assert rs(c, 4, 4, 0, 1, 1, 0, None, None, None) == npt.NPT_E["INVALID_ARG"]
    assert rs(c, 4, 4, 0, 1, 1, 0, C.c_void_p(8), None, None) == npt.NPT_E["INVALID_ARG"]
    assert "aligned" in npt.npt_last_error(c)
    assert rs(c, 4, 4, 0xFFFFFFFF, 1, 1, 0, C.c_void_p(16), None, None) == npt.NPT_E["INVALID_ARG"]
    assert rs(c, 4, 4, 0, 0, 1, 0, C.c_void_p(16), None, None) == npt.NPT_E["INVALID_ARG"]
    assert rs(c, 4, 4, 3, 1, 65, 0, C.c_void_p(16), None, None) == npt.NPT_E["INVALID_ARG"]
    assert rs(c, 4, 4, 3, 2, 8, 0, C.c_void_p(16), None, None) == npt.NPT_E["NO_DEVICE"]
    assert rs(None, 4, 4, 0, 1, 1, 0, C.c_void_p(16), None, None) == npt.NPT_E["INVALID_ARG"]


def test_host_only_bvh_build_and_state_survives_errors(host_ctx):
    c = host_ctx
    sc = synth.scene_for(3)
    npt.npt_scene_materials(c, sc["materials"])
    npt.npt_scene_triangles(c, sc["verts"], sc["tris"], sc["tri_mat"])
    nt = len(sc["tris"])
    for width in (2, 4):
        # built and structurally checked on the host, then no device to upload to
        assert _code(npt.npt_build_bvh, c, lds_levels=6, width=width) == "NO_DEVICE"
        info = npt.npt_bvh_info(c)
        assert info["prim_slots"] == nt and info["width"] == width
        assert nt / 4 <= info["leaves"] <= nt
        if width == 2:
            assert info["nodes"] == info["leaves"] - 1
            assert info["max_depth"] < 63
        else:
            assert (info["leaves"] - 1) / 3 <= info["nodes"] < info["leaves"]
            assert info["max_depth"] <= 21
    assert _code(npt.npt_build_bvh, c, width=3) == "INVALID_ARG"
    # a rejected upload leaves the previous scene intact
    assert _code(npt.npt_scene_triangles, c, sc["verts"], sc["tris"][:, ::-1] + 10**7) == "INVALID_ARG"
    assert _code(npt.npt_build_bvh, c, lds_levels=0) == "NO_DEVICE"
    assert npt.npt_bvh_info(c)["prim_slots"] == nt


def test_bvh_params_validated(host_ctx):
    c = host_ctx
    sc = synth.box_scene()
    npt.npt_scene_triangles(c, sc["verts"], sc["tris"], sc["tri_mat"])
    assert _code(npt.npt_build_bvh, c, bins=2) == "INVALID_ARG"
    assert _code(npt.npt_build_bvh, c, max_leaf=9) == "INVALID_ARG"
    assert _code(npt.npt_build_bvh, c, lds_levels=9) == "INVALID_ARG"
    assert _code(npt.npt_build_bvh, c, node_format=2) == "INVALID_ARG"
    assert _code(npt.npt_build_bvh, c, lds_levels=2, node_format=npt.NODES_Q8) == "INVALID_ARG"
    assert _code(npt.npt_build_bvh, c, lds_levels=0, width=2, node_format=1) == "INVALID_ARG"
    # material ids beyond the table (none uploaded -> one default material)
    assert _code(npt.npt_build_bvh, c) == "INVALID_ARG"


def test_half_extent_nodes_build_and_guard_wide_boxes(host_ctx):
    c = host_ctx
    npt.npt_scene_materials(c, [{"type": npt.LAMBERT, "albedo": (0.5, 0.5, 0.5)}])
    sc = synth.scene_for(3)
    npt.npt_scene_triangles(c, sc["verts"], sc["tris"])
    assert _code(npt.npt_build_bvh, c, lds_levels=0) == "NO_DEVICE"
    a = npt.npt_bvh_info(c)
    assert _code(npt.npt_build_bvh, c, lds_levels=0, node_format=npt.NODES_FP16_EXTENT) == "NO_DEVICE"
    b = npt.npt_bvh_info(c)
    assert a == b  # same tree, only the node encoding differs
    # a triangle wider than the binary16 range cannot be encoded
    v = np.array([[0, 0, 0], [1e5, 0, 0], [0, 1, 0]], np.float32)
    npt.npt_scene_triangles(c, v, np.array([[0, 1, 2]]))
    assert _code(npt.npt_build_bvh, c, lds_levels=0, node_format=npt.NODES_FP16_EXTENT) == "UNSUPPORTED"
    assert _code(npt.npt_build_bvh, c, lds_levels=0) == "NO_DEVICE"


def test_tiny_scenes_build(host_ctx):
    c = host_ctx
    npt.npt_scene_spheres(c, np.array([[0, 0, 0, 1.0]]))
    assert _code(npt.npt_build_bvh, c) == "NO_DEVICE"
    info = npt.npt_bvh_info(c)
    assert info["prim_slots"] == 1 and info["nodes"] == 1 and info["leaves"] == 1


def test_instances_validated_and_two_level_layout_built(host_ctx):
    c = host_ctx
    sc = synth.large_bvh_scene(grid=65, n_inst=12, ico_level=3, size=30.0, amp=4.0)
    npt.npt_scene_materials(c, sc["materials"])
    npt.npt_scene_triangles(c, sc["verts"], sc["tris"], sc["tri_mat"])
    b = sc["blas"][0]
    # ids are appended in order or replaced; instances name existing meshes
    assert _code(npt.npt_scene_blas_triangles, c, 1, b["verts"], b["tris"]) == "INVALID_ARG"
    npt.npt_scene_blas_triangles(c, 0, b["verts"], b["tris"], b["tri_mat"])
    assert _code(npt.npt_scene_instances, c, [{"blas": 1, "translate": (0, 0, 0), "scale": 1.0}]) == "INVALID_ARG"
    assert _code(npt.npt_scene_instances, c, [{"blas": 0, "translate": (0, 0, 0), "scale": 0.0}]) == "INVALID_ARG"
    assert _code(npt.npt_scene_instances, c,
                 [{"blas": 0, "translate": (0, float("nan"), 0), "scale": 1.0}]) == "NAN_INPUT"
    npt.npt_scene_instances(c, sc["instances"])
    # the two-level traversal is 4-wide; it stages its top tree's first
    # levels in LDS with binary16-extent nodes only
    assert _code(npt.npt_build_bvh, c, width=2, lds_levels=0) == "UNSUPPORTED"
    assert _code(npt.npt_build_bvh, c, width=4, lds_levels=3) == "UNSUPPORTED"
    assert _code(npt.npt_build_bvh, c, width=4, lds_levels=2, node_format=npt.NODES_FP16_EXTENT) == "NO_DEVICE"
    staged = npt.npt_bvh_export(c)
    assert _code(npt.npt_build_bvh, c, width=4, lds_levels=0, node_format=npt.NODES_FP16_EXTENT) == "NO_DEVICE"
    flat = npt.npt_bvh_export(c)
    # the same nodes (the top tree's first levels placed first), slots and records
    assert staged[0].size == flat[0].size and np.array_equal(staged[1], flat[1])
    assert np.array_equal(staged[2], flat[2])
    assert _code(npt.npt_build_bvh, c, max_leaf=2, lds_levels=0) == "NO_DEVICE"
    info = npt.npt_bvh_info(c)
    nt, nb, ni = len(sc["tris"]), len(b["tris"]), len(sc["instances"])
    # one copy of each mesh's slots, however many instances place it
    assert info["prim_slots"] == nt + nb
    assert info["width"] == 4
    # leaves: the top tree's (one per object) plus each bottom tree's
    assert ni + 1 + (nt + nb) / 2 <= info["leaves"] <= ni + 1 + nt + nb
    # removing the instances returns to the one-level tree
    npt.npt_scene_instances(c, [])
    assert _code(npt.npt_build_bvh, c, max_leaf=2, lds_levels=0) == "NO_DEVICE"
    assert npt.npt_bvh_info(c)["prim_slots"] == nt


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(npt, "_lib", None)
    monkeypatch.setattr(npt, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        npt.lib()
