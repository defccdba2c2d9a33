"""Python binding of libnpt (include/npt.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Device buffers
are torch.cuda tensors (their data pointers are passed); host arrays are
numpy arrays.  A non-zero status raises NptError with npt_last_error().
There is no fallback: without the built libnpt.so this module raises on
import of the library.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnpt.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "npt.h")

NPT_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "NO_SCENE", -3: "NO_ENV", -4: "OOM", -5: "HIP", -6: "UNSUPPORTED",
          -7: "NAN_INPUT", -8: "NO_DEVICE", -9: "STATE"}
NPT_E = {v: k for k, v in ERRORS.items()}
LAMBERT, MIRROR, DIELECTRIC, EMITTER = 0, 1, 2, 3
ENV_MAP, ENV_NIF, ENV_NONE = 0, 1, 2
NODES_FP32, NODES_FP16_EXTENT, NODES_Q8, NODES_FP16_CORNER = 0, 1, 2, 3
COLOUR_YUV, COLOUR_RGB, COLOUR_YCOCG = 0, 1, 2
FP32, FP16, BF16, FP8 = 0, 1, 2, 3
MAX_DEPTH = 64
MISS = 0xFFFFFFFF


class NptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class npt_material(C.Structure):
    _fields_ = [("type", C.c_uint32), ("albedo", C.c_float * 3), ("emission", C.c_float * 3),
                ("ior", C.c_float)]


class npt_instance(C.Structure):
    _fields_ = [("blas_id", C.c_uint32), ("translate", C.c_float * 3), ("scale", C.c_float)]


class npt_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float)]


class npt_bvh_params(C.Structure):
    _fields_ = [("bins", C.c_uint32), ("max_leaf", C.c_uint32), ("lds_levels", C.c_uint32), ("width", C.c_uint32),
                ("node_format", C.c_uint32), ("threads", C.c_uint32)]


class npt_nif_desc(C.Structure):
    _fields_ = [("n_freq", C.c_uint32), ("hidden", C.c_uint32), ("layers", C.c_uint32), ("colour", C.c_uint32),
                ("layered", C.c_uint32), ("skip", C.c_uint32)]


class npt_train_params(C.Structure):
    _fields_ = [("batch", C.c_uint32), ("samples", C.c_uint64), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("huber_delta", C.c_float), ("seed", C.c_uint64),
                ("grad_prec", C.c_uint32), ("loss_scale", C.c_float), ("master_prec", C.c_uint32),
                ("path", C.c_uint32)]


class npt_train_stats(C.Structure):
    _fields_ = [("steps", C.c_uint32), ("step_total", C.c_uint32), ("first_loss", C.c_float),
                ("last_loss", C.c_float), ("ms", C.c_float)]


class npt_render_options(C.Structure):
    _fields_ = [("rr_start", C.c_uint32), ("samples_per_pass", C.c_uint32), ("pool_paths", C.c_uint32),
                ("kernel_timing", C.c_uint32), ("count_visits", C.c_uint32), ("sort_rays", C.c_uint32)]


class npt_stats(C.Structure):
    _fields_ = [("paths", C.c_uint64), ("rays", C.c_uint64 * MAX_DEPTH), ("escaped", C.c_uint64 * MAX_DEPTH),
                ("env_queries", C.c_uint64), ("passes", C.c_uint32), ("samples_per_pass", C.c_uint32),
                ("ms_total", C.c_float), ("ms_trace", C.c_float), ("ms_env", C.c_float),
                ("trace_launches", C.c_uint32), ("env_launches", C.c_uint32),
                ("node_visits", C.c_uint64 * MAX_DEPTH), ("prim_tests", C.c_uint64 * MAX_DEPTH),
                ("ms_shade", C.c_float), ("shade_launches", C.c_uint32), ("ms_env_depth", C.c_float * MAX_DEPTH)]


_P = C.c_void_p
_SIGS = {
    "npt_create": [C.POINTER(_P), C.c_int],
    "npt_destroy": [_P],
    "npt_last_error": [_P],
    "npt_scene_triangles": [_P, _P, C.c_uint64, _P, C.c_uint64, _P],
    "npt_scene_spheres": [_P, _P, C.c_uint64, _P],
    "npt_scene_blas_triangles": [_P, C.c_uint32, _P, C.c_uint64, _P, C.c_uint64, _P],
    "npt_scene_instances": [_P, _P, C.c_uint32],
    "npt_scene_materials": [_P, _P, C.c_uint32],
    "npt_build_bvh": [_P, _P, _P],
    "npt_bvh_info": [_P, _P, _P, _P, _P, _P],
    "npt_bvh_export": [_P, _P, _P, _P, _P, _P, _P],
    "npt_set_camera": [_P, _P],
    "npt_set_render_options": [_P, _P],
    "npt_env_upload": [_P, _P, C.c_uint32, C.c_uint32, _P],
    "npt_set_env_mode": [_P, C.c_int],
    "npt_nif_upload": [_P, _P, _P, C.c_uint64, _P],
    "npt_nif_download": [_P, _P, C.c_uint64],
    "npt_nif_get_state": [_P, _P, _P, _P, C.c_uint64, _P],
    "npt_nif_set_state": [_P, _P, _P, _P, C.c_uint64, C.c_uint32, _P],
    "npt_nif_set_precision": [_P, C.c_int],
    "npt_nif_get_dequantized": [_P, _P, C.c_uint64],
    "npt_nif_train": [_P, _P, _P, _P],
    "npt_nif_train_grad": [_P, _P, C.c_uint32, _P, _P, _P],
    "npt_nif_eval_grid": [_P, C.c_uint32, C.c_uint32, _P, _P],
    "npt_env_query": [_P, C.c_int, _P, C.c_uint64, _P, _P],
    "npt_render": [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, _P, _P],
    "npt_render_noalloc": [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, _P, _P],
    "npt_render_samples": [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, _P, _P, _P],
    "npt_trace_primary": [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, _P, _P, _P, _P, _P],
    "npt_get_stats": [_P, _P],
}

_lib = None


def header_functions() -> list[str]:
    """Names of every function declared in include/npt.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(npt_\w+)\s*\(", txt, re.M)))


def lib():
    """The loaded libnpt.so; raises if it was not built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
        # torch ships its own HIP runtime under the same soname; load it first
        # so that libnpt and torch share one runtime (and one device context)
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_char_p if name == "npt_last_error" else C.c_int
        _lib = L
    return _lib


def _check(ctx, rc):
    if rc != NPT_OK:
        msg = lib().npt_last_error(ctx) if ctx else b""
        raise NptError(rc, (msg or b"").decode())
    return rc


def _host(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _hp(a):
    return None if a is None else a.ctypes.data_as(_P)


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return _P(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


def _dev(t, dtype=None, numel=None):
    """Data pointer of a contiguous CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise TypeError("device buffer must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("device buffer must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"device buffer must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"device buffer has {t.numel()} elements, needs {numel}")
    return _P(t.data_ptr())


# ------------------------------------------------------------------ context
def npt_create(device: int = 0):
    h = _P()
    _check(None, lib().npt_create(C.byref(h), device))
    return h


def npt_destroy(ctx):
    _check(None, lib().npt_destroy(ctx))


def npt_last_error(ctx) -> str:
    return (lib().npt_last_error(ctx) or b"").decode()


# -------------------------------------------------------------------- scene
def npt_scene_triangles(ctx, xyz, tri, mat_of_tri=None):
    v, t, m = _host(xyz, np.float32), _host(tri, np.uint32), _host(mat_of_tri, np.uint32)
    _check(ctx, lib().npt_scene_triangles(ctx, _hp(v), v.size // 3, _hp(t), t.size // 3, _hp(m)))


def npt_scene_spheres(ctx, cxyzr, mat=None):
    s, m = _host(cxyzr, np.float32), _host(mat, np.uint32)
    _check(ctx, lib().npt_scene_spheres(ctx, _hp(s), s.size // 4, _hp(m)))


def npt_scene_blas_triangles(ctx, blas_id, xyz, tri, mat_of_tri=None):
    v, t, m = _host(xyz, np.float32), _host(tri, np.uint32), _host(mat_of_tri, np.uint32)
    _check(ctx, lib().npt_scene_blas_triangles(ctx, blas_id, _hp(v), v.size // 3, _hp(t), t.size // 3, _hp(m)))


def npt_scene_instances(ctx, instances):
    arr = (npt_instance * max(1, len(instances)))()
    for i, it in enumerate(instances):
        arr[i].blas_id = int(it["blas"])
        arr[i].translate[:] = [float(x) for x in it["translate"]]
        arr[i].scale = float(it["scale"])
    _check(ctx, lib().npt_scene_instances(ctx, arr, len(instances)))


def npt_scene_materials(ctx, materials):
    arr = (npt_material * max(1, len(materials)))()
    for i, m in enumerate(materials):
        arr[i].type = int(m.get("type", LAMBERT))
        arr[i].albedo[:] = [float(x) for x in m.get("albedo", (0, 0, 0))]
        arr[i].emission[:] = [float(x) for x in m.get("emission", (0, 0, 0))]
        arr[i].ior = float(m.get("ior", 1.5))
    _check(ctx, lib().npt_scene_materials(ctx, arr, len(materials)))


def npt_build_bvh(ctx, bins=32, max_leaf=4, lds_levels=6, stream=None, width=0, node_format=0, threads=0):
    p = npt_bvh_params(bins, max_leaf, lds_levels, width, node_format, threads)
    _check(ctx, lib().npt_build_bvh(ctx, C.byref(p), _stream(stream)))


def npt_bvh_export(ctx):
    """(nodes, slots, records) of the host-built BVH as byte arrays."""
    sz = [C.c_uint64() for _ in range(3)]
    _check(ctx, lib().npt_bvh_export(ctx, None, C.byref(sz[0]), None, C.byref(sz[1]), None, C.byref(sz[2])))
    bufs = [np.zeros(s.value, np.uint8) for s in sz]
    _check(ctx, lib().npt_bvh_export(ctx, _hp(bufs[0]), C.byref(sz[0]), _hp(bufs[1]), C.byref(sz[1]),
                                     _hp(bufs[2]), C.byref(sz[2])))
    return tuple(bufs)


def npt_bvh_info(ctx):
    n, lv, s = C.c_uint64(), C.c_uint64(), C.c_uint64()
    d = C.c_uint32()
    w = C.c_uint32()
    _check(ctx, lib().npt_bvh_info(ctx, C.byref(n), C.byref(lv), C.byref(d), C.byref(s), C.byref(w)))
    return {"nodes": n.value, "leaves": lv.value, "max_depth": d.value, "prim_slots": s.value, "width": w.value}


def npt_set_camera(ctx, eye, look_at, up, vfov_deg):
    cam = npt_camera()
    cam.eye[:] = [float(x) for x in eye]
    cam.look_at[:] = [float(x) for x in look_at]
    cam.up[:] = [float(x) for x in up]
    cam.vfov_deg = float(vfov_deg)
    _check(ctx, lib().npt_set_camera(ctx, C.byref(cam)))


def npt_set_render_options(ctx, rr_start=3, samples_per_pass=0, pool_paths=0, kernel_timing=0, count_visits=0,
                           sort_rays=0):
    o = npt_render_options(rr_start, samples_per_pass, pool_paths, kernel_timing, count_visits, sort_rays)
    _check(ctx, lib().npt_set_render_options(ctx, C.byref(o)))


# -------------------------------------------------------------- environment
def npt_env_upload(ctx, rgb, stream=None):
    e = _host(rgb, np.float32)
    h, w = e.shape[:2]
    _check(ctx, lib().npt_env_upload(ctx, _hp(e), w, h, _stream(stream)))


def npt_set_env_mode(ctx, mode):
    _check(ctx, lib().npt_set_env_mode(ctx, mode))


# ---------------------------------------------------------------------- NIF
def nif_param_count(hidden=96, layers=5, skip=0, n_freq=16):
    """With a skip-concat the layer before it has hidden - 4 n_freq outputs."""
    F = 4 * n_freq
    return (F * hidden + hidden + (layers - 1) * (hidden * hidden + hidden) + 3 * hidden + 3
            - (F * (hidden + 1) if skip else 0))


def npt_nif_upload(ctx, params, n_freq=16, hidden=96, layers=5, stream=None, colour=0, layered=0, skip=0):
    p = _host(params, np.float32)
    d = npt_nif_desc(n_freq, hidden, layers, colour, layered, skip)
    _check(ctx, lib().npt_nif_upload(ctx, C.byref(d), _hp(p), p.size, _stream(stream)))


def npt_nif_download(ctx, n=43779):
    out = np.zeros(n, np.float32)
    _check(ctx, lib().npt_nif_download(ctx, _hp(out), n))
    return out


def npt_nif_get_state(ctx, n=43779):
    """(params, m, v, step): FP32 master parameters, Adam moments, Adam steps taken."""
    p, m, v = (np.zeros(n, np.float32) for _ in range(3))
    step = C.c_uint32(0)
    _check(ctx, lib().npt_nif_get_state(ctx, _hp(p), _hp(m), _hp(v), n, C.byref(step)))
    return p, m, v, int(step.value)


def npt_nif_set_state(ctx, params, m, v, step, stream=None):
    p, mm, vv = (_host(a, np.float32) for a in (params, m, v))
    if not (p.size == mm.size == vv.size):
        raise ValueError("params, m and v must have the same length")
    _check(ctx, lib().npt_nif_set_state(ctx, _hp(p), _hp(mm), _hp(vv), p.size, int(step), _stream(stream)))


def npt_nif_set_precision(ctx, prec):
    _check(ctx, lib().npt_nif_set_precision(ctx, prec))


def npt_nif_get_dequantized(ctx, n=43779):
    out = np.zeros(n, np.float32)
    _check(ctx, lib().npt_nif_get_dequantized(ctx, _hp(out), n))
    return out


TRAIN_AUTO, TRAIN_LAYERED = 0, 1  # npt_train_params.path


def train_params(batch=0, samples=0, lr=0.0, beta1=0.0, beta2=0.0, eps=0.0, huber_delta=0.0, seed=0,
                 grad_prec=FP32, loss_scale=0.0, master_prec=FP32, path=TRAIN_AUTO):
    return npt_train_params(batch, samples, lr, beta1, beta2, eps, huber_delta, seed, grad_prec, loss_scale,
                            master_prec, path)


def npt_nif_train(ctx, params: npt_train_params = None, stream=None):
    st = npt_train_stats()
    p = params if params is not None else train_params()
    _check(ctx, lib().npt_nif_train(ctx, C.byref(p), C.byref(st), _stream(stream)))
    return {"steps": st.steps, "step_total": st.step_total, "first_loss": st.first_loss,
            "last_loss": st.last_loss, "ms": st.ms}


def npt_nif_train_grad(ctx, params: npt_train_params, step, grad_out, loss_out, stream=None, n_params=43779):
    """n_params: parameter count of the uploaded network (nif_param_count)."""
    import torch
    _check(ctx, lib().npt_nif_train_grad(ctx, C.byref(params), step, _dev(grad_out, torch.float32, n_params),
                                         _dev(loss_out, torch.float32, 1), _stream(stream)))


def npt_nif_eval_grid(ctx, gw, gh, stream=None):
    out = (C.c_float * 2)()
    _check(ctx, lib().npt_nif_eval_grid(ctx, gw, gh, out, _stream(stream)))
    return {"log_mse": out[0], "psnr_log": out[1]}


def npt_env_query(ctx, mode, dirs, rgb_out, stream=None):
    import torch
    n = dirs.numel() // 3
    _check(ctx, lib().npt_env_query(ctx, mode, _dev(dirs, torch.float32), n, _dev(rgb_out, torch.float32, 3 * n),
                                    _stream(stream)))


# ---------------------------------------------------------------- rendering
def npt_render(ctx, width, height, spp, max_depth, seed, out, stream=None):
    import torch
    _check(ctx, lib().npt_render(ctx, width, height, spp, max_depth, seed,
                                 _dev(out, torch.float32, width * height * 3), _stream(stream)))


def npt_render_samples(ctx, width, height, sample0, samples, max_depth, seed, sums, out=None, stream=None):
    """Adds samples [sample0, sample0 + samples) to the running sums [H, W, 4]
    (overwritten when sample0 == 0); `out`, when given, gets the mean so far."""
    import torch
    n = width * height
    _check(ctx, lib().npt_render_samples(ctx, width, height, sample0, samples, max_depth, seed,
                                         _dev(sums, torch.float32, 4 * n), _dev(out, torch.float32, 3 * n),
                                         _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # NPT_NOALLOC_SCRATCH_BYTES


def npt_render_noalloc(ctx, width, height, spp, max_depth, seed, out, stream=None):
    """npt_render on the library's fixed device scratch (no allocation)."""
    import torch
    _check(ctx, lib().npt_render_noalloc(ctx, width, height, spp, max_depth, seed,
                                         _dev(out, torch.float32, width * height * 3), _stream(stream)))


def npt_trace_primary(ctx, width, height, sample, seed, prim=None, inst=None, t=None, normal=None, stream=None):
    import torch
    n = width * height
    _check(ctx, lib().npt_trace_primary(ctx, width, height, sample, seed, _dev(prim, torch.int32, n),
                                        _dev(inst, torch.int32, n), _dev(t, torch.float32, n),
                                        _dev(normal, torch.float32, 3 * n), _stream(stream)))


def npt_get_stats(ctx):
    s = npt_stats()
    _check(ctx, lib().npt_get_stats(ctx, C.byref(s)))
    return {"paths": s.paths, "rays": list(s.rays), "escaped": list(s.escaped), "env_queries": s.env_queries,
            "passes": s.passes, "samples_per_pass": s.samples_per_pass, "ms_total": s.ms_total,
            "ms_trace": s.ms_trace, "ms_env": s.ms_env, "trace_launches": s.trace_launches,
            "env_launches": s.env_launches, "node_visits": list(s.node_visits), "prim_tests": list(s.prim_tests),
            "ms_shade": s.ms_shade, "shade_launches": s.shade_launches, "ms_env_depth": list(s.ms_env_depth)}


# ------------------------------------------------------------ conveniences
def npt_load_scene(ctx, scene: dict, bins=32, max_leaf=4, lds_levels=6, stream=None, width=0, node_format=0,
                   threads=0):
    """Uploads a scene dict (paper_2305_20061_amd.synth layout) and builds its BVH."""
    npt_scene_materials(ctx, scene["materials"])
    if len(scene.get("tris", [])):
        npt_scene_triangles(ctx, scene["verts"], scene["tris"], scene.get("tri_mat"))
    if len(scene.get("spheres", [])):
        npt_scene_spheres(ctx, scene["spheres"], scene.get("sph_mat"))
    for i, b in enumerate(scene.get("blas", [])):
        npt_scene_blas_triangles(ctx, i, b["verts"], b["tris"], b.get("tri_mat"))
    if scene.get("instances"):
        npt_scene_instances(ctx, scene["instances"])
    cam = scene["camera"]
    npt_set_camera(ctx, cam["eye"], cam["look_at"], cam["up"], cam["vfov_deg"])
    if node_format in (NODES_Q8, NODES_FP16_CORNER) or (scene.get("instances") and node_format != NODES_FP16_EXTENT):
        lds_levels = 0  # LDS staging: FP32 one-level trees and binary16-extent trees only
    npt_build_bvh(ctx, bins, max_leaf, lds_levels, stream, width, node_format, threads)
