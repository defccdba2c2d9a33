"""CPU oracle of the neural path tracer ("Towards Neural Path Tracing in SRAM").

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg may import this package.  It wraps the plain
C oracle in ``npt_oracle.c`` (FP32 ray operations, FP64 radiance, FP64 NIF);
it shares nothing with the GPU library except the seeded inputs both sides
are handed.  See ``npt_oracle.h`` for what each function computes and the
passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpt_oracle.so")
SRC = os.path.join(HERE, "npt_oracle.c")

RNG_CAM, RNG_SCATTER, RNG_TRAIN, RNG_SCENE, RNG_SROUND = 0, 1, 2, 3, 4
LAMBERT, MIRROR, DIELECTRIC, EMITTER = 0, 1, 2, 3
ENV_MAP, ENV_NIF, ENV_CONST = 0, 1, 2
MISS = 0xFFFFFFFF


def build_oracle() -> str:
    """Compile the oracle with gcc: no FP contraction, no fast-math."""
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-fPIC", "-shared", SRC, "-o", LIB_PATH, "-lm"]
    subprocess.check_call(cmd)
    return LIB_PATH


class Material(C.Structure):
    _fields_ = [("type", C.c_uint32), ("albedo", C.c_float * 3),
                ("emission", C.c_float * 3), ("ior", C.c_float)]


class Instance(C.Structure):
    _fields_ = [("blas", C.c_uint32), ("translate", C.c_float * 3), ("scale", C.c_float)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3),
                ("up", C.c_float * 3), ("vfov_deg", C.c_float)]


class NifShape(C.Structure):
    _fields_ = [("n_freq", C.c_uint32), ("hidden", C.c_uint32), ("layers", C.c_uint32), ("colour", C.c_uint32),
                ("skip", C.c_uint32)]


class RenderDesc(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("spp", C.c_uint32),
                ("max_depth", C.c_uint32), ("rr_start", C.c_uint32), ("seed", C.c_uint64),
                ("env_mode", C.c_uint32), ("env_map", C.POINTER(C.c_float)),
                ("env_w", C.c_uint32), ("env_h", C.c_uint32),
                ("nif_params", C.POINTER(C.c_double)), ("nif", NifShape),
                ("env_const", C.c_double * 3), ("nif_prec", C.c_uint32)]


_P = C.c_void_p
_f32p = C.POINTER(C.c_float)
_f64p = C.POINTER(C.c_double)
_u32p = C.POINTER(C.c_uint32)

_lib = None


def lib():
    """The oracle library; NPT_ORACLE_LIB names another build of the same
    source to load instead (the sanitizer tests use an instrumented one)."""
    global _lib
    if _lib is None:
        path = os.environ.get("NPT_ORACLE_LIB")
        if not path:
            path = LIB_PATH
            if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
                build_oracle()
        L = C.CDLL(path)
        sig = {
            "or_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
            "or_u01": (C.c_float, [C.c_uint32]),
            "or_sincos2pi": (None, [C.c_float, _f32p, _f32p]),
            "or_intersect_triangle": (C.c_int, [_f32p, _f32p, _f32p, _f32p, _f32p, C.c_float, _f32p]),
            "or_intersect_sphere": (C.c_int, [_f32p, _f32p, _f32p, C.c_float, C.c_float, _f32p]),
            "or_offset_origin": (None, [_f32p, _f32p, _f32p]),
            "or_camera_ray": (None, [C.POINTER(Camera), C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.c_uint32, C.c_float, C.c_float, _f32p, _f32p]),
            "or_fresnel_dielectric": (C.c_float, [C.c_float, C.c_float, C.c_float]),
            "or_onb": (None, [_f32p, _f32p, _f32p]),
            "or_cosine_sample": (None, [_f32p, C.c_float, C.c_float, _f32p]),
            "or_dielectric_scatter": (C.c_int, [_f32p, _f32p, C.c_float, C.c_float, _f32p]),
            "or_dir_to_uv": (None, [C.c_double, C.c_double, C.c_double, _f64p, _f64p]),
            "or_uv_to_dir": (None, [C.c_double, C.c_double, _f64p]),
            "or_env_bilinear": (None, [_f32p, C.c_uint32, C.c_uint32, C.c_double, C.c_double, _f64p]),
            "or_nif_param_count": (C.c_uint64, [C.POINTER(NifShape)]),
            "or_nif_frequency": (C.c_uint32, [C.c_uint32]),
            "or_nif_features": (None, [C.POINTER(NifShape), C.c_double, C.c_double, _f64p]),
            "or_yuv_to_rgb_matrix": (None, [_f64p]),
            "or_colour_to_rgb_matrix": (None, [C.c_uint32, _f64p]),
            "or_nif_forward": (None, [C.POINTER(NifShape), _f64p, C.c_double, C.c_double, _f64p]),
            "or_nif_radiance": (None, [C.POINTER(NifShape), _f64p, C.c_double, C.c_double, _f64p]),
            "or_huber": (C.c_double, [C.c_double, C.c_double]),
            "or_huber_grad": (C.c_double, [C.c_double, C.c_double]),
            "or_nif_loss_grad": (C.c_double, [C.POINTER(NifShape), _f64p, C.c_uint64, _f64p, _f64p,
                                              C.c_double, _f64p]),
            "or_nif_loss_grad_q": (C.c_double, [C.POINTER(NifShape), _f64p, C.c_int, C.c_double, C.c_uint64,
                                                _f64p, _f64p, C.c_double, _f64p]),
            "or_nif_train_batch": (None, [_f32p, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32,
                                          C.c_uint64, _f64p, _f64p]),
            "or_adam_step": (None, [C.c_uint64, _f64p, _f64p, _f64p, _f64p, C.c_uint32, C.c_double,
                                    C.c_double, C.c_double, C.c_double]),
            "or_nif_train_step": (C.c_double, [C.POINTER(NifShape), _f64p, _f64p, _f64p, _f32p,
                                               C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32,
                                               C.c_uint64, C.c_double, C.c_double, C.c_double,
                                               C.c_double, C.c_double, C.c_int]),
            "or_fp16_toward_zero": (C.c_double, [C.c_double]),
            "or_fp16_stochastic": (C.c_double, [C.c_double, C.c_double]),
            "or_adam_step_fp16_master": (None, [C.c_uint64, _f64p, _f64p, _f64p, _f64p, C.c_uint32, C.c_double,
                                                C.c_double, C.c_double, C.c_double, C.c_uint64]),
            "or_scene_create": (_P, [_f32p, C.c_uint64, _u32p, C.c_uint64, _u32p, _f32p, C.c_uint64,
                                     _u32p, C.POINTER(Material), C.c_uint32, C.c_int]),
            "or_scene_add_blas": (C.c_int, [_P, _f32p, C.c_uint64, _u32p, C.c_uint64, _u32p]),
            "or_scene_set_instances": (C.c_int, [_P, C.POINTER(Instance), C.c_uint32]),
            "or_scene_destroy": (None, [_P]),
            "or_closest_hit": (C.c_int, [_P, _f32p, _f32p, C.c_float, _f32p, _u32p, _u32p, _f32p]),
            "or_render_rows": (C.c_uint64, [_P, C.POINTER(Camera), C.POINTER(RenderDesc), C.c_uint32,
                                            C.c_uint32, _f64p]),
            "or_path_sample": (None, [_P, C.POINTER(Camera), C.POINTER(RenderDesc), C.c_uint32,
                                      C.c_uint32, C.c_uint32, _f64p]),
            "or_trace_primary": (None, [_P, C.POINTER(Camera), C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint64, _u32p, _u32p, _f32p, _f32p]),
            "or_round_to": (C.c_double, [C.c_double, C.c_int]),
            "or_round_array": (None, [_f64p, _f64p, C.c_uint64, C.c_int]),
            "or_nif_fp8_scale_exp": (C.c_int, [C.c_double]),
            "or_nif_dequantize": (None, [C.POINTER(NifShape), _f64p, C.c_int, _f64p]),
            "or_nif_forward_q": (None, [C.POINTER(NifShape), _f64p, C.c_int, C.c_double, C.c_double, _f64p]),
            "or_nif_radiance_q": (None, [C.POINTER(NifShape), _f64p, C.c_int, C.c_double, C.c_double, _f64p]),
            "or_trace_pixels": (None, [_P, C.POINTER(Camera), C.c_uint32, C.c_uint32, C.c_uint32,
                                       C.c_uint64, _u32p, C.c_uint64, _u32p, _u32p, _f32p, _f32p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


# ---------------------------------------------------------------- primitives
def philox(ctr, key):
    c, k, out = u32(ctr), u32(key), np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def u01(x):
    return lib().or_u01(int(x))


def sincos2pi(u):
    s, c = C.c_float(), C.c_float()
    lib().or_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def intersect_triangle(o, d, v0, v1, v2, tmax=np.inf):
    t = C.c_float()
    args = [f32(x) for x in (o, d, v0, v1, v2)]
    h = lib().or_intersect_triangle(*[_ptr(a, C.c_float) for a in args], float(tmax), C.byref(t))
    return (t.value if h else None)


def intersect_sphere(o, d, c, r, tmax=np.inf):
    t = C.c_float()
    o, d, c = f32(o), f32(d), f32(c)
    h = lib().or_intersect_sphere(_ptr(o, C.c_float), _ptr(d, C.c_float), _ptr(c, C.c_float),
                                  float(r), float(tmax), C.byref(t))
    return (t.value if h else None)


def offset_origin(p, n):
    p, n, out = f32(p), f32(n), np.zeros(3, np.float32)
    lib().or_offset_origin(_ptr(p, C.c_float), _ptr(n, C.c_float), _ptr(out, C.c_float))
    return out


def make_camera(eye, look_at, up, vfov_deg):
    cam = Camera()
    cam.eye[:] = [float(x) for x in eye]
    cam.look_at[:] = [float(x) for x in look_at]
    cam.up[:] = [float(x) for x in up]
    cam.vfov_deg = float(vfov_deg)
    return cam


def camera_ray(cam, W, H, x, y, jx, jy):
    o, d = np.zeros(3, np.float32), np.zeros(3, np.float32)
    lib().or_camera_ray(C.byref(cam), W, H, x, y, float(jx), float(jy), _ptr(o, C.c_float),
                        _ptr(d, C.c_float))
    return o, d


def fresnel_dielectric(cos_i, eta_i, eta_t):
    return lib().or_fresnel_dielectric(float(cos_i), float(eta_i), float(eta_t))


def onb(n):
    n, t, b = f32(n), np.zeros(3, np.float32), np.zeros(3, np.float32)
    lib().or_onb(_ptr(n, C.c_float), _ptr(t, C.c_float), _ptr(b, C.c_float))
    return t, b


def cosine_sample(n, u0, u1):
    n, out = f32(n), np.zeros(3, np.float32)
    lib().or_cosine_sample(_ptr(n, C.c_float), float(u0), float(u1), _ptr(out, C.c_float))
    return out


def dielectric_scatter(d, n, ior, u):
    d, n, out = f32(d), f32(n), np.zeros(3, np.float32)
    refl = lib().or_dielectric_scatter(_ptr(d, C.c_float), _ptr(n, C.c_float), float(ior),
                                       float(u), _ptr(out, C.c_float))
    return out, bool(refl)


def dir_to_uv(d):
    u, v = C.c_double(), C.c_double()
    lib().or_dir_to_uv(float(d[0]), float(d[1]), float(d[2]), C.byref(u), C.byref(v))
    return u.value, v.value


def uv_to_dir(u, v):
    out = np.zeros(3, np.float64)
    lib().or_uv_to_dir(float(u), float(v), _ptr(out, C.c_double))
    return out


def env_bilinear(env, u, v):
    env = f32(env)
    h, w = env.shape[:2]
    out = np.zeros(3, np.float64)
    lib().or_env_bilinear(_ptr(env, C.c_float), w, h, float(u), float(v), _ptr(out, C.c_double))
    return out


# ---------------------------------------------------------------------- NIF
# output colour spaces of the network (Sec. 4.3)
COLOUR_YUV, COLOUR_RGB, COLOUR_YCOCG = 0, 1, 2


def nif_shape(n_freq=16, hidden=96, layers=5, colour=COLOUR_YUV, skip=0):
    """skip: 0, or the hidden layer (1..layers-1) whose input is the previous
    layer's output followed by the features (skip-concat); that previous layer
    has hidden - 4 n_freq outputs, so the skip layer reads hidden values."""
    s = NifShape()
    s.n_freq, s.hidden, s.layers, s.colour, s.skip = n_freq, hidden, layers, colour, skip
    return s


def nif_param_count(shape):
    return int(lib().or_nif_param_count(C.byref(shape)))


def nif_frequency(k):
    return int(lib().or_nif_frequency(k))


def nif_features(shape, u, v):
    out = np.zeros(4 * shape.n_freq, np.float64)
    lib().or_nif_features(C.byref(shape), float(u), float(v), _ptr(out, C.c_double))
    return out


def yuv_to_rgb_matrix():
    m = np.zeros(9, np.float64)
    lib().or_yuv_to_rgb_matrix(_ptr(m, C.c_double))
    return m.reshape(3, 3)


def colour_to_rgb_matrix(colour):
    m = np.zeros(9, np.float64)
    lib().or_colour_to_rgb_matrix(colour, _ptr(m, C.c_double))
    return m.reshape(3, 3)


def nif_forward(shape, params, u, v):
    p, z = f64(params), np.zeros(3, np.float64)
    lib().or_nif_forward(C.byref(shape), _ptr(p, C.c_double), float(u), float(v), _ptr(z, C.c_double))
    return z


def nif_radiance(shape, params, u, v):
    p, z = f64(params), np.zeros(3, np.float64)
    lib().or_nif_radiance(C.byref(shape), _ptr(p, C.c_double), float(u), float(v), _ptr(z, C.c_double))
    return z


PREC_FP32, PREC_FP16, PREC_BF16, PREC_FP8 = 0, 1, 2, 3
FMT_NONE, FMT_F16, FMT_BF16, FMT_E4M3 = 0, 1, 2, 3


def round_to(x, fmt):
    """Round every value to FMT_* (nearest, ties to even; E4M3 saturates)."""
    a = f64(np.atleast_1d(x))
    out = np.zeros_like(a)
    lib().or_round_array(_ptr(a, C.c_double), _ptr(out, C.c_double), a.size, int(fmt))
    return out.reshape(np.shape(x))


def nif_fp8_scale_exp(maxabs):
    return int(lib().or_nif_fp8_scale_exp(float(maxabs)))


def nif_dequantize(shape, params, prec):
    p = f64(params)
    out = np.zeros_like(p)
    lib().or_nif_dequantize(C.byref(shape), _ptr(p, C.c_double), int(prec), _ptr(out, C.c_double))
    return out


def nif_forward_q(shape, deq, prec, u, v):
    p, z = f64(deq), np.zeros(3, np.float64)
    lib().or_nif_forward_q(C.byref(shape), _ptr(p, C.c_double), int(prec), float(u), float(v),
                           _ptr(z, C.c_double))
    return z


def nif_radiance_q(shape, deq, prec, u, v):
    p, z = f64(deq), np.zeros(3, np.float64)
    lib().or_nif_radiance_q(C.byref(shape), _ptr(p, C.c_double), int(prec), float(u), float(v),
                            _ptr(z, C.c_double))
    return z


def huber(e, delta):
    return lib().or_huber(float(e), float(delta))


def huber_grad(e, delta):
    return lib().or_huber_grad(float(e), float(delta))


def _batch_chunks(n, threads):
    """Contiguous chunks [a, b) of a batch of n, one per thread."""
    k = max(1, min(int(threads), n))
    edges = [n * i // k for i in range(k + 1)]
    return [(edges[i], edges[i + 1]) for i in range(k) if edges[i + 1] > edges[i]]


def _chunked_mean(fn, n, want_grad, threads):
    """fn(a, b) -> (mean loss, mean gradient) of rows [a, b).  With threads >
    1 the chunks run on as many threads (a ctypes call releases the GIL) and
    their means are added back weighted by chunk size, in chunk order: the
    batch mean, summed in another order."""
    chunks = _batch_chunks(n, threads)
    if len(chunks) == 1:
        return fn(0, n)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(len(chunks)) as ex:
        parts = list(ex.map(lambda ab: fn(*ab), chunks))
    loss = sum(l * (b - a) for (a, b), (l, _) in zip(chunks, parts)) / n
    grad = None
    if want_grad:
        grad = np.zeros_like(parts[0][1])
        for (a, b), (_, g) in zip(chunks, parts):
            grad += g * ((b - a) / n)
    return loss, grad


def nif_loss_grad(shape, params, uv, target, delta, want_grad=True, threads=1):
    p, uv, tg = f64(params), f64(uv), f64(target)

    def run(a, b):
        g = np.zeros_like(p) if want_grad else None
        u, t = np.ascontiguousarray(uv[a:b]), np.ascontiguousarray(tg[a:b])
        loss = lib().or_nif_loss_grad(C.byref(shape), _ptr(p, C.c_double), b - a, _ptr(u, C.c_double),
                                      _ptr(t, C.c_double), float(delta),
                                      _ptr(g, C.c_double) if want_grad else None)
        return loss, g
    return _chunked_mean(run, uv.shape[0], want_grad, threads)


def nif_loss_grad_q(shape, params, prec, loss_scale, uv, target, delta, want_grad=True, threads=1):
    """Loss and gradient with the trainer's matrix operands rounded to prec
    (PREC_FP32: none), loss scale applied to the back-propagated gradients."""
    p, uv, tg = f64(params), f64(uv), f64(target)

    def run(a, b):
        g = np.zeros_like(p) if want_grad else None
        u, t = np.ascontiguousarray(uv[a:b]), np.ascontiguousarray(tg[a:b])
        loss = lib().or_nif_loss_grad_q(C.byref(shape), _ptr(p, C.c_double), int(prec), float(loss_scale),
                                        b - a, _ptr(u, C.c_double), _ptr(t, C.c_double), float(delta),
                                        _ptr(g, C.c_double) if want_grad else None)
        return loss, g
    return _chunked_mean(run, uv.shape[0], want_grad, threads)


def nif_train_batch(env, seed, step, n):
    env = f32(env)
    h, w = env.shape[:2]
    uv, tg = np.zeros((n, 2), np.float64), np.zeros((n, 3), np.float64)
    lib().or_nif_train_batch(_ptr(env, C.c_float), w, h, seed, step, n, _ptr(uv, C.c_double),
                             _ptr(tg, C.c_double))
    return uv, tg


def adam_step(params, grad, m, v, step, lr, beta1, beta2, eps):
    """In-place on params, m, v (float64 arrays); step is 1-based."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().or_adam_step(params.size, _ptr(params, C.c_double), _ptr(grad, C.c_double),
                       _ptr(m, C.c_double), _ptr(v, C.c_double), step, lr, beta1, beta2, eps)


def nif_train_step(shape, params, m, v, env, seed, step, batch, lr=1e-3, beta1=0.9,
                   beta2=0.999, eps=1e-7, delta=1e-3, fp16_master=False):
    """In-place training step on float64 params/m/v; returns the loss before it.
    fp16_master: binary16 master weights with stochastically rounded updates."""
    env = f32(env)
    h, w = env.shape[:2]
    return lib().or_nif_train_step(C.byref(shape), _ptr(params, C.c_double), _ptr(m, C.c_double),
                                   _ptr(v, C.c_double), _ptr(env, C.c_float), w, h, seed, step,
                                   batch, lr, beta1, beta2, eps, delta, int(fp16_master))


def fp16_toward_zero(x):
    return lib().or_fp16_toward_zero(float(x))


def fp16_stochastic(x, u):
    return lib().or_fp16_stochastic(float(x), float(u))


def adam_step_fp16_master(params, grad, m, v, step, seed, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-7):
    lib().or_adam_step_fp16_master(params.size, _ptr(params, C.c_double), _ptr(grad, C.c_double),
                                   _ptr(m, C.c_double), _ptr(v, C.c_double), step, lr, beta1, beta2, eps, seed)


# ------------------------------------------------------------------- scenes
def make_materials(mats):
    """mats: list of dicts {type, albedo, emission, ior}."""
    arr = (Material * max(1, len(mats)))()
    for i, m in enumerate(mats):
        arr[i].type = int(m.get("type", LAMBERT))
        arr[i].albedo[:] = [float(x) for x in m.get("albedo", (0.0, 0.0, 0.0))]
        arr[i].emission[:] = [float(x) for x in m.get("emission", (0.0, 0.0, 0.0))]
        arr[i].ior = float(m.get("ior", 1.5))
    return arr


class Scene:
    """Oracle scene: base triangles + spheres (instance 0), optional instanced
    meshes.  accel=0 brute force, 1 the oracle's median-split BVH."""

    def __init__(self, scene: dict, accel: int = 1):
        L = lib()
        self._keep = []
        verts = f32(scene.get("verts", np.zeros((0, 3))))
        tris = u32(scene.get("tris", np.zeros((0, 3))))
        tmat = u32(scene.get("tri_mat", np.zeros(len(tris))))
        sph = f32(scene.get("spheres", np.zeros((0, 4))))
        smat = u32(scene.get("sph_mat", np.zeros(len(sph))))
        mats = make_materials(scene["materials"])
        self._keep += [verts, tris, tmat, sph, smat, mats]
        self.h = L.or_scene_create(_ptr(verts, C.c_float), len(verts), _ptr(tris, C.c_uint32),
                                   len(tris), _ptr(tmat, C.c_uint32), _ptr(sph, C.c_float), len(sph),
                                   _ptr(smat, C.c_uint32), mats, len(scene["materials"]), accel)
        for blas in scene.get("blas", []):
            bv, bt = f32(blas["verts"]), u32(blas["tris"])
            bm = u32(blas.get("tri_mat", np.zeros(len(bt))))
            L.or_scene_add_blas(self.h, _ptr(bv, C.c_float), len(bv), _ptr(bt, C.c_uint32), len(bt),
                                _ptr(bm, C.c_uint32))
        inst = scene.get("instances", [])
        if len(inst):
            arr = (Instance * len(inst))()
            for i, it in enumerate(inst):
                arr[i].blas = int(it["blas"])
                arr[i].translate[:] = [float(x) for x in it["translate"]]
                arr[i].scale = float(it["scale"])
            rc = L.or_scene_set_instances(self.h, arr, len(inst))
            assert rc == 0, "instance references a missing mesh"

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_scene_destroy(self.h)
            self.h = None

    def closest_hit(self, o, d, tmax=np.inf):
        o, d = f32(o), f32(d)
        t, prim, inst, n = C.c_float(), C.c_uint32(), C.c_uint32(), np.zeros(3, np.float32)
        h = lib().or_closest_hit(self.h, _ptr(o, C.c_float), _ptr(d, C.c_float), float(tmax),
                                 C.byref(t), C.byref(prim), C.byref(inst), _ptr(n, C.c_float))
        if not h:
            return None
        return t.value, prim.value, inst.value, n


def render_desc(width, height, spp, max_depth, seed, rr_start=3, env=None, nif_params=None,
                nif=None, env_const=None, nif_prec=0):
    """nif_params: the dequantised parameters (nif_dequantize) of precision
    nif_prec (PREC_*), whose operand rounding the environment queries follow."""
    rd = RenderDesc()
    rd.width, rd.height, rd.spp, rd.max_depth, rd.rr_start, rd.seed = (
        width, height, spp, max_depth, rr_start, seed)
    keep = []
    if env_const is not None:
        rd.env_mode = ENV_CONST
        rd.env_const[:] = [float(x) for x in env_const]
    elif nif_params is not None:
        rd.env_mode = ENV_NIF
        p = f64(nif_params)
        keep.append(p)
        rd.nif_params = _ptr(p, C.c_double)
        rd.nif = nif if nif is not None else nif_shape()
        rd.nif_prec = int(nif_prec)
    else:
        rd.env_mode = ENV_MAP
        e = f32(env)
        keep.append(e)
        rd.env_map = _ptr(e, C.c_float)
        rd.env_h, rd.env_w = e.shape[:2]
    rd._keep = keep
    return rd


def render(scene: Scene, cam: Camera, rd: RenderDesc, y0=0, ystep=1):
    """FP64 image (H, W, 3); rows not in the subset are NaN."""
    out = np.full((rd.height, rd.width, 3), np.nan, np.float64)
    lib().or_render_rows(scene.h, C.byref(cam), C.byref(rd), y0, ystep, _ptr(out, C.c_double))
    return out


def path_sample(scene: Scene, cam: Camera, rd: RenderDesc, x, y, s):
    L = np.zeros(3, np.float64)
    lib().or_path_sample(scene.h, C.byref(cam), C.byref(rd), x, y, s, _ptr(L, C.c_double))
    return L


def trace_primary(scene: Scene, cam: Camera, W, H, sample, seed):
    prim = np.zeros(W * H, np.uint32)
    inst = np.zeros(W * H, np.uint32)
    t = np.zeros(W * H, np.float32)
    n = np.zeros((W * H, 3), np.float32)
    lib().or_trace_primary(scene.h, C.byref(cam), W, H, sample, seed, _ptr(prim, C.c_uint32),
                           _ptr(inst, C.c_uint32), _ptr(t, C.c_float), _ptr(n, C.c_float))
    return prim, inst, t, n


def trace_pixels(scene: Scene, cam: Camera, W, H, sample, seed, pixels):
    """trace_primary restricted to the listed pixel indices (y * W + x)."""
    px = u32(pixels)
    n = len(px)
    prim = np.zeros(n, np.uint32)
    inst = np.zeros(n, np.uint32)
    t = np.zeros(n, np.float32)
    nrm = np.zeros((n, 3), np.float32)
    lib().or_trace_pixels(scene.h, C.byref(cam), W, H, sample, seed, _ptr(px, C.c_uint32), n,
                          _ptr(prim, C.c_uint32), _ptr(inst, C.c_uint32), _ptr(t, C.c_float),
                          _ptr(nrm, C.c_float))
    return prim, inst, t, nrm
