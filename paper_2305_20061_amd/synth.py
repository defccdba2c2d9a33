"""Seeded synthetic inputs: scenes, the HDR environment map, initial NIF weights.

This module only *makes inputs*.  It holds none of the renderer's arithmetic
(no intersection, sampling, lookup or network evaluation); both the GPU
library and the CPU oracle are handed what it returns.  The scenes are shaped
like the paper's five test scenes (Fig. 1, Table 2): a Cornell-style box, the
same box opened to the environment, a field of spheres, a small displaced
mesh and a large terrain with instanced meshes.  The paper's Polyhaven HDRIs
are replaced by a synthetic sky with a sun (Sec. 3.2, Table 4 discusses a
sun-lit map).

Scene dict layout (shared by the binding and the oracle wrapper):
  verts (nv,3) f32, tris (nt,3) u32, tri_mat (nt,) u32,
  spheres (ns,4) f32 (cx,cy,cz,r), sph_mat (ns,) u32,
  materials: list of {type, albedo, emission, ior},
  blas: list of {verts, tris, tri_mat}  (object-space meshes for instancing),
  instances: list of {blas, translate, scale},
  camera: {eye, look_at, up, vfov_deg}.
"""
from __future__ import annotations

import math

import numpy as np

LAMBERT, MIRROR, DIELECTRIC, EMITTER = 0, 1, 2, 3


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def _mat(type_, albedo=(0.0, 0.0, 0.0), emission=(0.0, 0.0, 0.0), ior=1.5):
    return {"type": type_, "albedo": tuple(float(a) for a in albedo),
            "emission": tuple(float(e) for e in emission), "ior": float(ior)}


class _Mesh:
    def __init__(self):
        self.v, self.t, self.m = [], [], []

    def quad(self, p0, p1, p2, p3, mat):
        """Quad p0..p3 counter-clockwise seen from the side its normal faces."""
        b = len(self.v)
        self.v += [p0, p1, p2, p3]
        self.t += [(b, b + 1, b + 2), (b, b + 2, b + 3)]
        self.m += [mat, mat]

    def arrays(self):
        return (np.asarray(self.v, np.float32).reshape(-1, 3),
                np.asarray(self.t, np.uint32).reshape(-1, 3),
                np.asarray(self.m, np.uint32))


# --------------------------------------------------------------------------
# Box scenes (Fig. 1a/1b): 12 axis-aligned wall triangles plus a quad light
# --------------------------------------------------------------------------
def box_scene(open_front: bool = False, light_radiance: float = 15.0):
    """Box x in [-1,1], y in [0,2], z in [-1,1]; walls face inward.

    Materials: 0 white 0.75, 1 red (0.75,0,0), 2 green (0,0.75,0),
    3 light (emitter, albedo 0).  The light quad hangs 2e-3 (1e-3 of the box
    size) under the ceiling and faces down, so it never shares a plane with a
    wall.  open_front removes the z = +1 wall (12 -> 10 wall triangles +2
    light)."""
    m = _Mesh()
    W, R, G, Lm = 0, 1, 2, 3
    # floor y=0, normal +y
    m.quad((-1, 0, -1), (-1, 0, 1), (1, 0, 1), (1, 0, -1), W)
    # ceiling y=2, normal -y
    m.quad((-1, 2, -1), (1, 2, -1), (1, 2, 1), (-1, 2, 1), W)
    # back wall z=-1, normal +z
    m.quad((-1, 0, -1), (1, 0, -1), (1, 2, -1), (-1, 2, -1), W)
    # left wall x=-1 (red), normal +x
    m.quad((-1, 0, -1), (-1, 2, -1), (-1, 2, 1), (-1, 0, 1), R)
    # right wall x=+1 (green), normal -x
    m.quad((1, 0, -1), (1, 0, 1), (1, 2, 1), (1, 2, -1), G)
    if not open_front:
        # front wall z=+1, normal -z
        m.quad((-1, 0, 1), (-1, 2, 1), (1, 2, 1), (1, 0, 1), W)
    # light quad, normal -y
    y = 2.0 - 2e-3
    m.quad((-0.25, y, -0.6), (0.25, y, -0.6), (0.25, y, -0.1), (-0.25, y, -0.1), Lm)
    v, t, mt = m.arrays()
    mats = [_mat(LAMBERT, (0.75, 0.75, 0.75)), _mat(LAMBERT, (0.75, 0.0, 0.0)),
            _mat(LAMBERT, (0.0, 0.75, 0.0)),
            _mat(EMITTER, (0.0, 0.0, 0.0), (light_radiance,) * 3)]
    if open_front:
        cam = {"eye": (0.0, 1.0, 3.6), "look_at": (0.0, 1.0, 0.0), "up": (0.0, 1.0, 0.0),
               "vfov_deg": 40.0}
    else:
        cam = {"eye": (0.0, 1.0, 0.95), "look_at": (0.0, 1.2, -1.0), "up": (0.0, 1.0, 0.0),
               "vfov_deg": 80.0}
    return {"verts": v, "tris": t, "tri_mat": mt, "materials": mats, "camera": cam}


# --------------------------------------------------------------------------
# Spheres (Fig. 1c): 64 spheres on a 20 x 20 ground quad
# --------------------------------------------------------------------------
def spheres_scene(seed: int = 7, n: int = 64):
    """Non-overlapping spheres (rejection sampling, <= 1000 tries each) resting
    on the ground (centre y = r), radii U(0.2, 1.0); materials 60 % Lambertian
    (albedo U(0.2,0.9)^3), 25 % mirror (reflectance 1), 15 % dielectric (IOR
    1.5); ground Lambertian 0.5 (two triangles)."""
    rng = _rng(seed)
    spheres, smat = [], []
    mats = [_mat(LAMBERT, (0.5, 0.5, 0.5))]
    tries = 0
    while len(spheres) < n and tries < 1000 * n:
        tries += 1
        r = rng.uniform(0.2, 1.0)
        x, z = rng.uniform(-10 + r, 10 - r, size=2)
        ok = all((x - s[0]) ** 2 + (z - s[2]) ** 2 + (r - s[1]) ** 2 > (r + s[3]) ** 2
                 for s in spheres)
        if not ok:
            continue
        c = rng.uniform()
        if c < 0.60:
            mats.append(_mat(LAMBERT, rng.uniform(0.2, 0.9, size=3)))
        elif c < 0.85:
            mats.append(_mat(MIRROR, (1.0, 1.0, 1.0)))
        else:
            mats.append(_mat(DIELECTRIC, (1.0, 1.0, 1.0), ior=1.5))
        spheres.append((x, r, z, r))
        smat.append(len(mats) - 1)
    m = _Mesh()
    m.quad((-10, 0, -10), (-10, 0, 10), (10, 0, 10), (10, 0, -10), 0)
    v, t, mt = m.arrays()
    cam = {"eye": (0.0, 5.0, 17.0), "look_at": (0.0, 0.6, 0.0), "up": (0.0, 1.0, 0.0),
           "vfov_deg": 45.0}
    return {"verts": v, "tris": t, "tri_mat": mt, "spheres": np.asarray(spheres, np.float32),
            "sph_mat": np.asarray(smat, np.uint32), "materials": mats, "camera": cam}


# --------------------------------------------------------------------------
# Value noise (lattice noise with smoothstep interpolation)
# --------------------------------------------------------------------------
class _ValueNoise:
    def __init__(self, seed: int, size: int = 256):
        rng = _rng(seed)
        self.perm = rng.permutation(size).astype(np.int64)
        self.vals = rng.uniform(0.0, 1.0, size)
        self.size = size

    def _h(self, *ix):
        h = np.zeros_like(ix[0])
        for a in ix:
            h = self.perm[(h + a) % self.size]
        return self.vals[h]

    def noise3(self, p):
        p = np.asarray(p, np.float64)
        i = np.floor(p).astype(np.int64)
        f = p - i
        w = f * f * (3.0 - 2.0 * f)
        out = 0.0
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    wt = ((w[..., 0] if dx else 1 - w[..., 0]) * (w[..., 1] if dy else 1 - w[..., 1])
                          * (w[..., 2] if dz else 1 - w[..., 2]))
                    out = out + wt * self._h(i[..., 0] + dx, i[..., 1] + dy, i[..., 2] + dz)
        return out

    def noise2(self, p):
        p = np.asarray(p, np.float64)
        i = np.floor(p).astype(np.int64)
        f = p - i
        w = f * f * (3.0 - 2.0 * f)
        out = 0.0
        for dx in (0, 1):
            for dy in (0, 1):
                wt = (w[..., 0] if dx else 1 - w[..., 0]) * (w[..., 1] if dy else 1 - w[..., 1])
                out = out + wt * self._h(i[..., 0] + dx, i[..., 1] + dy)
        return out

    def fbm3(self, p, octaves, base=1.0, gain=0.5):
        acc, amp, norm, f = 0.0, 1.0, 0.0, base
        for _ in range(octaves):
            acc = acc + amp * self.noise3(np.asarray(p) * f)
            norm += amp
            amp *= gain
            f *= 2.0
        return acc / norm

    def fbm2(self, p, octaves, base=1.0, gain=0.5):
        acc, amp, norm, f = 0.0, 1.0, 0.0, base
        for _ in range(octaves):
            acc = acc + amp * self.noise2(np.asarray(p) * f)
            norm += amp
            amp *= gain
            f *= 2.0
        return acc / norm


# --------------------------------------------------------------------------
# Displaced icosphere (Fig. 1d "Small BVH")
# --------------------------------------------------------------------------
def icosphere(level: int = 6):
    """Unit icosphere: 20 * 4^level triangles, 10 * 4^level + 2 vertices."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
                  (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)],
                 np.float64)
    f = np.array([(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9),
                  (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2),
                  (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
                  (8, 6, 7), (9, 8, 1)], np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        key = np.minimum(e[:, 0], e[:, 1]) * (len(v) + 1) + np.maximum(e[:, 0], e[:, 1])
        uk, inv = np.unique(key, return_inverse=True)
        a, b = uk // (len(v) + 1), uk % (len(v) + 1)
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(v)
        v = np.concatenate([v, mid])
        m = inv.reshape(3, -1).T + base  # midpoints of edges (01, 12, 20)
        f = np.concatenate([np.stack([f[:, 0], m[:, 0], m[:, 2]], 1),
                            np.stack([f[:, 1], m[:, 1], m[:, 0]], 1),
                            np.stack([f[:, 2], m[:, 2], m[:, 1]], 1),
                            np.stack([m[:, 0], m[:, 1], m[:, 2]], 1)])
    return v, f


def displaced_icosphere(level: int = 6, seed: int = 11, amplitude: float = 0.1):
    """Radius 1 +- amplitude, radial displacement by 3-octave value noise."""
    v, f = icosphere(level)
    noise = _ValueNoise(seed)
    n = noise.fbm3(v * 2.0 + 17.0, 3)  # in [0,1]
    r = 1.0 + amplitude * (2.0 * n - 1.0)
    return (v * r[:, None]).astype(np.float32), f.astype(np.uint32)


def small_bvh_scene(level: int = 6, seed: int = 11):
    """Displaced icosphere (81,920 triangles at level 6) over a 2-triangle
    ground plane; Lambertian 0.6 everywhere."""
    v, f = displaced_icosphere(level, seed)
    v = v + np.array([0.0, 1.12, 0.0], np.float32)
    m = _Mesh()
    m.quad((-20, 0, -20), (-20, 0, 20), (20, 0, 20), (20, 0, -20), 0)
    gv, gt, gm = m.arrays()
    verts = np.concatenate([v, gv]).astype(np.float32)
    tris = np.concatenate([f, gt + len(v)]).astype(np.uint32)
    tmat = np.zeros(len(tris), np.uint32)
    cam = {"eye": (0.0, 1.7, 4.6), "look_at": (0.0, 1.0, 0.0), "up": (0.0, 1.0, 0.0),
           "vfov_deg": 40.0}
    return {"verts": verts, "tris": tris, "tri_mat": tmat,
            "materials": [_mat(LAMBERT, (0.6, 0.6, 0.6))], "camera": cam}


# --------------------------------------------------------------------------
# Terrain + instances (Fig. 1e "Large BVH")
# --------------------------------------------------------------------------
def _terrain_height(noise, x, z, size, amp):
    return amp * noise.fbm2(np.stack([x, z], -1) / size * 6.0 + 3.0, 8)


def large_bvh_scene(grid: int = 2048, n_inst: int = 256, seed: int = 13, size: float = 200.0,
                    amp: float = 24.0, ico_level: int = 6):
    """Fractal heightfield on a grid x grid vertex lattice (2 (grid-1)^2
    triangles, 8-octave fBm value noise) plus n_inst translated and uniformly
    scaled copies of the displaced icosphere, resting on the terrain."""
    noise = _ValueNoise(seed)
    lin = np.linspace(-size / 2, size / 2, grid)
    X, Z = np.meshgrid(lin, lin, indexing="xy")
    Y = _terrain_height(noise, X, Z, size, amp)
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3).astype(np.float32)
    idx = np.arange(grid * grid, dtype=np.int64).reshape(grid, grid)
    a, b = idx[:-1, :-1].ravel(), idx[:-1, 1:].ravel()
    c, d = idx[1:, 1:].ravel(), idx[1:, :-1].ravel()
    # upward-facing winding (normal +y for flat terrain)
    tris = np.concatenate([np.stack([a, d, c], 1), np.stack([a, c, b], 1)]).astype(np.uint32)
    rng = _rng(seed + 1)
    bv, bt = displaced_icosphere(ico_level, seed=11)
    inst = []
    for _ in range(n_inst):
        s = float(rng.uniform(0.8, 3.0))
        x, z = rng.uniform(-0.4 * size, 0.4 * size, size=2)
        y = float(_terrain_height(noise, np.array(x), np.array(z), size, amp)) + 0.9 * s
        inst.append({"blas": 0, "translate": (float(x), y, float(z)), "scale": s})
    h0 = float(_terrain_height(noise, np.array(0.0), np.array(60.0), size, amp))
    cam = {"eye": (0.0, h0 + 14.0, 60.0), "look_at": (0.0, h0 - 2.0, 0.0), "up": (0.0, 1.0, 0.0),
           "vfov_deg": 50.0}
    return {"verts": verts, "tris": tris, "tri_mat": np.zeros(len(tris), np.uint32),
            "blas": [{"verts": bv, "tris": bt, "tri_mat": np.zeros(len(bt), np.uint32)}],
            "instances": inst, "materials": [_mat(LAMBERT, (0.6, 0.6, 0.6))], "camera": cam}


# --------------------------------------------------------------------------
# HDR environment map: sky gradient, value-noise clouds, 0.5 deg sun at 1e4
# --------------------------------------------------------------------------
SUN_ELEVATION_DEG = 35.0
SUN_AZIMUTH_DEG = 120.0
SUN_RADIUS_DEG = 0.5
SUN_RADIANCE = 1.0e4


def sun_direction():
    e, a = math.radians(SUN_ELEVATION_DEG), math.radians(SUN_AZIMUTH_DEG)
    return np.array([math.cos(e) * math.cos(a), math.sin(e), math.cos(e) * math.sin(a)])


def env_map(width: int = 2048, height: int = 1024, seed: int = 5, sun: bool = True,
            sun_radius_deg: float = SUN_RADIUS_DEG):
    """Equirectangular FP32 RGB map (height, width, 3).  Texel (i,j) centre is
    (u,v) = ((i+.5)/W, (j+.5)/H); direction phi = 2 pi u - pi, theta = pi v,
    d = (sin th cos ph, cos th, sin th sin ph) (y up)."""
    u = (np.arange(width) + 0.5) / width
    v = (np.arange(height) + 0.5) / height
    ph = 2 * np.pi * u[None, :] - np.pi
    th = np.pi * v[:, None]
    dx, dy, dz = np.sin(th) * np.cos(ph), np.cos(th) * np.ones_like(ph), np.sin(th) * np.sin(ph)
    el = np.clip(dy, -1, 1)
    # sky: 0.2 at the horizon to 1.0 at the zenith, bluish; ground: dim brown
    t = np.clip(el, 0, 1) ** 0.5
    sky = np.stack([0.20 + 0.35 * t, 0.25 + 0.50 * t, 0.35 + 0.65 * t], -1)
    gnd = (np.stack([0.12 + 0 * el, 0.10 + 0 * el, 0.08 + 0 * el], -1)
           * (1 + 0.5 * np.clip(-el, 0, 1))[..., None])
    col = np.where((el >= 0)[..., None], sky, gnd)
    # clouds: fBm value noise on the direction, only above the horizon
    noise = _ValueNoise(seed)
    p = np.stack([dx, dy, dz], -1) * 4.0 + 31.0
    cl = noise.fbm3(p, 5)
    cov = np.clip((cl - 0.5) * 4.0, 0, 1) * np.clip(el * 6.0, 0, 1)
    cloud = np.array([1.4, 1.4, 1.45])
    col = col * (1 - cov[..., None]) + cloud * cov[..., None]
    # log-normal-like texture variation
    col = col * np.exp(0.3 * (noise.fbm3(p * 3.0 + 5.0, 3) - 0.5))[..., None]
    if sun:
        s = sun_direction()
        cosang = dx * s[0] + dy * s[1] + dz * s[2]
        disk = cosang >= math.cos(math.radians(sun_radius_deg))
        col[disk] = SUN_RADIANCE
    return np.ascontiguousarray(col, dtype=np.float32)


def uniform_env(width: int = 64, height: int = 32, value: float = 1.0):
    return np.full((height, width, 3), value, np.float32)


# --------------------------------------------------------------------------
# NIF initial parameters (Glorot-uniform weights, zero biases)
# --------------------------------------------------------------------------
def nif_layer_dims(n_freq=16, hidden=96, layers=5, skip=0):
    """(fan_in, fan_out) per layer; with skip > 0, hidden layer `skip` reads
    the previous layer's output followed by the 4 n_freq features
    (skip-concat), and the previous layer is hidden - 4 n_freq wide so that
    the concatenation is hidden wide."""
    feat = 4 * n_freq
    outs = [hidden - feat if skip and l + 1 == skip else hidden for l in range(layers)] + [3]
    ins = [feat] + [hidden] * layers
    return list(zip(ins, outs))


def nif_param_count(n_freq=16, hidden=96, layers=5, skip=0):
    return sum(o * i + o for i, o in nif_layer_dims(n_freq, hidden, layers, skip))


def nif_init(seed: int = 3, n_freq=16, hidden=96, layers=5, skip=0):
    """Flat FP32 vector [W1, b1, ..., W_{L+1}, b_{L+1}], W row-major [out][in]."""
    rng = _rng(seed)
    out = []
    for fi, fo in nif_layer_dims(n_freq, hidden, layers, skip):
        a = math.sqrt(6.0 / (fi + fo))
        out.append(rng.uniform(-a, a, size=fo * fi))
        out.append(np.zeros(fo))
    return np.concatenate(out).astype(np.float32)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------
CONFIGS = {
    0: dict(name="box", width=128, height=128, spp=4, max_depth=5, seed=1, env="none", nif=None),
    1: dict(name="box+nif", width=512, height=512, spp=16, max_depth=6, seed=1, env="sky",
            nif="fp16"),
    2: dict(name="spheres+nif", width=1024, height=1024, spp=64, max_depth=8, seed=1, env="sky",
            nif="bf16"),
    3: dict(name="small-bvh+nif", width=1920, height=1080, spp=32, max_depth=6, seed=1, env="sky",
            nif="fp16"),
    4: dict(name="large-bvh+nif", width=1920, height=1080, spp=64, max_depth=8, seed=1, env="sky",
            nif="fp8"),
}


def scene_for(cfg: int):
    if cfg == 0:
        return box_scene(open_front=False)
    if cfg == 1:
        return box_scene(open_front=True)
    if cfg == 2:
        return spheres_scene()
    if cfg == 3:
        return small_bvh_scene()
    if cfg == 4:
        return large_bvh_scene()
    raise ValueError(cfg)
