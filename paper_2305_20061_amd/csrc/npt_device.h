// npt_device.h -- device functions of the path tracer (gfx950).
//
// Every FP32 expression here is evaluated exactly as written: the library
// is compiled with -ffp-contract=off, so each + - * / and sqrtf rounds once
// (IEEE, correctly rounded division and square root) and fmaf appears only
// where it is written.  That is what lets a CPU implementation of the same
// definitions take the same integer decisions (closest primitive, Fresnel
// branch, roulette) for every path at equal seeds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace npt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter-based RNG standing in for the
// IPU's hardware generator (Sec. 3.1.3).  Counter = (a, b, c, purpose).
// ---------------------------------------------------------------------------
enum : uint32_t { kRngCamera = 0, kRngScatter = 1, kRngTrain = 2, kRngStochRound = 4 };

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t a, uint32_t b, uint32_t c, uint32_t purpose,
                                     uint32_t k0, uint32_t k1) {
  uint32_t x0 = a, x1 = b, x2 = c, x3 = purpose;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
    const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
    const uint32_t n0 = hi1 ^ x1 ^ k0;
    const uint32_t n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{x0, x1, x2, x3};
}

// 24 random bits -> [0, 1), exact in FP32.
__device__ __forceinline__ float unit_float(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// sin/cos of 2*pi*u in FP32 (Sec. 3.2.3 computes sincos in software with the
// Cephes routines).  4u splits exactly into a quadrant and a remainder of at
// most half a quarter turn; the remainder in radians feeds the Cephes
// minimax polynomials for [-pi/4, pi/4].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_turns(float u, float& s, float& c) {
  const float quarter_turn = 1.57079632679489661923f;
  const float q = 4.0f * u;
  const float qn = rintf(q);
  const float rem = q - qn;
  const int quadrant = ((int)qn) & 3;
  const float x = rem * quarter_turn;
  const float x2 = x * x;
  const float sp = __builtin_fmaf(__builtin_fmaf(-1.9515295891e-4f, x2, 8.3321608736e-3f), x2,
                                  -1.6666654611e-1f);
  const float sv = __builtin_fmaf(sp * x2, x, x);
  const float cp = __builtin_fmaf(__builtin_fmaf(2.443315711809948e-5f, x2, -1.388731625493765e-3f),
                                  x2, 4.166664568298827e-2f);
  const float cv = __builtin_fmaf(cp * x2, x2, __builtin_fmaf(-0.5f, x2, 1.0f));
  if (quadrant == 0) {
    s = sv; c = cv;
  } else if (quadrant == 1) {
    s = cv; c = -sv;
  } else if (quadrant == 2) {
    s = -sv; c = -cv;
  } else {
    s = -cv; c = sv;
  }
}

// Fractional part of f * x for an integer-valued f, to full FP32 accuracy:
// the product's rounding error is recovered exactly with an FMA (two-product),
// so high Fourier frequencies keep their phase.
__device__ __forceinline__ float frac_product(float f, float x) {
  const float p = f * x;
  const float err = __builtin_fmaf(f, x, -p);
  float r = (p - floorf(p)) + err;
  r = r < 0.0f ? r + 1.0f : (r >= 1.0f ? r - 1.0f : r);
  return r;
}

// ---------------------------------------------------------------------------
// small FP32 vector type with explicit, fixed-order arithmetic
// ---------------------------------------------------------------------------
struct V3 {
  float x, y, z;
};

__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 neg(V3 a) { return V3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 normalized(V3 v) {
  const float len = sqrtf(dot(v, v));
  return V3{v.x / len, v.y / len, v.z / len};
}
__device__ __forceinline__ float comp(V3 v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }

// ---------------------------------------------------------------------------
// Watertight ray/triangle test (Woop, Benthin, Wald 2013) -- the PBRT-v3
// method the paper's kernel derives from (Sec. 3.1.3), FP32 only.  The
// per-ray shear is computed once per ray.
// ---------------------------------------------------------------------------
struct Shear {
  int kx, ky, kz;
  float sx, sy, sz;
};

__device__ __forceinline__ Shear make_shear(V3 d) {
  int kz = 0;
  if (fabsf(d.y) > fabsf(comp(d, kz))) kz = 1;
  if (fabsf(d.z) > fabsf(comp(d, kz))) kz = 2;
  int kx = kz + 1 == 3 ? 0 : kz + 1;
  int ky = kx + 1 == 3 ? 0 : kx + 1;
  const float dz = comp(d, kz);
  if (dz < 0.0f) {
    const int t = kx;
    kx = ky;
    ky = t;
  }
  Shear s;
  s.kx = kx;
  s.ky = ky;
  s.kz = kz;
  s.sx = comp(d, kx) / dz;
  s.sy = comp(d, ky) / dz;
  s.sz = 1.0f / dz;
  return s;
}

// Returns true and t in (0, tmax] on a hit.
__device__ __forceinline__ bool hit_triangle(V3 o, const Shear& s, V3 p0, V3 p1, V3 p2, float tmax,
                                             float& t_out) {
  const V3 a = sub(p0, o), b = sub(p1, o), c = sub(p2, o);
  const float az_ = comp(a, s.kz), bz_ = comp(b, s.kz), cz_ = comp(c, s.kz);
  const float ax = comp(a, s.kx) - s.sx * az_;
  const float ay = comp(a, s.ky) - s.sy * az_;
  const float bx = comp(b, s.kx) - s.sx * bz_;
  const float by = comp(b, s.ky) - s.sy * bz_;
  const float cx = comp(c, s.kx) - s.sx * cz_;
  const float cy = comp(c, s.ky) - s.sy * cz_;
  const float w0 = cx * by - cy * bx;
  const float w1 = ax * cy - ay * cx;
  const float w2 = bx * ay - by * ax;
  const bool any_neg = (w0 < 0.0f) | (w1 < 0.0f) | (w2 < 0.0f);
  const bool any_pos = (w0 > 0.0f) | (w1 > 0.0f) | (w2 > 0.0f);
  if (any_neg & any_pos) return false;
  const float det = (w0 + w1) + w2;
  if (det == 0.0f) return false;
  const float tz = (w0 * (s.sz * az_) + w1 * (s.sz * bz_)) + w2 * (s.sz * cz_);
  const float t = tz / det;
  if (!(t > 0.0f) || !(t <= tmax)) return false;
  t_out = t;
  return true;
}

// Ray/sphere, Ray Tracing Gems ch. 7 form; d must be unit length.
__device__ __forceinline__ bool hit_sphere(V3 o, V3 d, V3 c, float r, float tmax, float& t_out) {
  const V3 f = sub(o, c);
  const float b = -dot(f, d);
  const V3 g = V3{f.x + b * d.x, f.y + b * d.y, f.z + b * d.z};
  const float rr = r * r;
  const float disc = rr - dot(g, g);
  if (disc < 0.0f) return false;
  const float cc = dot(f, f) - rr;
  const float q = b + copysignf(sqrtf(disc), b);
  if (q == 0.0f) return false;
  const float t0 = cc / q, t1 = q;
  const float tn = fminf(t0, t1), tf = fmaxf(t0, t1);
  const float t = tn > 0.0f ? tn : tf;
  if (!(t > 0.0f) || !(t <= tmax)) return false;
  t_out = t;
  return true;
}

// ---------------------------------------------------------------------------
// Spawned-ray origin: Waechter & Binder (Ray Tracing Gems ch. 6) -- offset by
// 256*n ulps on the float bit pattern, or by n/65536 within 1/32 of the
// world origin.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float offset_axis(float p, float n) {
  const int ofs = (int)(256.0f * n);
  const float pi = __int_as_float(__float_as_int(p) + (p < 0.0f ? -ofs : ofs));
  return fabsf(p) < (1.0f / 32.0f) ? p + (1.0f / 65536.0f) * n : pi;
}

__device__ __forceinline__ V3 offset_origin(V3 p, V3 n) {
  return V3{offset_axis(p.x, n.x), offset_axis(p.y, n.y), offset_axis(p.z, n.z)};
}

// ---------------------------------------------------------------------------
// BSDF sampling (Sec. 3.1): Lambertian, mirror, smooth dielectric
// ---------------------------------------------------------------------------
// Orthonormal basis around unit n: Duff et al., JCGT 2017.
__device__ __forceinline__ void basis_around(V3 n, V3& t, V3& b) {
  const float sign = copysignf(1.0f, n.z);
  const float a = -1.0f / (sign + n.z);
  const float k = n.x * n.y * a;
  t = V3{1.0f + sign * n.x * n.x * a, sign * k, -sign * n.x};
  b = V3{k, sign + n.y * n.y * a, -n.y};
}

// Cosine-weighted direction around unit n (disk point lifted to the hemisphere).
__device__ __forceinline__ V3 sample_cosine(V3 n, float u0, float u1) {
  V3 t, b;
  basis_around(n, t, b);
  const float r = sqrtf(u0);
  float sv, cv;
  sincos_turns(u1, sv, cv);
  const float x = r * cv;
  const float y = r * sv;
  const float z = sqrtf(fmaxf(0.0f, 1.0f - u0));
  return V3{(x * t.x + y * b.x) + z * n.x, (x * t.y + y * b.y) + z * n.y,
            (x * t.z + y * b.z) + z * n.z};
}

// Smooth dielectric: exact unpolarised Fresnel; reflect on total internal
// reflection or when u < F, otherwise refract by Snell's law.
__device__ __forceinline__ V3 sample_dielectric(V3 d, V3 n, float ior, float u) {
  const float dn = dot(d, n);
  const bool entering = dn < 0.0f;
  const float eta_i = entering ? 1.0f : ior;
  const float eta_t = entering ? ior : 1.0f;
  const V3 nf = entering ? n : neg(n);
  const float cos_i = entering ? -dn : dn;
  const float eta = eta_i / eta_t;
  const float sin_i = sqrtf(fmaxf(0.0f, 1.0f - cos_i * cos_i));
  const float sin_t = eta * sin_i;
  bool reflect = true;
  float cos_t = 0.0f;
  if (sin_t < 1.0f) {
    cos_t = sqrtf(fmaxf(0.0f, 1.0f - sin_t * sin_t));
    const float rpar = (eta_t * cos_i - eta_i * cos_t) / (eta_t * cos_i + eta_i * cos_t);
    const float rper = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t);
    const float F = (rpar * rpar + rper * rper) * 0.5f;
    reflect = u < F;
  }
  if (reflect) {
    const float k = 2.0f * cos_i;
    return V3{d.x + k * nf.x, d.y + k * nf.y, d.z + k * nf.z};
  }
  const float k = eta * cos_i - cos_t;
  return V3{eta * d.x + k * nf.x, eta * d.y + k * nf.y, eta * d.z + k * nf.z};
}

// ---------------------------------------------------------------------------
// Equirectangular (u, v) of a direction, y up (Sec. 3.3).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void direction_to_uv(V3 d, float& u, float& v) {
  const float kPi = 3.14159265358979323846f;
  const float cy = fminf(1.0f, fmaxf(-1.0f, d.y));
  u = (atan2f(d.z, d.x) + kPi) * (0.5f / kPi);
  v = acosf(cy) * (1.0f / kPi);
}

// Bilinear lookup of an equirect FP32 map (texel centres at half-integers,
// wrap in u, clamp in v).
__device__ __forceinline__ float3 env_bilinear(const float4* map, int W, int H, float u, float v) {
  const float x = u * (float)W - 0.5f;
  const float y = v * (float)H - 0.5f;
  const float x0 = floorf(x), y0 = floorf(y);
  const float fx = x - x0, fy = y - y0;
  int i0 = (int)x0, j0 = (int)y0;
  int i1 = i0 + 1, j1 = j0 + 1;
  i0 = i0 < 0 ? i0 + W : (i0 >= W ? i0 - W : i0);
  i1 = i1 < 0 ? i1 + W : (i1 >= W ? i1 - W : i1);
  j0 = j0 < 0 ? 0 : (j0 > H - 1 ? H - 1 : j0);
  j1 = j1 < 0 ? 0 : (j1 > H - 1 ? H - 1 : j1);
  const float4 t00 = map[(size_t)j0 * W + i0], t01 = map[(size_t)j0 * W + i1];
  const float4 t10 = map[(size_t)j1 * W + i0], t11 = map[(size_t)j1 * W + i1];
  const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
  const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
  return make_float3(w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x,
                     w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y,
                     w00 * t00.z + w01 * t01.z + w10 * t10.z + w11 * t11.z);
}

}  // namespace npt
