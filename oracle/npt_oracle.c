/*
 * npt_oracle.c -- plain, slow, single-threaded CPU oracle of the neural path
 * tracer in "Towards Neural Path Tracing in SRAM" (Pupilli, 2023).
 *
 * TEST INFRASTRUCTURE ONLY (see npt_oracle.h).  Nothing here is reached by the
 * GPU library; the GPU library's code is not reached from here.
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (no contraction, so every FP32 expression below is evaluated exactly as
 * written: one IEEE rounding per + - * / sqrt, and fmaf only where written).
 *
 * Parity-pin status (tests/test_oracle_*.py):
 *   Philox4x32-10 ........... pinned (rocRAND host engine, independent code)
 *   or_u01 .................. pinned (closed form at the range ends)
 *   or_sincos2pi ............ pinned (<= 2 ulp of libm FP64 sin/cos)
 *   camera .................. pinned (FP64 pinhole closed form)
 *   triangle / sphere ....... pinned (FP64 plane / quadratic closed forms,
 *                             watertightness on shared edges)
 *   BVH closest hit ......... pinned (brute force over all primitives)
 *   offset origin ........... pinned (side and no-self-hit invariants)
 *   Fresnel / Snell ......... pinned (angle form of the Fresnel equations,
 *                             Snell's law, F(0) = ((n-1)/(n+1))^2)
 *   ONB / cosine sampling ... pinned (orthonormality, chi^2 vs cos/pi)
 *   env lookup / equirect ... pinned (texel-centre exactness, round trip)
 *   render estimator ........ pinned (closed-box furnace sum rho^k, convex
 *                             furnace, roulette expectation, energy bound)
 *   NIF forward ............. pinned (zero-weight, single-path closed forms,
 *                             positive homogeneity, YUV inverse of BT.601)
 *   NIF backward / Huber .... pinned (FP64 central finite differences)
 *   Adam .................... pinned (constant-gradient closed form)
 */
#define _GNU_SOURCE
#include "npt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Stands in for the IPU's hardware RNG            */
/* (Sec. 3.1.3, App. A.1).                                                    */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u; /* Weyl key schedule */
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Top 24 bits scaled by 2^-24: exactly representable in FP32, range [0, 1). */
float or_u01(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

static void rng4(uint32_t a, uint32_t b, uint32_t c, uint32_t purpose, uint64_t seed,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {a, b, c, purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* FP32 sin/cos of 2*pi*u.  The paper computes sincos in software FP32 with   */
/* the Cephes routines (Sec. 3.2.3, Moshier 1992).  Range reduction here is   */
/* in revolutions: 4u is split exactly into an integer quadrant and a         */
/* remainder in [-1/2, 1/2] quarter turns; the remainder times pi/2 feeds     */
/* the Cephes minimax polynomials for sin and cos on [-pi/4, pi/4].           */
/* ------------------------------------------------------------------------ */
void or_sincos2pi(float u, float *s, float *c)
{
    const float half_pi = 1.57079632679489661923f;
    float q4 = 4.0f * u;
    float qi = rintf(q4);
    float r = q4 - qi; /* exact */
    int quad = ((int)qi) & 3;
    float x = r * half_pi;
    float z = x * x;
    float ps = fmaf(fmaf(-1.9515295891e-4f, z, 8.3321608736e-3f), z, -1.6666654611e-1f);
    float sn = fmaf(ps * z, x, x);
    float pc = fmaf(fmaf(2.443315711809948e-5f, z, -1.388731625493765e-3f), z,
                    4.166664568298827e-2f);
    float cs = fmaf(pc * z, z, fmaf(-0.5f, z, 1.0f));
    switch (quad) {
    case 0: *s = sn; *c = cs; break;
    case 1: *s = cs; *c = -sn; break;
    case 2: *s = -sn; *c = -cs; break;
    default: *s = -cs; *c = sn; break;
    }
}

/* ------------------------------------------------------------------------ */
/* small FP32 vector helpers (written out; no contraction)                    */
/* ------------------------------------------------------------------------ */
static float dot3f(const float a[3], const float b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

static void normalize3f(float v[3])
{
    float len = sqrtf(dot3f(v, v));
    v[0] = v[0] / len;
    v[1] = v[1] / len;
    v[2] = v[2] / len;
}

static void cross3f(const float a[3], const float b[3], float out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------------ */
/* Pinhole camera (primary rays of Sec. 3.1).  Basis and tan(vfov/2) are      */
/* formed on the CPU in FP32; the tangent is taken in FP64 and rounded.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    float eye[3], fwd[3], right[3], up[3];
    float tan_y, tan_x;
} cam_basis;

static void camera_basis(const or_camera *cam, uint32_t W, uint32_t H, cam_basis *b)
{
    for (int i = 0; i < 3; ++i) {
        b->eye[i] = cam->eye[i];
        b->fwd[i] = cam->look_at[i] - cam->eye[i];
    }
    normalize3f(b->fwd);
    cross3f(b->fwd, cam->up, b->right);
    normalize3f(b->right);
    cross3f(b->right, b->fwd, b->up);
    b->tan_y = (float)tan((double)cam->vfov_deg * (M_PI / 360.0));
    float aspect = (float)W / (float)H;
    b->tan_x = b->tan_y * aspect;
}

static void basis_ray(const cam_basis *b, uint32_t W, uint32_t H, uint32_t x, uint32_t y,
                      float jx, float jy, float o[3], float d[3])
{
    float px = ((float)x + jx) / (float)W;
    float py = ((float)y + jy) / (float)H;
    float sx = 2.0f * px - 1.0f;
    float sy = 1.0f - 2.0f * py;
    float cx = sx * b->tan_x;
    float cy = sy * b->tan_y;
    for (int i = 0; i < 3; ++i) {
        o[i] = b->eye[i];
        d[i] = (b->fwd[i] + cx * b->right[i]) + cy * b->up[i];
    }
    normalize3f(d);
}

void or_camera_ray(const or_camera *cam, uint32_t W, uint32_t H, uint32_t x, uint32_t y,
                   float jx, float jy, float o[3], float d[3])
{
    cam_basis b;
    camera_basis(cam, W, H, &b);
    basis_ray(&b, W, H, x, y, jx, jy, o, d);
}

/* ------------------------------------------------------------------------ */
/* Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013), the method  */
/* PBRT-v3 uses and the paper's kernel derives from (Sec. 3.1.3).  FP32 only: */
/* there is no FP64 fallback for zero edge functions (the paper avoids double */
/* emulation); an edge function of exactly zero counts as inside, det == 0 is */
/* a miss, back faces are hit.                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kx, ky, kz;
    float sx, sy, sz;
} shear;

static void ray_shear(const float d[3], shear *s)
{
    int kz = 0;
    if (fabsf(d[1]) > fabsf(d[kz])) kz = 1;
    if (fabsf(d[2]) > fabsf(d[kz])) kz = 2;
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    if (d[kz] < 0.0f) { int t = kx; kx = ky; ky = t; }
    s->kx = kx; s->ky = ky; s->kz = kz;
    s->sx = d[kx] / d[kz];
    s->sy = d[ky] / d[kz];
    s->sz = 1.0f / d[kz];
}

static int tri_test(const float o[3], const shear *s, const float v0[3], const float v1[3],
                    const float v2[3], float tmax, float *t)
{
    float a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = v0[i] - o[i];
        b[i] = v1[i] - o[i];
        c[i] = v2[i] - o[i];
    }
    float ax = a[s->kx] - s->sx * a[s->kz];
    float ay = a[s->ky] - s->sy * a[s->kz];
    float bx = b[s->kx] - s->sx * b[s->kz];
    float by = b[s->ky] - s->sy * b[s->kz];
    float cx = c[s->kx] - s->sx * c[s->kz];
    float cy = c[s->ky] - s->sy * c[s->kz];
    float e0 = cx * by - cy * bx; /* weight of v0 */
    float e1 = ax * cy - ay * cx; /* weight of v1 */
    float e2 = bx * ay - by * ax; /* weight of v2 */
    if ((e0 < 0.0f || e1 < 0.0f || e2 < 0.0f) && (e0 > 0.0f || e1 > 0.0f || e2 > 0.0f))
        return 0;
    float det = (e0 + e1) + e2;
    if (det == 0.0f) return 0;
    float az = s->sz * a[s->kz];
    float bz = s->sz * b[s->kz];
    float cz = s->sz * c[s->kz];
    float tn = (e0 * az + e1 * bz) + e2 * cz;
    float tt = tn / det;
    if (!(tt > 0.0f) || !(tt <= tmax)) return 0;
    *t = tt;
    return 1;
}

int or_intersect_triangle(const float o[3], const float d[3], const float v0[3],
                          const float v1[3], const float v2[3], float tmax, float *t)
{
    shear s;
    ray_shear(d, &s);
    return tri_test(o, &s, v0, v1, v2, tmax, t);
}

/* ------------------------------------------------------------------------ */
/* Ray/sphere (Haines, Guenther, Akenine-Moeller, "Precision improvements for */
/* ray/sphere intersection", Ray Tracing Gems ch. 7).  The paper's Spheres    */
/* scene implies this test but does not give a method.  d must be unit.       */
/* ------------------------------------------------------------------------ */
int or_intersect_sphere(const float o[3], const float d[3], const float c[3], float r,
                        float tmax, float *t)
{
    float f0 = o[0] - c[0], f1 = o[1] - c[1], f2 = o[2] - c[2];
    float b = -((f0 * d[0] + f1 * d[1]) + f2 * d[2]);
    float g0 = f0 + b * d[0], g1 = f1 + b * d[1], g2 = f2 + b * d[2];
    float rr = r * r;
    float disc = rr - ((g0 * g0 + g1 * g1) + g2 * g2);
    if (disc < 0.0f) return 0;
    float cc = ((f0 * f0 + f1 * f1) + f2 * f2) - rr;
    float q = b + copysignf(sqrtf(disc), b);
    if (q == 0.0f) return 0;
    float t0 = cc / q, t1 = q;
    float tn = fminf(t0, t1), tf = fmaxf(t0, t1);
    float tt = tn > 0.0f ? tn : tf;
    if (!(tt > 0.0f) || !(tt <= tmax)) return 0;
    *t = tt;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Spawned-ray origin offset (Waechter & Binder, Ray Tracing Gems ch. 6):    */
/* move p along n by a fixed number of float ulps (integer arithmetic on the */
/* bit pattern), or by a small absolute step near the world origin.  The     */
/* paper does not say how it avoids self-intersection.                       */
/* ------------------------------------------------------------------------ */
static int32_t f2i(float f) { int32_t i; memcpy(&i, &f, 4); return i; }
static float i2f(int32_t i) { float f; memcpy(&f, &i, 4); return f; }

void or_offset_origin(const float p[3], const float n[3], float out[3])
{
    const float near_origin = 1.0f / 32.0f;
    const float float_step = 1.0f / 65536.0f;
    const float int_step = 256.0f;
    for (int i = 0; i < 3; ++i) {
        int32_t ofs = (int32_t)(int_step * n[i]);
        float pi = i2f(f2i(p[i]) + (p[i] < 0.0f ? -ofs : ofs));
        out[i] = fabsf(p[i]) < near_origin ? p[i] + float_step * n[i] : pi;
    }
}

/* ------------------------------------------------------------------------ */
/* BSDFs of the scenes (Sec. 3.1: diffuse, mirror and dielectric surfaces).  */
/* ------------------------------------------------------------------------ */

/* Unpolarised Fresnel reflectance of a smooth dielectric interface.  cos_i
 * >= 0 is measured on the incident side (index eta_i).  Total internal
 * reflection returns 1. */
float or_fresnel_dielectric(float cos_i, float eta_i, float eta_t)
{
    float sin_i = sqrtf(fmaxf(0.0f, 1.0f - cos_i * cos_i));
    float sin_t = (eta_i / eta_t) * sin_i;
    if (sin_t >= 1.0f) return 1.0f;
    float cos_t = sqrtf(fmaxf(0.0f, 1.0f - sin_t * sin_t));
    float rpar = (eta_t * cos_i - eta_i * cos_t) / (eta_t * cos_i + eta_i * cos_t);
    float rper = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t);
    return (rpar * rpar + rper * rper) * 0.5f;
}

/* Orthonormal basis around unit n (Duff et al., "Building an Orthonormal
 * Basis, Revisited", JCGT 2017). */
void or_onb(const float n[3], float t[3], float b[3])
{
    float sign = copysignf(1.0f, n[2]);
    float a = -1.0f / (sign + n[2]);
    float k = n[0] * n[1] * a;
    t[0] = 1.0f + sign * n[0] * n[0] * a;
    t[1] = sign * k;
    t[2] = -sign * n[0];
    b[0] = k;
    b[1] = sign + n[1] * n[1] * a;
    b[2] = -n[1];
}

/* Cosine-weighted hemisphere direction around n (Malley's method: uniform
 * disk point lifted to the hemisphere). */
void or_cosine_sample(const float n[3], float u0, float u1, float out[3])
{
    float t[3], b[3];
    or_onb(n, t, b);
    float r = sqrtf(u0);
    float sn, cs;
    or_sincos2pi(u1, &sn, &cs);
    float x = r * cs;
    float y = r * sn;
    float z = sqrtf(fmaxf(0.0f, 1.0f - u0));
    for (int i = 0; i < 3; ++i) out[i] = (x * t[i] + y * b[i]) + z * n[i];
}

int or_dielectric_scatter(const float d[3], const float n_geom[3], float ior, float u,
                          float out[3])
{
    float dn = dot3f(d, n_geom);
    int entering = dn < 0.0f;
    float eta_i = entering ? 1.0f : ior;
    float eta_t = entering ? ior : 1.0f;
    float nf[3];
    for (int i = 0; i < 3; ++i) nf[i] = entering ? n_geom[i] : -n_geom[i];
    float cos_i = entering ? -dn : dn;
    float eta = eta_i / eta_t;
    float sin_i = sqrtf(fmaxf(0.0f, 1.0f - cos_i * cos_i));
    float sin_t = eta * sin_i;
    int reflect = 1;
    float cos_t = 0.0f;
    if (sin_t < 1.0f) {
        cos_t = sqrtf(fmaxf(0.0f, 1.0f - sin_t * sin_t));
        float rpar = (eta_t * cos_i - eta_i * cos_t) / (eta_t * cos_i + eta_i * cos_t);
        float rper = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t);
        float F = (rpar * rpar + rper * rper) * 0.5f;
        reflect = u < F;
    }
    if (reflect) {
        float k = 2.0f * cos_i;
        for (int i = 0; i < 3; ++i) out[i] = d[i] + k * nf[i];
        return 1;
    }
    float k = eta * cos_i - cos_t;
    for (int i = 0; i < 3; ++i) out[i] = eta * d[i] + k * nf[i];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Environment: equirectangular (u,v) of a world direction (Sec. 3.3), y up, */
/* and FP64 bilinear lookup (texel centres at half-integers, wrap in u,      */
/* clamp in v).  Also the sub-pixel filter of the training samples            */
/* (Sec. 3.2.1).                                                              */
/* ------------------------------------------------------------------------ */
void or_dir_to_uv(double dx, double dy, double dz, double *u, double *v)
{
    double cy = dy < -1.0 ? -1.0 : (dy > 1.0 ? 1.0 : dy);
    *u = (atan2(dz, dx) + M_PI) / (2.0 * M_PI);
    *v = acos(cy) / M_PI;
}

void or_uv_to_dir(double u, double v, double d[3])
{
    double phi = 2.0 * M_PI * u - M_PI;
    double theta = M_PI * v;
    d[0] = sin(theta) * cos(phi);
    d[1] = cos(theta);
    d[2] = sin(theta) * sin(phi);
}

void or_env_bilinear(const float *rgb, uint32_t w, uint32_t h, double u, double v, double out[3])
{
    double x = u * (double)w - 0.5;
    double y = v * (double)h - 0.5;
    double x0 = floor(x), y0 = floor(y);
    double fx = x - x0, fy = y - y0;
    long i0 = (long)x0, j0 = (long)y0;
    long i1 = i0 + 1, j1 = j0 + 1;
    long W = (long)w, H = (long)h;
    i0 = ((i0 % W) + W) % W;
    i1 = ((i1 % W) + W) % W;
    j0 = j0 < 0 ? 0 : (j0 > H - 1 ? H - 1 : j0);
    j1 = j1 < 0 ? 0 : (j1 > H - 1 ? H - 1 : j1);
    for (int c = 0; c < 3; ++c) {
        double t00 = rgb[((size_t)j0 * w + i0) * 3 + c];
        double t01 = rgb[((size_t)j0 * w + i1) * 3 + c];
        double t10 = rgb[((size_t)j1 * w + i0) * 3 + c];
        double t11 = rgb[((size_t)j1 * w + i1) * 3 + c];
        out[c] = (1.0 - fx) * (1.0 - fy) * t00 + fx * (1.0 - fy) * t01 + (1.0 - fx) * fy * t10 +
                 fx * fy * t11;
    }
}

/* ------------------------------------------------------------------------ */
/* HDR-NIF (Sec. 3.2): Fourier features of (u,v) (Tancik et al. 2020), dense */
/* ReLU layers, a linear output layer predicting YUV, and a fixed YUV->RGB   */
/* matrix; outputs are log-compressed radiance, inverted with expm1.         */
/* Parameters: [W1, b1, ..., W_{L+1}, b_{L+1}], W row-major [out][in].       */
/* ------------------------------------------------------------------------ */
uint32_t or_nif_frequency(uint32_t k) { return (uint32_t)llround(pow(2.0, (double)(k + 1) * 0.5)); }

/* Layer widths.  With a skip-concat (Sec. 3.2) the features join the output
 * of the layer before hidden layer `skip`, and that layer is narrowed by the
 * feature count so that the concatenated input of layer `skip` stays
 * `hidden` wide: layer skip-1 has hidden - 4 n_freq outputs.  Every hidden
 * layer after the first therefore reads `hidden` values. */
static uint32_t layer_in(const or_nif_shape *s, uint32_t l) { return l == 0 ? 4 * s->n_freq : s->hidden; }
static uint32_t layer_out(const or_nif_shape *s, uint32_t l)
{
    if (l == s->layers) return 3;
    if (s->skip != 0 && l + 1 == s->skip) return s->hidden - 4 * s->n_freq;
    return s->hidden;
}

uint64_t or_nif_param_count(const or_nif_shape *s)
{
    uint64_t n = 0;
    for (uint32_t l = 0; l <= s->layers; ++l)
        n += (uint64_t)layer_out(s, l) * layer_in(s, l) + layer_out(s, l);
    return n;
}

/* feat = [sin 2pi f_k u | cos 2pi f_k u | sin 2pi f_k v | cos 2pi f_k v], k = 0..n_freq-1 */
void or_nif_features(const or_nif_shape *s, double u, double v, double *feat)
{
    uint32_t nf = s->n_freq;
    for (uint32_t k = 0; k < nf; ++k) {
        double f = (double)or_nif_frequency(k);
        double pu = f * u - floor(f * u);
        double pv = f * v - floor(f * v);
        feat[k] = sin(2.0 * M_PI * pu);
        feat[nf + k] = cos(2.0 * M_PI * pu);
        feat[2 * nf + k] = sin(2.0 * M_PI * pv);
        feat[3 * nf + k] = cos(2.0 * M_PI * pv);
    }
}

/* YUV -> RGB, BT.601 analogue coefficients (row-major 3x3, RGB = M * YUV). */
void or_yuv_to_rgb_matrix(double m[9])
{
    const double k[9] = {1.0, 0.0, 1.13983, 1.0, -0.39465, -0.58060, 1.0, 2.03211, 0.0};
    memcpy(m, k, sizeof(k));
}

/* Output colour spaces compared in Sec. 4.3: YUV (above), RGB (identity) and
 * YCoCg (Malvar & Sullivan): R = Y + Co - Cg, G = Y + Cg, B = Y - Co - Cg,
 * the exact inverse of Y = R/4 + G/2 + B/4, Co = (R - B)/2,
 * Cg = -R/4 + G/2 - B/4. */
void or_colour_to_rgb_matrix(uint32_t colour, double m[9])
{
    static const double rgb[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    static const double ycocg[9] = {1, 1, -1, 1, 0, 1, 1, -1, -1};
    if (colour == OR_COLOUR_RGB)
        memcpy(m, rgb, sizeof(rgb));
    else if (colour == OR_COLOUR_YCOCG)
        memcpy(m, ycocg, sizeof(ycocg));
    else
        or_yuv_to_rgb_matrix(m);
}

/* Forward pass keeping post-activation values: act[l] has layer_in(l) values
 * for l = 0..layers (act[0] = features; act[skip] ends with the features
 * again); y = network output, z = RGB log. */
static void nif_forward_full(const or_nif_shape *s, const double *params, double u, double v,
                             double **act, double y[3], double z[3])
{
    or_nif_features(s, u, v, act[0]);
    const double *p = params;
    for (uint32_t l = 0; l <= s->layers; ++l) {
        uint32_t ni = layer_in(s, l), no = layer_out(s, l);
        const double *W = p, *b = p + (size_t)no * ni;
        double *out = l == s->layers ? y : act[l + 1];
        for (uint32_t j = 0; j < no; ++j) {
            double acc = b[j];
            for (uint32_t i = 0; i < ni; ++i) acc += W[(size_t)j * ni + i] * act[l][i];
            out[j] = (l == s->layers) ? acc : (acc > 0.0 ? acc : 0.0);
        }
        if (s->skip != 0 && l + 1 == s->skip)
            memcpy(act[l + 1] + no, act[0], sizeof(double) * 4 * s->n_freq);
        p += (size_t)no * ni + no;
    }
    double m[9];
    or_colour_to_rgb_matrix(s->colour, m);
    for (int r = 0; r < 3; ++r) z[r] = m[3 * r] * y[0] + m[3 * r + 1] * y[1] + m[3 * r + 2] * y[2];
}

static double **alloc_acts(const or_nif_shape *s)
{
    double **act = (double **)malloc(sizeof(double *) * (s->layers + 1));
    for (uint32_t l = 0; l <= s->layers; ++l) act[l] = (double *)malloc(sizeof(double) * layer_in(s, l));
    return act;
}

static void free_acts(const or_nif_shape *s, double **act)
{
    for (uint32_t l = 0; l <= s->layers; ++l) free(act[l]);
    free(act);
}

void or_nif_forward(const or_nif_shape *s, const double *params, double u, double v, double z[3])
{
    double **act = alloc_acts(s);
    double y[3];
    nif_forward_full(s, params, u, v, act, y, z);
    free_acts(s, act);
}

void or_nif_radiance(const or_nif_shape *s, const double *params, double u, double v, double rgb[3])
{
    double z[3];
    or_nif_forward(s, params, u, v, z);
    for (int c = 0; c < 3; ++c) {
        double e = expm1(z[c]);
        rgb[c] = e > 0.0 ? e : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision NIF inference.  The network is unchanged; what changes  */
/* is where values are rounded: every weight once, and the input vector of   */
/* every layer, each to the format of its matrix-core operands.  Biases stay */
/* exact, and products and sums are exact here (FP64), which the FP32        */
/* accumulation of the device approximates.  Per precision:                  */
/*   FP16 / BF16: weights and layer inputs in binary16 / bfloat16.           */
/*   FP8: the first layer and the output layer as in FP16; the hidden-to-    */
/*        hidden layers with OCP E4M3 weights W * 2^s (s the largest integer */
/*        with max|W| * 2^s <= 448, one per layer), E4M3 inputs (saturating  */
/*        at 448), and the sums taken back by 2^-s.                           */
/* ------------------------------------------------------------------------ */
double or_round_format(double x, int frac_bits, int emin, double maxv, int saturate)
{
    if (x == 0.0 || isnan(x)) return x;
    if (isinf(x)) return saturate ? copysign(maxv, x) : x;
    int e;
    (void)frexp(x, &e); /* |x| in [2^(e-1), 2^e) */
    int lead = e - 1 < emin ? emin : e - 1;
    /* spacing of the format around x is 2^(lead - frac_bits); nearbyint rounds */
    /* to nearest, ties to even, in the default rounding mode                   */
    double q = ldexp(nearbyint(ldexp(x, frac_bits - lead)), lead - frac_bits);
    if (fabs(q) > maxv) q = saturate ? copysign(maxv, x) : copysign(INFINITY, x);
    return q;
}

double or_round_to(double x, int fmt)
{
    switch (fmt) {
    case OR_FMT_F16: return or_round_format(x, 10, -14, 65504.0, 0);
    case OR_FMT_BF16: return or_round_format(x, 7, -126, ldexp(255.0, 120), 0);
    case OR_FMT_E4M3: return or_round_format(x, 3, -6, 448.0, 1);
    default: return x;
    }
}

void or_round_array(const double *in, double *out, uint64_t n, int fmt)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = or_round_to(in[i], fmt);
}

int or_nif_fp8_scale_exp(double maxabs)
{
    if (!(maxabs > 0.0)) return 0;
    int e;
    (void)frexp(maxabs, &e);
    int s = 9 - e; /* maxabs * 2^s in [256, 512) */
    if (ldexp(maxabs, s) > 448.0) s -= 1;
    return s;
}

/* format of the weights and of the input vector of layer l at precision prec */
static int nif_operand_format(const or_nif_shape *s, int prec, uint32_t l)
{
    switch (prec) {
    case OR_PREC_FP16: return OR_FMT_F16;
    case OR_PREC_BF16: return OR_FMT_BF16;
    case OR_PREC_FP8: return (l == 0 || l == s->layers) ? OR_FMT_F16 : OR_FMT_E4M3;
    default: return OR_FMT_NONE;
    }
}

void or_nif_dequantize(const or_nif_shape *s, const double *params, int prec, double *out)
{
    const double *p = params;
    double *q = out;
    for (uint32_t l = 0; l <= s->layers; ++l) {
        uint64_t nw = (uint64_t)layer_out(s, l) * layer_in(s, l), nb = layer_out(s, l);
        int fmt = nif_operand_format(s, prec, l);
        if (fmt == OR_FMT_E4M3) {
            double m = 0.0;
            for (uint64_t i = 0; i < nw; ++i) m = fabs(p[i]) > m ? fabs(p[i]) : m;
            int sc = or_nif_fp8_scale_exp(m);
            for (uint64_t i = 0; i < nw; ++i) q[i] = ldexp(or_round_to(ldexp(p[i], sc), fmt), -sc);
        } else {
            for (uint64_t i = 0; i < nw; ++i) q[i] = or_round_to(p[i], fmt);
        }
        for (uint64_t i = 0; i < nb; ++i) q[nw + i] = p[nw + i];
        p += nw + nb;
        q += nw + nb;
    }
}

void or_nif_forward_q(const or_nif_shape *s, const double *deq, int prec, double u, double v, double z[3])
{
    uint32_t width = 4 * s->n_freq + s->hidden;
    double *x = (double *)malloc(sizeof(double) * width);
    double *h = (double *)malloc(sizeof(double) * width);
    double *feat = (double *)malloc(sizeof(double) * 4 * s->n_freq);
    double y[3];
    or_nif_features(s, u, v, feat);
    memcpy(x, feat, sizeof(double) * 4 * s->n_freq);
    const double *p = deq;
    for (uint32_t l = 0; l <= s->layers; ++l) {
        uint32_t ni = layer_in(s, l), no = layer_out(s, l);
        int fmt = nif_operand_format(s, prec, l);
        for (uint32_t i = 0; i < ni; ++i) x[i] = or_round_to(x[i], fmt);
        const double *W = p, *b = p + (size_t)no * ni;
        double *out = l == s->layers ? y : h;
        for (uint32_t j = 0; j < no; ++j) {
            double acc = b[j];
            for (uint32_t i = 0; i < ni; ++i) acc += W[(size_t)j * ni + i] * x[i];
            out[j] = (l == s->layers) ? acc : (acc > 0.0 ? acc : 0.0);
        }
        if (l < s->layers) memcpy(x, h, sizeof(double) * no);
        if (s->skip != 0 && l + 1 == s->skip) memcpy(x + no, feat, sizeof(double) * 4 * s->n_freq);
        p += (size_t)no * ni + no;
    }
    double m[9];
    or_colour_to_rgb_matrix(s->colour, m);
    for (int r = 0; r < 3; ++r) z[r] = m[3 * r] * y[0] + m[3 * r + 1] * y[1] + m[3 * r + 2] * y[2];
    free(x);
    free(h);
    free(feat);
}

void or_nif_radiance_q(const or_nif_shape *s, const double *deq, int prec, double u, double v, double rgb[3])
{
    double z[3];
    or_nif_forward_q(s, deq, prec, u, v, z);
    for (int c = 0; c < 3; ++c) {
        double e = expm1(z[c]);
        rgb[c] = e > 0.0 ? e : 0.0;
    }
}

/* Huber loss with threshold delta (Sec. 3.2.1 uses delta = 0.001). */
double or_huber(double e, double delta)
{
    double a = fabs(e);
    return a <= delta ? 0.5 * e * e : delta * (a - 0.5 * delta);
}

double or_huber_grad(double e, double delta)
{
    if (fabs(e) <= delta) return e;
    return e > 0.0 ? delta : -delta;
}

double or_nif_loss_grad(const or_nif_shape *s, const double *params, uint64_t n,
                        const double *uv, const double *target, double delta, double *grad)
{
    uint64_t np = or_nif_param_count(s);
    if (grad) memset(grad, 0, sizeof(double) * np);
    double **act = alloc_acts(s);
    double *da = (double *)malloc(sizeof(double) * (s->hidden + 4 * s->n_freq));
    double *dprev = (double *)malloc(sizeof(double) * (s->hidden + 4 * s->n_freq));
    /* offsets of each layer's W in the flat parameter vector */
    size_t *off = (size_t *)malloc(sizeof(size_t) * (s->layers + 1));
    size_t o = 0;
    for (uint32_t l = 0; l <= s->layers; ++l) {
        off[l] = o;
        o += (size_t)layer_out(s, l) * layer_in(s, l) + layer_out(s, l);
    }
    double m[9];
    or_colour_to_rgb_matrix(s->colour, m);
    double loss = 0.0;
    double scale = 1.0 / (3.0 * (double)n);
    for (uint64_t i = 0; i < n; ++i) {
        double y[3], z[3];
        nif_forward_full(s, params, uv[2 * i], uv[2 * i + 1], act, y, z);
        double dz[3];
        for (int c = 0; c < 3; ++c) {
            double e = z[c] - target[3 * i + c];
            loss += or_huber(e, delta);
            dz[c] = or_huber_grad(e, delta) * scale;
        }
        if (!grad) continue;
        /* through the fixed colour matrix: dy = M^T dz */
        double dy[3];
        for (int k = 0; k < 3; ++k) dy[k] = m[k] * dz[0] + m[3 + k] * dz[1] + m[6 + k] * dz[2];
        /* output layer */
        uint32_t L = s->layers;
        {
            uint32_t ni = layer_in(s, L);
            double *gW = grad + off[L], *gb = gW + (size_t)3 * ni;
            const double *W = params + off[L];
            for (uint32_t j = 0; j < 3; ++j) {
                gb[j] += dy[j];
                for (uint32_t q = 0; q < ni; ++q) gW[(size_t)j * ni + q] += dy[j] * act[L][q];
            }
            for (uint32_t q = 0; q < ni; ++q) {
                double acc = 0.0;
                for (uint32_t j = 0; j < 3; ++j) acc += W[(size_t)j * ni + q] * dy[j];
                da[q] = acc;
            }
        }
        /* hidden layers, top down: act[l+1] = relu(W_l act[l] + b_l) */
        for (int l = (int)L - 1; l >= 0; --l) {
            uint32_t ni = layer_in(s, (uint32_t)l), no = layer_out(s, (uint32_t)l);
            double *gW = grad + off[l], *gb = gW + (size_t)no * ni;
            const double *W = params + off[l];
            for (uint32_t j = 0; j < no; ++j) {
                double g = act[l + 1][j] > 0.0 ? da[j] : 0.0;
                da[j] = g;
                gb[j] += g;
                for (uint32_t q = 0; q < ni; ++q) gW[(size_t)j * ni + q] += g * act[l][q];
            }
            if (l > 0) {
                for (uint32_t q = 0; q < ni; ++q) {
                    double acc = 0.0;
                    for (uint32_t j = 0; j < no; ++j) acc += W[(size_t)j * ni + q] * da[j];
                    dprev[q] = acc;
                }
                memcpy(da, dprev, sizeof(double) * ni);
            }
        }
    }
    free(off);
    free(dprev);
    free(da);
    free_acts(s, act);
    return loss * scale;
}

/* Loss and gradient of a training batch with the matrix operands of the    */
/* on-device trainer rounded to the gradient precision (Sec. 3.2.1 trains   */
/* in reduced precision with FP32 accumulation and a loss scale).  As in    */
/* or_nif_forward_q, sums and products are exact; what is rounded, to the   */
/* format of `prec` (nothing for OR_PREC_FP32):                             */
/*   - the weights of the hidden layers 0..L-1, once (the output layer and  */
/*     all biases are used as given: the head runs on the FP32 master);     */
/*   - every layer input: the features, and each ReLU output;               */
/*   - the back-propagated gradient at the output of every hidden layer,    */
/*     after the ReLU mask and with the loss scale S applied: the output-   */
/*     layer gradient dL/dy = M^T (Huber'(z - target) * S) is exact, its    */
/*     product with the output weights is rounded, and so is each product   */
/*     with a hidden layer's rounded weights.  The mask is "the rounded     */
/*     activation is > 0".                                                  */
/* Weight and bias gradients are the exact sums of products of these        */
/* rounded operands, divided by 3 n S at the end; the loss is the mean      */
/* Huber loss of the rounded forward pass.  In OR_PREC_FP32 mode this is     */
/* the gradient of or_nif_loss_grad.                                        */
double or_nif_loss_grad_q(const or_nif_shape *s, const double *params, int prec, double loss_scale,
                          uint64_t n, const double *uv, const double *target, double delta, double *grad)
{
    const int fmt = prec == OR_PREC_FP16 ? OR_FMT_F16 : prec == OR_PREC_BF16 ? OR_FMT_BF16 : OR_FMT_NONE;
    const uint32_t L = s->layers, F = 4 * s->n_freq;
    const uint64_t np = or_nif_param_count(s);
    /* offsets of W_l in the flat vector, and the rounded hidden-layer weights */
    size_t *off = (size_t *)malloc(sizeof(size_t) * (L + 1));
    double *wq = (double *)malloc(sizeof(double) * np);
    size_t o = 0;
    for (uint32_t l = 0; l <= L; ++l) {
        const size_t nw = (size_t)layer_out(s, l) * layer_in(s, l), nb = layer_out(s, l);
        off[l] = o;
        for (size_t i = 0; i < nw; ++i) wq[o + i] = l < L ? or_round_to(params[o + i], fmt) : params[o + i];
        for (size_t i = 0; i < nb; ++i) wq[o + nw + i] = params[o + nw + i];
        o += nw + nb;
    }
    /* x[l]: rounded input of layer l (layer_in(l) values) */
    double **x = (double **)malloc(sizeof(double *) * (L + 1));
    for (uint32_t l = 0; l <= L; ++l) x[l] = (double *)malloc(sizeof(double) * layer_in(s, l));
    double *feat = (double *)malloc(sizeof(double) * F);
    double *g = (double *)malloc(sizeof(double) * s->hidden);  /* gradient at a layer's output */
    double *gp = (double *)malloc(sizeof(double) * s->hidden); /* ... and at its input        */
    double m[9];
    or_colour_to_rgb_matrix(s->colour, m);
    if (grad) memset(grad, 0, sizeof(double) * np);
    double loss = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        or_nif_features(s, uv[2 * i], uv[2 * i + 1], feat);
        for (uint32_t k = 0; k < F; ++k) x[0][k] = or_round_to(feat[k], fmt);
        for (uint32_t l = 0; l < L; ++l) {
            const uint32_t ni = layer_in(s, l), no = layer_out(s, l);
            const double *W = wq + off[l], *b = W + (size_t)no * ni;
            for (uint32_t j = 0; j < no; ++j) {
                double acc = b[j];
                for (uint32_t q = 0; q < ni; ++q) acc += W[(size_t)j * ni + q] * x[l][q];
                x[l + 1][j] = or_round_to(acc > 0.0 ? acc : 0.0, fmt);
            }
            if (s->skip != 0 && l + 1 == s->skip) memcpy(x[l + 1] + no, x[0], sizeof(double) * F);
        }
        const uint32_t H = layer_in(s, L);
        const double *WL = wq + off[L], *bL = WL + (size_t)3 * H;
        double y[3], z[3], dz[3], dy[3];
        for (uint32_t j = 0; j < 3; ++j) {
            double acc = bL[j];
            for (uint32_t q = 0; q < H; ++q) acc += WL[(size_t)j * H + q] * x[L][q];
            y[j] = acc;
        }
        for (int r = 0; r < 3; ++r) z[r] = m[3 * r] * y[0] + m[3 * r + 1] * y[1] + m[3 * r + 2] * y[2];
        for (int c = 0; c < 3; ++c) {
            const double e = z[c] - target[3 * i + c];
            loss += or_huber(e, delta);
            dz[c] = or_huber_grad(e, delta) * loss_scale;
        }
        if (!grad) continue;
        for (int k = 0; k < 3; ++k) dy[k] = m[k] * dz[0] + m[3 + k] * dz[1] + m[6 + k] * dz[2];
        {
            double *gW = grad + off[L], *gb = gW + (size_t)3 * H;
            for (uint32_t j = 0; j < 3; ++j) {
                gb[j] += dy[j];
                for (uint32_t q = 0; q < H; ++q) gW[(size_t)j * H + q] += dy[j] * x[L][q];
            }
            for (uint32_t q = 0; q < H; ++q) {
                double acc = 0.0;
                for (uint32_t j = 0; j < 3; ++j) acc += WL[(size_t)j * H + q] * dy[j];
                g[q] = x[L][q] > 0.0 ? or_round_to(acc, fmt) : 0.0;
            }
        }
        for (int l = (int)L - 1; l >= 0; --l) {
            const uint32_t ni = layer_in(s, (uint32_t)l), no = layer_out(s, (uint32_t)l);
            const double *W = wq + off[l];
            double *gW = grad + off[l], *gb = gW + (size_t)no * ni;
            for (uint32_t j = 0; j < no; ++j) {
                gb[j] += g[j];
                for (uint32_t q = 0; q < ni; ++q) gW[(size_t)j * ni + q] += g[j] * x[l][q];
            }
            if (l == 0) break;
            /* the gradient at the output of layer l-1: the hidden part of */
            /* layer l's input (its first layer_out(l-1) columns)          */
            const uint32_t nprev = layer_out(s, (uint32_t)l - 1);
            for (uint32_t q = 0; q < nprev; ++q) {
                double acc = 0.0;
                for (uint32_t j = 0; j < no; ++j) acc += W[(size_t)j * ni + q] * g[j];
                gp[q] = x[l][q] > 0.0 ? or_round_to(acc, fmt) : 0.0;
            }
            memcpy(g, gp, sizeof(double) * nprev);
        }
    }
    if (grad) {
        const double sc = 1.0 / (3.0 * (double)n * loss_scale);
        for (uint64_t k = 0; k < np; ++k) grad[k] *= sc;
    }
    for (uint32_t l = 0; l <= L; ++l) free(x[l]);
    free(x);
    free(feat);
    free(g);
    free(gp);
    free(wq);
    free(off);
    return loss / (3.0 * (double)n);
}

void or_nif_train_batch(const float *map, uint32_t w, uint32_t h, uint64_t seed, uint32_t step,
                        uint64_t n, double *uv, double *target)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t r[4];
        rng4((uint32_t)i, step, 0, OR_RNG_TRAIN, seed, r);
        double u = (double)or_u01(r[0]);
        double v = (double)or_u01(r[1]);
        double rgb[3];
        or_env_bilinear(map, w, h, u, v, rgb);
        uv[2 * i] = u;
        uv[2 * i + 1] = v;
        for (int c = 0; c < 3; ++c) target[3 * i + c] = log1p(rgb[c]);
    }
}

void or_adam_step(uint64_t n, double *params, const double *grad, double *m, double *v,
                  uint32_t step, double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)step);
    double c2 = 1.0 - pow(beta2, (double)step);
    for (uint64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* FP16 master weights with stochastic rounding (Sec. 3.2.1 keeps the IPU's */
/* master weights in binary16 and rounds updates stochastically, after      */
/* Gupta et al. 2015).  x lies between adjacent binary16 magnitudes a       */
/* (toward zero) and a + q (away from zero), q their spacing; it becomes    */
/* a + q with probability (|x| - a)/q, i.e. when u < (|x| - a)/q for u      */
/* uniform in [0,1).  Magnitudes from 65504 up saturate to 65504.           */
/* ------------------------------------------------------------------------ */
static double fp16_spacing(double ax)
{
    int e;
    (void)frexp(ax, &e); /* ax in [2^(e-1), 2^e) */
    int lead = e - 1 < -14 ? -14 : e - 1;
    return ldexp(1.0, lead - 10);
}

double or_fp16_toward_zero(double x)
{
    if (x == 0.0 || isnan(x)) return x;
    double ax = fabs(x);
    if (ax >= 65504.0) return copysign(65504.0, x);
    double q = fp16_spacing(ax);
    return copysign(floor(ax / q) * q, x);
}

double or_fp16_stochastic(double x, double u)
{
    if (x == 0.0 || isnan(x)) return x;
    double ax = fabs(x);
    if (ax >= 65504.0) return copysign(65504.0, x);
    double q = fp16_spacing(ax);
    double a = floor(ax / q) * q;
    return copysign(u < (ax - a) / q ? a + q : a, x);
}

/* Adam with FP16 master weights: the master is first rounded to the nearest */
/* binary16 (a no-op after the first step), the update is taken in FP64 and */
/* rounded to FP32, then rounded stochastically to binary16 with u from the */
/* Philox stream (parameter index, Adam step t, 0, OR_RNG_SROUND).          */
void or_adam_step_fp16_master(uint64_t n, double *params, const double *grad, double *m, double *v,
                              uint32_t step, double lr, double beta1, double beta2, double eps,
                              uint64_t seed)
{
    double c1 = 1.0 - pow(beta1, (double)step);
    double c2 = 1.0 - pow(beta2, (double)step);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint64_t i = 0; i < n; ++i) {
        double w0 = or_round_to(params[i], OR_FMT_F16);
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        double x = (double)(float)(w0 - lr * mh / (sqrt(vh) + eps));
        const uint32_t ctr[4] = {(uint32_t)i, step, 0u, OR_RNG_SROUND};
        uint32_t r[4];
        or_philox4x32_10(ctr, key, r);
        params[i] = or_fp16_stochastic(x, (double)or_u01(r[0]));
    }
}

double or_nif_train_step(const or_nif_shape *s, double *params, double *m, double *v,
                         const float *map, uint32_t w, uint32_t h, uint64_t seed, uint32_t step,
                         uint64_t batch, double lr, double beta1, double beta2, double eps,
                         double delta, int fp16_master)
{
    uint64_t np = or_nif_param_count(s);
    double *uv = (double *)malloc(sizeof(double) * 2 * batch);
    double *tg = (double *)malloc(sizeof(double) * 3 * batch);
    double *g = (double *)malloc(sizeof(double) * np);
    if (fp16_master)
        for (uint64_t i = 0; i < np; ++i) params[i] = or_round_to(params[i], OR_FMT_F16);
    or_nif_train_batch(map, w, h, seed, step, batch, uv, tg);
    double loss = or_nif_loss_grad(s, params, batch, uv, tg, delta, g);
    if (fp16_master)
        or_adam_step_fp16_master(np, params, g, m, v, step + 1, lr, beta1, beta2, eps, seed);
    else
        or_adam_step(np, params, g, m, v, step + 1, lr, beta1, beta2, eps);
    free(g);
    free(tg);
    free(uv);
    return loss;
}

/* ------------------------------------------------------------------------ */
/* Scenes and the oracle's own acceleration structure: a median-split BVH2  */
/* with FP64 boxes padded outward, so that it can only add work, never drop */
/* a primitive the FP32 tests would hit.  Closest hit is defined over all   */
/* primitives: smallest t, ties to the lowest (instance, primitive).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double lo[3], hi[3];
    uint32_t left, right; /* children (inner) */
    uint32_t first, count; /* primitive range in `order` (leaf when count > 0) */
} bvh_node;

typedef struct {
    const float *verts; /* owned copies */
    const uint32_t *tris;
    const uint32_t *tmat;
    const float *sph;
    const uint32_t *smat;
    uint64_t nv, nt, ns;
    bvh_node *nodes;
    uint32_t nnodes;
    uint32_t *order; /* global primitive ids in leaf order */
    double lo[3], hi[3];
} mesh;

struct or_scene {
    mesh base;
    mesh *blas;
    uint32_t nblas;
    or_instance *inst;
    uint32_t ninst;
    or_material *mats;
    uint32_t nmat;
    int accel;
};

static void prim_bounds(const mesh *m, uint32_t prim, double lo[3], double hi[3])
{
    if (prim < m->nt) {
        const uint32_t *t = m->tris + 3 * (size_t)prim;
        for (int a = 0; a < 3; ++a) {
            lo[a] = hi[a] = m->verts[3 * (size_t)t[0] + a];
        }
        for (int k = 1; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                double x = m->verts[3 * (size_t)t[k] + a];
                if (x < lo[a]) lo[a] = x;
                if (x > hi[a]) hi[a] = x;
            }
    } else {
        const float *s = m->sph + 4 * (size_t)(prim - m->nt);
        for (int a = 0; a < 3; ++a) {
            lo[a] = (double)s[a] - (double)s[3];
            hi[a] = (double)s[a] + (double)s[3];
        }
    }
}

/* Outward padding: 1e-5 of the largest coordinate magnitude. */
static void pad_box(double lo[3], double hi[3])
{
    double mag = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (fabs(lo[a]) > mag) mag = fabs(lo[a]);
        if (fabs(hi[a]) > mag) mag = fabs(hi[a]);
    }
    double pad = 1e-5 * mag + 1e-30;
    for (int a = 0; a < 3; ++a) {
        lo[a] -= pad;
        hi[a] += pad;
    }
}

/* Build-time copy of the primitive bounds in `order` position: ob[6 i ..]  */
/* = (lo, hi) of primitive order[i], permuted together with order, so the  */
/* median splits below read memory in sequence.                            */
static double slot_centroid(const double *ob, uint32_t i, int axis)
{
    return 0.5 * (ob[6 * (size_t)i + axis] + ob[6 * (size_t)i + 3 + axis]);
}

static void swap_slots(uint32_t *order, double *ob, uint32_t i, uint32_t j)
{
    uint32_t t = order[i]; order[i] = order[j]; order[j] = t;
    for (int k = 0; k < 6; ++k) {
        double x = ob[6 * (size_t)i + k];
        ob[6 * (size_t)i + k] = ob[6 * (size_t)j + k];
        ob[6 * (size_t)j + k] = x;
    }
}

/* Quickselect with a three-way partition on the centroid along `axis`: */
/* afterwards order[nth] holds the nth smallest and is a median split.  */
/* Pivots come from a fixed pseudo-random sequence (xorshift64), which   */
/* keeps the expected work linear also on grid-ordered meshes, where the */
/* middle element of a range is often near one end of its key range.    */
static void select_nth(uint32_t *order, double *ob, uint32_t lo, uint32_t hi, uint32_t nth, int axis)
{
    uint64_t r = 0x9E3779B97F4A7C15ull ^ ((uint64_t)lo << 32 | hi);
    while (hi - lo > 1) {
        r ^= r << 13;
        r ^= r >> 7;
        r ^= r << 17;
        double pivot = slot_centroid(ob, lo + (uint32_t)(r % (hi - lo)), axis);
        uint32_t lt = lo, i = lo, gt = hi;
        while (i < gt) {
            double c = slot_centroid(ob, i, axis);
            if (c < pivot) {
                swap_slots(order, ob, lt, i);
                ++lt; ++i;
            } else if (c > pivot) {
                --gt;
                swap_slots(order, ob, gt, i);
            } else {
                ++i;
            }
        }
        if (nth < lt) hi = lt;
        else if (nth >= gt) lo = gt;
        else return;
    }
}

static uint32_t build_node(mesh *m, double *ob, uint32_t lo, uint32_t hi)
{
    uint32_t id = m->nnodes++;
    bvh_node *n = &m->nodes[id];
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = lo; i < hi; ++i) {
        const double *pl = ob + 6 * (size_t)i, *ph = pl + 3;
        for (int a = 0; a < 3; ++a) {
            if (pl[a] < blo[a]) blo[a] = pl[a];
            if (ph[a] > bhi[a]) bhi[a] = ph[a];
            double c = 0.5 * (pl[a] + ph[a]);
            if (c < clo[a]) clo[a] = c;
            if (c > chi[a]) chi[a] = c;
        }
    }
    pad_box(blo, bhi);
    for (int a = 0; a < 3; ++a) {
        n->lo[a] = blo[a];
        n->hi[a] = bhi[a];
    }
    if (hi - lo <= 4) {
        n->first = lo;
        n->count = hi - lo;
        n->left = n->right = 0;
        return id;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    uint32_t mid = lo + (hi - lo) / 2;
    select_nth(m->order, ob, lo, hi, mid, axis);
    n->count = 0;
    n->first = 0;
    uint32_t l = build_node(m, ob, lo, mid);
    uint32_t r = build_node(m, ob, mid, hi);
    m->nodes[id].left = l;
    m->nodes[id].right = r;
    return id;
}

static void mesh_init(mesh *m, const float *verts, uint64_t nv, const uint32_t *tris, uint64_t nt,
                      const uint32_t *tmat, const float *sph, uint64_t ns, const uint32_t *smat,
                      int accel)
{
    memset(m, 0, sizeof(*m));
    float *v = (float *)malloc(sizeof(float) * 3 * (nv ? nv : 1));
    uint32_t *t = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (nt ? nt : 1));
    uint32_t *tm = (uint32_t *)malloc(sizeof(uint32_t) * (nt ? nt : 1));
    float *s = (float *)malloc(sizeof(float) * 4 * (ns ? ns : 1));
    uint32_t *sm = (uint32_t *)malloc(sizeof(uint32_t) * (ns ? ns : 1));
    if (nv) memcpy(v, verts, sizeof(float) * 3 * nv);
    if (nt) {
        memcpy(t, tris, sizeof(uint32_t) * 3 * nt);
        if (tmat) memcpy(tm, tmat, sizeof(uint32_t) * nt); else memset(tm, 0, sizeof(uint32_t) * nt);
    }
    if (ns) {
        memcpy(s, sph, sizeof(float) * 4 * ns);
        if (smat) memcpy(sm, smat, sizeof(uint32_t) * ns); else memset(sm, 0, sizeof(uint32_t) * ns);
    }
    m->verts = v; m->tris = t; m->tmat = tm; m->sph = s; m->smat = sm;
    m->nv = nv; m->nt = nt; m->ns = ns;
    uint64_t np = nt + ns;
    for (int a = 0; a < 3; ++a) { m->lo[a] = INFINITY; m->hi[a] = -INFINITY; }
    for (uint64_t p = 0; p < np; ++p) {
        double pl[3], ph[3];
        prim_bounds(m, (uint32_t)p, pl, ph);
        for (int a = 0; a < 3; ++a) {
            if (pl[a] < m->lo[a]) m->lo[a] = pl[a];
            if (ph[a] > m->hi[a]) m->hi[a] = ph[a];
        }
    }
    pad_box(m->lo, m->hi);
    m->order = (uint32_t *)malloc(sizeof(uint32_t) * (np ? np : 1));
    for (uint64_t p = 0; p < np; ++p) m->order[p] = (uint32_t)p;
    if (accel && np > 0) {
        double *ob = (double *)malloc(sizeof(double) * 6 * np);
        for (uint64_t p = 0; p < np; ++p) prim_bounds(m, (uint32_t)p, ob + 6 * p, ob + 6 * p + 3);
        m->nodes = (bvh_node *)malloc(sizeof(bvh_node) * (2 * np + 1));
        m->nnodes = 0;
        build_node(m, ob, 0, (uint32_t)np);
        free(ob);
    }
}

static void mesh_free(mesh *m)
{
    free((void *)m->verts); free((void *)m->tris); free((void *)m->tmat);
    free((void *)m->sph); free((void *)m->smat);
    free(m->nodes); free(m->order);
}

or_scene *or_scene_create(const float *verts, uint64_t nv, const uint32_t *tris, uint64_t nt,
                          const uint32_t *tri_mat, const float *spheres, uint64_t ns,
                          const uint32_t *sph_mat, const or_material *mats, uint32_t nmat,
                          int accel)
{
    or_scene *sc = (or_scene *)calloc(1, sizeof(or_scene));
    sc->accel = accel;
    mesh_init(&sc->base, verts, nv, tris, nt, tri_mat, spheres, ns, sph_mat, accel);
    sc->mats = (or_material *)malloc(sizeof(or_material) * (nmat ? nmat : 1));
    if (nmat) memcpy(sc->mats, mats, sizeof(or_material) * nmat);
    sc->nmat = nmat;
    return sc;
}

int or_scene_add_blas(or_scene *sc, const float *verts, uint64_t nv, const uint32_t *tris,
                      uint64_t nt, const uint32_t *tri_mat)
{
    sc->blas = (mesh *)realloc(sc->blas, sizeof(mesh) * (sc->nblas + 1));
    mesh_init(&sc->blas[sc->nblas], verts, nv, tris, nt, tri_mat, NULL, 0, NULL, sc->accel);
    return (int)sc->nblas++;
}

int or_scene_set_instances(or_scene *sc, const or_instance *inst, uint32_t n)
{
    free(sc->inst);
    sc->inst = (or_instance *)malloc(sizeof(or_instance) * (n ? n : 1));
    if (n) memcpy(sc->inst, inst, sizeof(or_instance) * n);
    sc->ninst = n;
    for (uint32_t i = 0; i < n; ++i)
        if (inst[i].blas >= sc->nblas) return -1;
    return 0;
}

void or_scene_destroy(or_scene *sc)
{
    if (!sc) return;
    mesh_free(&sc->base);
    for (uint32_t i = 0; i < sc->nblas; ++i) mesh_free(&sc->blas[i]);
    free(sc->blas);
    free(sc->inst);
    free(sc->mats);
    free(sc);
}

/* FP64 slab test against [0, tmax]; conservative on the padded boxes. */
static int box_hit(const double lo[3], const double hi[3], const float o[3], const float d[3],
                   double tmax)
{
    double tn = 0.0, tf = tmax;
    for (int a = 0; a < 3; ++a) {
        double oa = o[a], da = d[a];
        if (da == 0.0) {
            if (oa < lo[a] || oa > hi[a]) return 0;
            continue;
        }
        double inv = 1.0 / da;
        double t0 = (lo[a] - oa) * inv, t1 = (hi[a] - oa) * inv;
        if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
        if (t0 > tn) tn = t0;
        if (t1 < tf) tf = t1;
        if (tn > tf) return 0;
    }
    return 1;
}

typedef struct {
    float t;
    uint32_t prim, inst;
    int hit;
} best_hit;

static int better(float t, uint32_t inst, uint32_t prim, const best_hit *b)
{
    if (!b->hit) return 1;
    if (t < b->t) return 1;
    if (t > b->t) return 0;
    if (inst != b->inst) return inst < b->inst;
    return prim < b->prim;
}

static void test_prim(const mesh *m, uint32_t prim, uint32_t inst, const float o[3],
                      const float d[3], const shear *s, best_hit *b)
{
    float tmax = b->hit ? b->t : INFINITY;
    float t;
    int h;
    if (prim < m->nt) {
        const uint32_t *tr = m->tris + 3 * (size_t)prim;
        h = tri_test(o, s, m->verts + 3 * (size_t)tr[0], m->verts + 3 * (size_t)tr[1],
                     m->verts + 3 * (size_t)tr[2], tmax, &t);
    } else {
        const float *sp = m->sph + 4 * (size_t)(prim - m->nt);
        h = or_intersect_sphere(o, d, sp, sp[3], tmax, &t);
    }
    if (h && better(t, inst, prim, b)) {
        b->t = t;
        b->prim = prim;
        b->inst = inst;
        b->hit = 1;
    }
}

static void mesh_closest(const mesh *m, uint32_t inst, const float o[3], const float d[3],
                         int accel, best_hit *b)
{
    shear s;
    ray_shear(d, &s);
    uint64_t np = m->nt + m->ns;
    if (np == 0) return;
    if (!accel) {
        for (uint64_t p = 0; p < np; ++p) test_prim(m, (uint32_t)p, inst, o, d, &s, b);
        return;
    }
    uint32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const bvh_node *n = &m->nodes[stack[--sp]];
        double tmax = b->hit ? (double)b->t * (1.0 + 1e-6) : INFINITY;
        if (!box_hit(n->lo, n->hi, o, d, tmax)) continue;
        if (n->count > 0) {
            for (uint32_t i = 0; i < n->count; ++i) test_prim(m, m->order[n->first + i], inst, o, d, &s, b);
        } else {
            stack[sp++] = n->left;
            stack[sp++] = n->right;
        }
    }
}

static void mesh_tri_normal(const mesh *m, uint32_t prim, float n[3])
{
    const uint32_t *tr = m->tris + 3 * (size_t)prim;
    const float *v0 = m->verts + 3 * (size_t)tr[0];
    const float *v1 = m->verts + 3 * (size_t)tr[1];
    const float *v2 = m->verts + 3 * (size_t)tr[2];
    float e1[3], e2[3];
    for (int i = 0; i < 3; ++i) {
        e1[i] = v1[i] - v0[i];
        e2[i] = v2[i] - v0[i];
    }
    cross3f(e1, e2, n);
    normalize3f(n);
}

int or_closest_hit(const or_scene *sc, const float o[3], const float d[3], float tmax,
                   float *t, uint32_t *prim, uint32_t *inst, float n_geom[3])
{
    /* the global closest hit is found first; tmax only filters it */
    best_hit b = {INFINITY, 0, 0, 0};
    mesh_closest(&sc->base, 0, o, d, sc->accel, &b); /* base geometry: instance 0 */
    for (uint32_t k = 0; k < sc->ninst; ++k) {
        const or_instance *in = &sc->inst[k];
        const mesh *m = &sc->blas[in->blas];
        double wlo[3], whi[3];
        for (int a = 0; a < 3; ++a) {
            wlo[a] = m->lo[a] * in->scale + in->translate[a];
            whi[a] = m->hi[a] * in->scale + in->translate[a];
        }
        pad_box(wlo, whi);
        double bt = b.hit ? (double)b.t * (1.0 + 1e-6) : INFINITY;
        if (!box_hit(wlo, whi, o, d, bt)) continue;
        /* object ray: both terms scaled by r = 1 / scale, rounded to FP32 once
           (instancing is not in the paper; this is the library's definition) */
        const float r = 1.0f / in->scale;
        float oo[3], od[3];
        for (int a = 0; a < 3; ++a) {
            oo[a] = (o[a] - in->translate[a]) * r;
            od[a] = d[a] * r;
        }
        mesh_closest(m, k + 1, oo, od, sc->accel, &b);
    }
    if (!b.hit || !(b.t <= tmax)) return 0;
    *t = b.t;
    *prim = b.prim;
    *inst = b.inst;
    if (n_geom) {
        if (b.inst == 0) {
            const mesh *m = &sc->base;
            if (b.prim < m->nt) {
                mesh_tri_normal(m, b.prim, n_geom);
            } else {
                const float *sp = m->sph + 4 * (size_t)(b.prim - m->nt);
                for (int a = 0; a < 3; ++a) {
                    float p = o[a] + b.t * d[a];
                    n_geom[a] = (p - sp[a]) / sp[3];
                }
            }
        } else {
            mesh_tri_normal(&sc->blas[sc->inst[b.inst - 1].blas], b.prim, n_geom);
        }
    }
    return 1;
}

static const or_material *hit_material(const or_scene *sc, uint32_t prim, uint32_t inst)
{
    uint32_t id;
    if (inst == 0) {
        const mesh *m = &sc->base;
        id = prim < m->nt ? m->tmat[prim] : m->smat[prim - m->nt];
    } else {
        id = sc->blas[sc->inst[inst - 1].blas].tmat[prim];
    }
    return &sc->mats[id < sc->nmat ? id : 0];
}

static void env_radiance(const or_render_desc *rd, const float d[3], double out[3])
{
    if (rd->env_mode == OR_ENV_CONST) {
        for (int c = 0; c < 3; ++c) out[c] = rd->env_const[c];
        return;
    }
    double u, v;
    or_dir_to_uv(d[0], d[1], d[2], &u, &v);
    if (rd->env_mode == OR_ENV_MAP) {
        or_env_bilinear(rd->env_map, rd->env_w, rd->env_h, u, v, out);
    } else {
        or_nif_radiance_q(&rd->nif, rd->nif_params, (int)rd->nif_prec, u, v, out);
    }
}

/* ------------------------------------------------------------------------ */
/* The estimator (Sec. 3.1): contributions are added only when a path hits  */
/* an emissive surface by chance (front face) or escapes to the environment */
/* (Sec. 3.3); Russian roulette from depth rr_start (3 in Sec. 4) keeps a   */
/* path with probability min(1, max channel of throughput) and divides the  */
/* throughput by it.  max_depth counts ray segments including the primary.  */
/* ------------------------------------------------------------------------ */
static void path_sample(const or_scene *sc, const cam_basis *cb, const or_render_desc *rd,
                        uint32_t x, uint32_t y, uint32_t s, double L[3])
{
    uint32_t pix = y * rd->width + x;
    uint32_t r[4];
    rng4(pix, s, 0, OR_RNG_CAM, rd->seed, r);
    float o[3], d[3];
    basis_ray(cb, rd->width, rd->height, x, y, or_u01(r[0]), or_u01(r[1]), o, d);
    float beta[3] = {1.0f, 1.0f, 1.0f};
    double beta64[3] = {1.0, 1.0, 1.0};
    L[0] = L[1] = L[2] = 0.0;
    for (uint32_t k = 1; k <= rd->max_depth; ++k) {
        float t, n[3];
        uint32_t prim, inst;
        if (!or_closest_hit(sc, o, d, INFINITY, &t, &prim, &inst, n)) {
            double env[3];
            env_radiance(rd, d, env);
            for (int c = 0; c < 3; ++c) L[c] += beta64[c] * env[c];
            break;
        }
        const or_material *mat = hit_material(sc, prim, inst);
        float dn = dot3f(d, n);
        if (dn < 0.0f)
            for (int c = 0; c < 3; ++c) L[c] += beta64[c] * (double)mat->emission[c];
        if (k == rd->max_depth || mat->type == OR_EMITTER) break;
        rng4(pix, s, k, OR_RNG_SCATTER, rd->seed, r);
        float nd[3];
        if (mat->type == OR_LAMBERT) {
            float nf[3];
            for (int i = 0; i < 3; ++i) nf[i] = dn > 0.0f ? -n[i] : n[i];
            or_cosine_sample(nf, or_u01(r[0]), or_u01(r[1]), nd);
            for (int c = 0; c < 3; ++c) {
                beta[c] = beta[c] * mat->albedo[c];
                beta64[c] *= (double)mat->albedo[c];
            }
        } else if (mat->type == OR_MIRROR) {
            float k2 = 2.0f * dn;
            for (int i = 0; i < 3; ++i) nd[i] = d[i] - k2 * n[i];
            for (int c = 0; c < 3; ++c) {
                beta[c] = beta[c] * mat->albedo[c];
                beta64[c] *= (double)mat->albedo[c];
            }
        } else {
            or_dielectric_scatter(d, n, mat->ior, or_u01(r[2]), nd);
        }
        if (k >= rd->rr_start) {
            float q = fminf(1.0f, fmaxf(fmaxf(beta[0], beta[1]), beta[2]));
            if (or_u01(r[3]) >= q) break;
            for (int c = 0; c < 3; ++c) {
                beta[c] = beta[c] / q;
                beta64[c] /= (double)q;
            }
        }
        float p[3], side[3];
        for (int i = 0; i < 3; ++i) p[i] = o[i] + t * d[i];
        float sd = dot3f(nd, n);
        for (int i = 0; i < 3; ++i) side[i] = sd > 0.0f ? n[i] : -n[i];
        or_offset_origin(p, side, o);
        for (int i = 0; i < 3; ++i) d[i] = nd[i];
    }
}

void or_path_sample(const or_scene *sc, const or_camera *cam, const or_render_desc *rd,
                    uint32_t x, uint32_t y, uint32_t s, double L[3])
{
    cam_basis cb;
    camera_basis(cam, rd->width, rd->height, &cb);
    path_sample(sc, &cb, rd, x, y, s, L);
}

uint64_t or_render_rows(const or_scene *sc, const or_camera *cam, const or_render_desc *rd,
                        uint32_t y0, uint32_t ystep, double *out)
{
    cam_basis cb;
    camera_basis(cam, rd->width, rd->height, &cb);
    uint64_t paths = 0;
    if (ystep == 0) ystep = 1;
    for (uint32_t y = y0; y < rd->height; y += ystep) {
        for (uint32_t x = 0; x < rd->width; ++x) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (uint32_t s = 0; s < rd->spp; ++s) {
                double L[3];
                path_sample(sc, &cb, rd, x, y, s, L);
                for (int c = 0; c < 3; ++c) acc[c] += L[c];
                ++paths;
            }
            for (int c = 0; c < 3; ++c) out[((size_t)y * rd->width + x) * 3 + c] = acc[c] / (double)rd->spp;
        }
    }
    return paths;
}

/* First hit of the camera ray of one pixel (sample s); outputs at index i. */
static void primary_one(const or_scene *sc, const cam_basis *cb, uint32_t W, uint32_t H, uint32_t pix,
                        uint32_t s, uint64_t seed, size_t i, uint32_t *prim, uint32_t *inst, float *t,
                        float *normal)
{
    uint32_t r[4];
    rng4(pix, s, 0, OR_RNG_CAM, seed, r);
    float o[3], d[3], n[3], th;
    uint32_t pr, in;
    basis_ray(cb, W, H, pix % W, pix / W, or_u01(r[0]), or_u01(r[1]), o, d);
    if (or_closest_hit(sc, o, d, INFINITY, &th, &pr, &in, n)) {
        prim[i] = pr;
        inst[i] = in;
        t[i] = th;
        for (int a = 0; a < 3; ++a) normal[3 * i + a] = n[a];
    } else {
        prim[i] = 0xffffffffu;
        inst[i] = 0xffffffffu;
        t[i] = INFINITY;
        for (int a = 0; a < 3; ++a) normal[3 * i + a] = 0.0f;
    }
}

void or_trace_primary(const or_scene *sc, const or_camera *cam, uint32_t W, uint32_t H,
                      uint32_t s, uint64_t seed, uint32_t *prim, uint32_t *inst, float *t,
                      float *normal)
{
    cam_basis cb;
    camera_basis(cam, W, H, &cb);
    for (uint32_t pix = 0; pix < W * H; ++pix) primary_one(sc, &cb, W, H, pix, s, seed, pix, prim, inst, t, normal);
}

void or_trace_pixels(const or_scene *sc, const or_camera *cam, uint32_t W, uint32_t H, uint32_t s,
                     uint64_t seed, const uint32_t *pixels, uint64_t n, uint32_t *prim, uint32_t *inst,
                     float *t, float *normal)
{
    cam_basis cb;
    camera_basis(cam, W, H, &cb);
    for (uint64_t i = 0; i < n; ++i) primary_one(sc, &cb, W, H, pixels[i], s, seed, (size_t)i, prim, inst, t, normal);
}
