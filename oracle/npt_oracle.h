/*
 * npt_oracle.h -- CPU oracle for the neural path tracer of
 * "Towards Neural Path Tracing in SRAM" (Pupilli, 2023).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library.  It shares no
 * code, header, table or helper with the GPU library; the two meet only on
 * the seeded inputs both are given.
 *
 * What it computes, and in which precision:
 *   - the Monte-Carlo path-tracing estimator of Sec. 3.1 (no light sampling,
 *     Russian roulette from depth 3 as in Sec. 4), with every ray operation
 *     (camera, intersection, BSDF sampling, roulette decision, origin offset)
 *     in IEEE FP32 with a fixed operation order and no contraction -- the
 *     paper's own ray kernels are FP32 and are checked against the same
 *     kernels on a CPU in Sec. 4.2 (Table 3);
 *   - radiance accumulation, environment lookup and HDR-NIF evaluation in
 *     FP64 (Sec. 3.2, 3.3);
 *   - NIF training (Sec. 3.2.1): forward, Huber loss, hand-written backward
 *     and Adam, all in FP64.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), one counter per
 * (pixel, sample, depth, purpose); the paper's IPU uses a hardware RNG
 * (Sec. 3.1.3, App. A.1), which is not reproducible, so a counter-based
 * generator stands in for it on both sides.
 *
 * Parity-pin status of every function is listed beside it.  A function
 * marked "parity unpinned" has no independent check.
 */
#ifndef NPT_ORACLE_H
#define NPT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* RNG purposes (the fourth counter word). */
enum { OR_RNG_CAM = 0, OR_RNG_SCATTER = 1, OR_RNG_TRAIN = 2, OR_RNG_SCENE = 3, OR_RNG_SROUND = 4 };

/* Material types. */
enum { OR_LAMBERT = 0, OR_MIRROR = 1, OR_DIELECTRIC = 2, OR_EMITTER = 3 };

/* Environment modes. */
enum { OR_ENV_MAP = 0, OR_ENV_NIF = 1, OR_ENV_CONST = 2 };

typedef struct {
    uint32_t type;
    float albedo[3];
    float emission[3];
    float ior;
} or_material;

typedef struct {
    uint32_t blas;       /* index of the instanced mesh (0-based) */
    float translate[3];
    float scale;
} or_instance;

typedef struct {
    float eye[3];
    float look_at[3];
    float up[3];
    float vfov_deg;
} or_camera;

/* NIF shape: 4*n_freq Fourier features -> `layers` x [dense `hidden` + ReLU]
 * -> dense 3 -> fixed 3x3 colour matrix to RGB.  colour: the space the
 * network's outputs live in (Sec. 4.3): OR_COLOUR_YUV (default), RGB, YCOCG.
 * skip: 0, or the hidden layer l (1..layers-1) whose input is the previous
 * layer's output followed by the features again (the skip-concat of Sec. 3.2);
 * the previous layer is narrowed to hidden - 4 n_freq outputs so that layer
 * l still reads `hidden` values (needs hidden > 4 n_freq). */
enum { OR_COLOUR_YUV = 0, OR_COLOUR_RGB = 1, OR_COLOUR_YCOCG = 2 };
typedef struct {
    uint32_t n_freq;
    uint32_t hidden;
    uint32_t layers;
    uint32_t colour;
    uint32_t skip;
} or_nif_shape;

typedef struct or_scene or_scene;

/* ---- Philox and uniforms (pinned: rocRAND host engine; U01 closed form) -- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float or_u01(uint32_t x);

/* ---- FP32 sin/cos of 2*pi*u (pinned: <= 2 ulp of libm FP64) ------------- */
void or_sincos2pi(float u, float *s, float *c);

/* ---- geometry primitives (pinned: FP64 closed forms, brute force) ------- */
int or_intersect_triangle(const float o[3], const float d[3], const float v0[3],
                          const float v1[3], const float v2[3], float tmax, float *t);
int or_intersect_sphere(const float o[3], const float d[3], const float c[3], float r,
                        float tmax, float *t);
void or_offset_origin(const float p[3], const float n[3], float out[3]);
void or_camera_ray(const or_camera *cam, uint32_t W, uint32_t H, uint32_t x, uint32_t y,
                   float jx, float jy, float o[3], float d[3]);

/* ---- BSDF pieces (pinned: Fresnel angle form, Snell, chi^2, closed forms) */
float or_fresnel_dielectric(float cos_i, float eta_i, float eta_t);
void or_onb(const float n[3], float t[3], float b[3]);
void or_cosine_sample(const float n[3], float u0, float u1, float out[3]);
/* Dielectric scatter: returns 1 if reflected, 0 if refracted. */
int or_dielectric_scatter(const float d[3], const float n_geom[3], float ior, float u,
                          float out[3]);

/* ---- environment (pinned: texel-centre exactness, round trip) ----------- */
void or_dir_to_uv(double dx, double dy, double dz, double *u, double *v);
void or_uv_to_dir(double u, double v, double d[3]);
void or_env_bilinear(const float *rgb, uint32_t w, uint32_t h, double u, double v, double out[3]);

/* ---- HDR-NIF (pinned: structural closed forms, finite differences) ------ */
uint64_t or_nif_param_count(const or_nif_shape *s);
uint32_t or_nif_frequency(uint32_t k);
void or_nif_features(const or_nif_shape *s, double u, double v, double *feat);
void or_yuv_to_rgb_matrix(double m[9]);
/* Row-major M with RGB = M * (network output) for an OR_COLOUR_* space. */
void or_colour_to_rgb_matrix(uint32_t colour, double m[9]);
/* Log-space RGB output z of the network (before expm1). */
void or_nif_forward(const or_nif_shape *s, const double *params, double u, double v, double z[3]);
/* Radiance = max(0, expm1(z)). */
void or_nif_radiance(const or_nif_shape *s, const double *params, double u, double v, double rgb[3]);
/* Reduced-precision inference (FP16 / BF16 / FP8 operands, exact sums). */
enum { OR_PREC_FP32 = 0, OR_PREC_FP16 = 1, OR_PREC_BF16 = 2, OR_PREC_FP8 = 3 };
enum { OR_FMT_NONE = 0, OR_FMT_F16 = 1, OR_FMT_BF16 = 2, OR_FMT_E4M3 = 3 };
/* Nearest value with ties to even in a binary format with frac_bits fraction
 * bits, minimum normal exponent emin and largest finite maxv; beyond maxv
 * the result saturates (saturate != 0) or is infinite. */
double or_round_format(double x, int frac_bits, int emin, double maxv, int saturate);
double or_round_to(double x, int fmt); /* OR_FMT_*: binary16, bfloat16, E4M3 (saturating) */
void or_round_array(const double *in, double *out, uint64_t n, int fmt);
/* FP8 weight scale: the largest s with maxabs * 2^s <= 448 (0 for maxabs 0). */
int or_nif_fp8_scale_exp(double maxabs);
/* The weights as rounded for inference at `prec` (biases unchanged). */
void or_nif_dequantize(const or_nif_shape *s, const double *params, int prec, double *out);
/* Forward pass with every layer input rounded to its operand format; deq
 * from or_nif_dequantize.  OR_PREC_FP32 is or_nif_forward. */
void or_nif_forward_q(const or_nif_shape *s, const double *deq, int prec, double u, double v, double z[3]);
void or_nif_radiance_q(const or_nif_shape *s, const double *deq, int prec, double u, double v, double rgb[3]);
double or_huber(double e, double delta);
double or_huber_grad(double e, double delta);
/* Mean Huber loss over n samples x 3 channels and its gradient w.r.t. params
 * (grad may be NULL).  uv: n x 2, target: n x 3 (log-space). */
double or_nif_loss_grad(const or_nif_shape *s, const double *params, uint64_t n,
                        const double *uv, const double *target, double delta, double *grad);
/* The same loss and gradient with the on-device trainer's matrix operands
 * rounded to prec (OR_PREC_FP16 / BF16; OR_PREC_FP32 rounds nothing): hidden-
 * layer weights, layer inputs and the back-propagated gradients at the
 * hidden layers' outputs (after the ReLU mask, loss scale loss_scale
 * applied); exact sums; the output layer on the given weights; gradient
 * divided by 3 n loss_scale.  Pinned: FP32 mode = or_nif_loss_grad; FP16 /
 * BF16 = a batched NumPy layer loop with library casts; BF16 independent of
 * the loss scale; FP16 closer to FP64 with the paper's scale than without. */
double or_nif_loss_grad_q(const or_nif_shape *s, const double *params, int prec, double loss_scale,
                          uint64_t n, const double *uv, const double *target, double delta, double *grad);
/* Training batch of Sec. 3.2.1: uniform (u,v) from the TRAIN Philox stream and
 * log1p(bilinear) targets.  uv: n x 2, target: n x 3. */
void or_nif_train_batch(const float *map, uint32_t w, uint32_t h, uint64_t seed, uint32_t step,
                        uint64_t n, double *uv, double *target);
/* One Adam step (Kingma & Ba 2015, Alg. 1); step is 1-based. */
void or_adam_step(uint64_t n, double *params, const double *grad, double *m, double *v,
                  uint32_t step, double lr, double beta1, double beta2, double eps);
/* binary16 round toward zero (saturating at 65504) and stochastic rounding
 * with u in [0,1) (FP16 master weights, Sec. 3.2.1). */
double or_fp16_toward_zero(double x);
double or_fp16_stochastic(double x, double u);
/* Adam step on FP16 master weights with stochastic rounding; step 1-based,
 * u of parameter i from Philox (i, step, 0, OR_RNG_SROUND) under seed. */
void or_adam_step_fp16_master(uint64_t n, double *params, const double *grad, double *m, double *v,
                              uint32_t step, double lr, double beta1, double beta2, double eps,
                              uint64_t seed);
/* One full training step; returns the loss before the update.  fp16_master:
 * master weights in binary16 (rounded to nearest first) with stochastic
 * rounding of the update. */
double or_nif_train_step(const or_nif_shape *s, double *params, double *m, double *v,
                         const float *map, uint32_t w, uint32_t h, uint64_t seed, uint32_t step,
                         uint64_t batch, double lr, double beta1, double beta2, double eps,
                         double delta, int fp16_master);

/* ---- scenes, closest hit and the render estimator ---------------------- */
/* accel: 0 = brute force over all primitives, 1 = the oracle's own median-split BVH. */
or_scene *or_scene_create(const float *verts, uint64_t nv, const uint32_t *tris, uint64_t nt,
                          const uint32_t *tri_mat, const float *spheres, uint64_t ns,
                          const uint32_t *sph_mat, const or_material *mats, uint32_t nmat,
                          int accel);
/* Register instanced mesh `blas` (object space, must be added in order 0,1,...). */
int or_scene_add_blas(or_scene *sc, const float *verts, uint64_t nv, const uint32_t *tris,
                      uint64_t nt, const uint32_t *tri_mat);
int or_scene_set_instances(or_scene *sc, const or_instance *inst, uint32_t n);
void or_scene_destroy(or_scene *sc);

/* Closest hit; returns 1 on hit.  inst = 0 for base geometry, k+1 for instance k. */
int or_closest_hit(const or_scene *sc, const float o[3], const float d[3], float tmax,
                   float *t, uint32_t *prim, uint32_t *inst, float n_geom[3]);

typedef struct {
    uint32_t width, height, spp, max_depth, rr_start;
    uint64_t seed;
    uint32_t env_mode;        /* OR_ENV_* */
    const float *env_map;     /* OR_ENV_MAP: w x h x 3 FP32 */
    uint32_t env_w, env_h;
    const double *nif_params; /* OR_ENV_NIF: dequantised parameters */
    or_nif_shape nif;
    double env_const[3];      /* OR_ENV_CONST */
    uint32_t nif_prec;        /* OR_ENV_NIF: OR_PREC_* of or_nif_forward_q */
} or_render_desc;

/* Renders rows y0, y0+ystep, ... into out (full W*H*3 FP64 image; other rows
 * untouched).  Returns the number of path samples traced. */
uint64_t or_render_rows(const or_scene *sc, const or_camera *cam, const or_render_desc *rd,
                        uint32_t y0, uint32_t ystep, double *out);
/* Same estimator for a single pixel/sample, returning L (FP64). */
void or_path_sample(const or_scene *sc, const or_camera *cam, const or_render_desc *rd,
                    uint32_t x, uint32_t y, uint32_t s, double L[3]);
/* Primary hits of sample s for all pixels: prim/inst = 0xffffffff on miss. */
void or_trace_primary(const or_scene *sc, const or_camera *cam, uint32_t W, uint32_t H,
                      uint32_t s, uint64_t seed, uint32_t *prim, uint32_t *inst, float *t,
                      float *normal);
/* or_trace_primary for a list of pixel indices (y * W + x); outputs [n]. */
void or_trace_pixels(const or_scene *sc, const or_camera *cam, uint32_t W, uint32_t H, uint32_t s,
                     uint64_t seed, const uint32_t *pixels, uint64_t n, uint32_t *prim, uint32_t *inst,
                     float *t, float *normal);

#ifdef __cplusplus
}
#endif
#endif
