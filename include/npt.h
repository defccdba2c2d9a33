/*
 * npt.h -- C ABI of libnpt, an MI355X (gfx950) neural path tracer after
 * "Towards Neural Path Tracing in SRAM" (Pupilli, 2023).
 *
 * Conventions (all calls):
 *   - Every call returns an int status: NPT_OK (0) or a negative NPT_E_* code.
 *     Nothing throws across the ABI (a host allocation failure inside a call
 *     returns NPT_E_OOM).  npt_last_error() returns a message owned by the
 *     context, valid until the next call on that context.
 *   - Host input arrays are copied during the call; the caller keeps ownership.
 *   - Device output buffers are caller-owned (e.g. the data pointer of a
 *     torch.cuda tensor).  `stream` is a hipStream_t (NULL = the null stream);
 *     calls that take a stream only enqueue work on it and return; the caller
 *     synchronises before reading outputs.  Calls without a stream are
 *     synchronous.
 *   - One context per host thread; a context owns all of its device scratch.
 *   - A failed call leaves the context usable (its previous state intact).
 */
#ifndef NPT_H
#define NPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define NPT_OK 0
#define NPT_E_INVALID_ARG (-1) /* bad pointer, size, enum or overflow          */
#define NPT_E_NO_SCENE (-2)    /* render / BVH build before geometry           */
#define NPT_E_NO_ENV (-3)      /* render before env map or NIF weights         */
#define NPT_E_OOM (-4)         /* host or device allocation failed             */
#define NPT_E_HIP (-5)         /* HIP runtime error                            */
#define NPT_E_UNSUPPORTED (-6) /* e.g. FP8 on a device without gfx950 FP8 MFMA */
#define NPT_E_NAN_INPUT (-7)   /* NaN or Inf in uploaded floats                */
#define NPT_E_NO_DEVICE (-8)   /* no usable GPU (host-only context)           */
#define NPT_E_STATE (-9)       /* call order, e.g. render before npt_build_bvh */

/* ---- enums --------------------------------------------------------------- */
enum { NPT_LAMBERT = 0, NPT_MIRROR = 1, NPT_DIELECTRIC = 2, NPT_EMITTER = 3 };
enum { NPT_ENV_MAP = 0, NPT_ENV_NIF = 1, NPT_ENV_NONE = 2 };
enum { NPT_FP32 = 0, NPT_FP16 = 1, NPT_BF16 = 2, NPT_FP8 = 3 };

typedef struct npt_ctx npt_ctx;

/* Surface material (Sec. 3.1: diffuse, mirror and dielectric surfaces; the
 * paper adds emission only when a path hits an emitter by chance).
 * type: NPT_*; albedo: Lambertian reflectance or mirror tint (dielectrics
 * ignore it); emission: radiance emitted from the front face (the side the
 * triangle's counter-clockwise normal points to, the outside of a sphere);
 * ior: dielectric index of refraction (outside medium has index 1).
 * NPT_EMITTER emits and ends the path. */
typedef struct {
    uint32_t type;
    float albedo[3];
    float emission[3];
    float ior;
} npt_material;

/* Instance of an object-space mesh (blas_id from npt_scene_blas_triangles):
 * world = translate + scale * object.  Uniform scale > 0 only. */
typedef struct {
    uint32_t blas_id;
    float translate[3];
    float scale;
} npt_instance;

/* Pinhole camera; vfov_deg is the full vertical field of view. */
typedef struct {
    float eye[3];
    float look_at[3];
    float up[3];
    float vfov_deg;
} npt_camera;

/* Host BVH build (Sec. 3.1.4 builds a BVH2 on the host).  bins: SAH bins per
 * axis (4..256, 0 = 32); max_leaf: primitives per leaf (1..8, 0 = 4);
 * lds_levels: top tree levels staged in LDS by the traversal kernel (0..8,
 * 0 = none; of an instanced scene: levels of its top tree); width:
 * children per node, 2 (the paper's BVH2) or 4 (the binary SAH tree
 * collapsed to 4-wide nodes), 0 = 4.  node_format (width 4; Q8 and
 * FP16_CORNER with lds_levels 0): NPT_NODES_FP32 (112-byte nodes, FP32
 * boxes) or
 * NPT_NODES_FP16_EXTENT (96-byte nodes: FP32 lower planes and binary16
 * extents rounded up so that the FP32 sum lo + ext covers the box, after
 * Sec. 3.1.4; NPT_E_UNSUPPORTED if an extent exceeds 65504) or NPT_NODES_Q8
 * (64-byte nodes: per node and axis an FP32 origin and a power-of-two step,
 * 8-bit child planes rounded outward, after Ylitie et al. 2017) or
 * NPT_NODES_FP16_CORNER (80-byte nodes: per node and axis an FP32 corner,
 * the children's lower and upper planes as binary16 offsets from it, rounded
 * outward so that the FP32 sum corner + offset covers the box: the relative
 * coordinates of Sec. 3.1.4 for both planes; NPT_E_UNSUPPORTED if a node
 * spans more than 65504 on an axis). */
#define NPT_NODES_FP32 0
#define NPT_NODES_FP16_EXTENT 1
#define NPT_NODES_Q8 2
#define NPT_NODES_FP16_CORNER 3
typedef struct {
    uint32_t bins;
    uint32_t max_leaf;
    uint32_t lds_levels;
    uint32_t width;
    uint32_t node_format;
    uint32_t threads; /* host threads of the build, 0 = all (at most 64); the
                         tree is the same byte for byte on any number */
} npt_bvh_params;

/* HDR-NIF shape (Sec. 3.2): 4*n_freq Fourier features -> layers x
 * [dense hidden + ReLU] -> dense 3 -> fixed colour matrix to log-space RGB.
 * Supported: n_freq 1..16 (frequencies round(2^((k+1)/2)), k < n_freq);
 * hidden 32..1024, a multiple of 32; layers 1..8.  skip: 0, or the hidden
 * layer (1..layers-1) whose input is the previous layer's output followed by
 * the features again (the paper's skip-concat, Sec. 3.2); that previous
 * layer has hidden - 4 n_freq outputs (needs hidden > 4 n_freq), so the
 * concatenation is hidden wide.  Four shapes
 * (n_freq/hidden/layers/skip) run on an LDS-resident MFMA kernel in FP32,
 * FP16, BF16 or FP8: 16/96/5/0 (the default), 10/128/4/2 (the paper's
 * network: 40-d features, four dense-ReLU layers, the second narrowed to 88
 * outputs; with the output layer five trainable layers, 50,011 parameters =
 * 97.7 KiB in FP16), 16/128/4/2 and 16/64/2/0.  Every other shape, or layered = 1,
 * runs on layer-serial MFMA GEMMs in FP32, FP16 or BF16 (Sec. 4.6 sweeps
 * model sizes); uploading such a shape while FP8 is selected, or selecting
 * FP8 for it, fails with NPT_E_UNSUPPORTED.
 * colour: the space the
 * network's three outputs live in (Sec. 4.3 compares them):
 * NPT_COLOUR_YUV (default; BT.601 analogue, R = Y + 1.13983 V,
 * G = Y - 0.39465 U - 0.58060 V, B = Y + 2.03211 U), NPT_COLOUR_RGB
 * (identity), NPT_COLOUR_YCOCG (R = Y + Co - Cg, G = Y + Cg, B = Y - Co - Cg).
 * The matrix applies to training, inference and grid evaluation alike. */
#define NPT_COLOUR_YUV 0
#define NPT_COLOUR_RGB 1
#define NPT_COLOUR_YCOCG 2
typedef struct {
    uint32_t n_freq;
    uint32_t hidden;
    uint32_t layers;
    uint32_t colour;
    uint32_t layered;
    uint32_t skip;
} npt_nif_desc;

/* NIF training (Sec. 3.2.1): uniform (u,v) samples of the uploaded map,
 * targets log1p(bilinear), Huber loss, Adam (FP32 moments).
 * grad_prec: NPT_FP32 / NPT_FP16 / NPT_BF16 operands of the GEMMs (FP32
 * accumulation).  master_prec: NPT_FP32 master weights (default), or
 * NPT_FP16 as on the paper's IPU: the master is rounded to the nearest
 * binary16 first, and every Adam update, taken in FP32, is rounded to
 * binary16 stochastically with u from the Philox stream (parameter index,
 * Adam step, 0, 4) under the seed.  Zero fields take the defaults in brackets:
 * batch [65536; a multiple of 2048], samples [2^24], lr [1e-3], beta1 [0.9], beta2 [0.999],
 * eps [1e-7], huber_delta [1e-3], loss_scale [16384 with FP16 GEMM operands, the
 * scale Sec. 3.2.1 trains with; 1 otherwise, where the range of FP32 / BF16
 * makes a power-of-two scale cancel exactly].  The loss scale multiplies the
 * per-sample output gradients before the backward GEMMs and is divided out
 * of the weight gradients.  path: NPT_TRAIN_AUTO (0) takes the fused
 * two-launch step (forward, backward and per-workgroup gradient sums in one
 * kernel; fixed-order sums and Adam in a second) for the four LDS-resident
 * shapes with FP16 operands, and layer-by-layer MFMA GEMMs otherwise;
 * NPT_TRAIN_LAYERED (1) always takes the layer-by-layer GEMMs.  Both round at
 * the same points and are deterministic; their results differ only in the
 * order of FP32 sums. */
#define NPT_TRAIN_AUTO 0
#define NPT_TRAIN_LAYERED 1
typedef struct {
    uint32_t batch;
    uint64_t samples;
    float lr, beta1, beta2, eps, huber_delta;
    uint64_t seed;
    uint32_t grad_prec;
    float loss_scale;
    uint32_t master_prec;
    uint32_t path;
} npt_train_params;

typedef struct {
    uint32_t steps;      /* optimiser steps taken                    */
    uint32_t step_total; /* Adam step counter after the call         */
    float first_loss;    /* mean Huber loss of the first batch       */
    float last_loss;     /* mean Huber loss of the last batch        */
    float ms;            /* device time of the call                  */
} npt_train_stats;

/* Render options.  rr_start: first depth with Russian roulette (Sec. 4: 3);
 * samples_per_pass: samples traced together (0 = library default, sized
 * from the pool); pool_paths: upper bound on paths in flight (0 = 2^27,
 * 160 bytes of device queues per path, allocated as far as a render needs
 * them);
 * kernel_timing: 1 = time every extend (closest hit), shade and
 * environment launch with HIP events on the render stream
 * (npt_stats.ms_trace / ms_shade / ms_env);
 * count_visits: 1 = use the counting variant of the extend kernel
 * (npt_stats.node_visits / prim_tests; slower, for byte accounting only).
 * sort_rays: 1 = before each extend launch of depth 2 and beyond, sort every
 * chunk of 1024 queued rays by direction octant, origin (Morton order over a
 * 32^3 grid on the scene bounds) and direction, and trace them in that order
 * (hits, shading and images unchanged; the sort's time counts as trace time;
 * npt_render_noalloc ignores it). */
typedef struct {
    uint32_t rr_start;
    uint32_t samples_per_pass;
    uint32_t pool_paths;
    uint32_t kernel_timing;
    uint32_t count_visits;
    uint32_t sort_rays;
} npt_render_options;

#define NPT_MAX_DEPTH 64

/* Counters of the last render (read back synchronously by npt_get_stats). */
typedef struct {
    uint64_t paths;                      /* W*H*spp                               */
    uint64_t rays[NPT_MAX_DEPTH];        /* rays traced at depth k (index k-1)    */
    uint64_t escaped[NPT_MAX_DEPTH];     /* rays lit by the environment at depth k */
    uint64_t env_queries;                /* total environment lookups / NIF queries */
    uint32_t passes;
    uint32_t samples_per_pass;
    float ms_total;                      /* device time of the last render         */
    /* kernel_timing: summed event time and launch counts (trace = the
     * extend kernel: BVH traversal and primitive tests) */
    float ms_trace, ms_env;
    uint32_t trace_launches, env_launches;
    /* count_visits: BVH nodes fetched / primitives tested at depth k */
    uint64_t node_visits[NPT_MAX_DEPTH];
    uint64_t prim_tests[NPT_MAX_DEPTH];
    /* kernel_timing: the shade kernel (emission, BSDF sampling, roulette) */
    float ms_shade;
    uint32_t shade_launches;
    /* kernel_timing: environment (map or NIF) time of the queries of depth k
     * (index k-1), summed over passes; their count is escaped[k-1] */
    float ms_env_depth[NPT_MAX_DEPTH];
} npt_stats;

/* ---- context ------------------------------------------------------------- */
/* device >= 0: HIP device index.  device = -1: host-only context (scene and
 * BVH calls work, anything needing a GPU returns NPT_E_NO_DEVICE). */
int npt_create(npt_ctx **out, int device);
int npt_destroy(npt_ctx *ctx);
const char *npt_last_error(npt_ctx *ctx);

/* ---- scene (Sec. 3.1.1 scene data; Fig. 1 scenes) -------------------------- */
/* Base (instance 0) triangles: xyz [nv][3] FP32, tri [nt][3] vertex indices,
 * mat_of_tri [nt] material ids (NULL = all 0).  Primitive ids 0..nt-1.
 * Replaces any previous base triangles.  NPT_E_NAN_INPUT on NaN/Inf;
 * NPT_E_INVALID_ARG on out-of-range indices. */
int npt_scene_triangles(npt_ctx *ctx, const float *xyz, uint64_t nv, const uint32_t *tri,
                        uint64_t nt, const uint32_t *mat_of_tri);
/* Base spheres: cxyzr [n][4] (centre, radius > 0), mat [n] (NULL = 0).
 * Primitive ids nt..nt+n-1 after the base triangles. */
int npt_scene_spheres(npt_ctx *ctx, const float *cxyzr, uint64_t n, const uint32_t *mat);
/* Object-space mesh for instancing (Sec. 3.1.4 scenes; the large-BVH
 * scene of Fig. 1 places copies of one mesh): xyz [nv][3], tri [nt][3],
 * mat_of_tri [nt] (NULL = 0).  blas_id must be an existing id (replaced) or
 * the next one (appended); nt > 0.  Hits on instance k report primitive ids
 * 0..nt-1 of its mesh.  Copied; the caller keeps its arrays. */
int npt_scene_blas_triangles(npt_ctx *ctx, uint32_t blas_id, const float *xyz, uint64_t nv,
                             const uint32_t *tri, uint64_t nt, const uint32_t *mat_of_tri);
/* Instances k = 0..n-1 get instance id k+1 (the base geometry is 0).
 * world = translate + scale * object, scale > 0 (NPT_E_INVALID_ARG
 * otherwise or for an unknown blas_id; NPT_E_NAN_INPUT on NaN/Inf).  A scene
 * with instances is traced through a two-level BVH (4-wide top tree over
 * object boxes, one 4-wide tree per mesh; the object-space ray is
 * ((o - translate) * r, d * r) with r = 1 / scale rounded to FP32 once, so
 * t is shared by both spaces);
 * npt_build_bvh then requires width 4 (or 0), and lds_levels > 0 (top
 * tree levels in LDS) binary16-extent nodes (NPT_E_UNSUPPORTED otherwise).
 * n = 0 removes all instances. */
int npt_scene_instances(npt_ctx *ctx, const npt_instance *inst, uint32_t n);
int npt_scene_materials(npt_ctx *ctx, const npt_material *m, uint32_t n);
/* Builds the BVH(s) on the host (binned SAH), flattens them and uploads on
 * `stream`.  NPT_E_NO_SCENE if no geometry; NPT_E_NO_DEVICE only for the
 * upload on a host-only context (the host build still happens). */
int npt_build_bvh(npt_ctx *ctx, const npt_bvh_params *p, void *stream);
/* Host-side BVH summary: nodes, leaves, max depth (root = 0), primitive
 * slots, children per node.  Any output may be NULL. */
int npt_bvh_info(npt_ctx *ctx, uint64_t *nodes, uint64_t *leaves, uint32_t *max_depth,
                 uint64_t *prim_slots, uint32_t *width);
/* The flattened BVH as built on the host, in the device layout the traversal
 * reads (nodes, then primitive slots, then for a two-level scene the
 * instance records): bytes copied to host memory.  Call with NULL buffers to
 * get the three sizes; a buffer smaller than its size is NPT_E_INVALID_ARG.
 * NPT_E_STATE before npt_build_bvh.  The arrays depend only on the scene and
 * the build parameters, not on the build's thread count. */
int npt_bvh_export(npt_ctx *ctx, void *nodes, uint64_t *node_bytes, void *slots, uint64_t *slot_bytes,
                   void *records, uint64_t *record_bytes);
int npt_set_camera(npt_ctx *ctx, const npt_camera *cam);
int npt_set_render_options(npt_ctx *ctx, const npt_render_options *opt);

/* ---- environment (Sec. 3.3) ------------------------------------------------ */
/* Equirectangular FP32 RGB map rgb [h][w][3] (row j = polar angle, column i
 * = azimuth, texel centres at half-integers).  Kept on the device for lookup
 * and training.  NPT_E_NAN_INPUT on NaN/Inf or negative radiance. */
int npt_env_upload(npt_ctx *ctx, const float *rgb, uint32_t w, uint32_t h, void *stream);
/* NPT_ENV_MAP: bilinear lookup; NPT_ENV_NIF: the HDR-NIF; NPT_ENV_NONE: no
 * environment light (escaped paths add nothing; closed scenes). */
int npt_set_env_mode(npt_ctx *ctx, int mode);

/* ---- HDR-NIF (Sec. 3.2) ----------------------------------------------------- */
/* params_fp32: [W1, b1, ..., W_{L+1}, b_{L+1}], W row-major [out][in], n
 * values (43,779 for 16/96/5; with F = 4 n_freq: F H + H + (L - 1)(H^2 + H)
 * + 3 H + 3, less F (H + 1) with a skip-concat: 50,011 for the paper's
 * 10/128/4 network with the features at layer 2).  Becomes the FP32 master copy; Adam state is reset;
 * the inference pack of the current precision is rebuilt; desc->colour
 * selects the output colour space (NPT_E_INVALID_ARG if unknown). */
int npt_nif_upload(npt_ctx *ctx, const npt_nif_desc *desc, const float *params_fp32,
                   uint64_t n, void *stream);
/* Copies the FP32 master parameters to host memory (synchronous). */
int npt_nif_download(npt_ctx *ctx, float *params_fp32, uint64_t n);
/* Training state of the uploaded network (checkpoint and resume of the
 * training of Sec. 3.2.1): the FP32 master parameters, Adam's first and
 * second moments (n values each, the npt_nif_upload order) and the number of
 * Adam steps taken, copied to host memory (synchronous).  Any of params, m,
 * v, step may be NULL.  NPT_E_STATE without an uploaded network,
 * NPT_E_INVALID_ARG if n is not the network's parameter count. */
int npt_nif_get_state(npt_ctx *ctx, float *params_fp32, float *m, float *v, uint64_t n, uint32_t *step);
/* Restores a training state taken by npt_nif_get_state into the uploaded
 * network, which must have the same shape (n parameters): master
 * parameters, moments and step count are copied from host memory (the
 * caller keeps them), the inference pack is rebuilt.  Training on from a
 * restored state takes the steps an uninterrupted run would have taken,
 * bit for bit.  NPT_E_NAN_INPUT for non-finite values or negative second
 * moments. */
int npt_nif_set_state(npt_ctx *ctx, const float *params_fp32, const float *m, const float *v, uint64_t n,
                      uint32_t step, void *stream);
/* Inference precision NPT_FP32 / FP16 / BF16 / FP8 (OCP E4M3 weights and
 * activations with power-of-two scales).  Packs the weights. */
int npt_nif_set_precision(npt_ctx *ctx, int prec);
/* Copies the dequantised inference weights (the values the MFMA kernel
 * multiplies, in the npt_nif_upload order) to host memory. */
int npt_nif_get_dequantized(npt_ctx *ctx, float *params, uint64_t n);
/* Trains in place on the uploaded env map (Sec. 3.2.1). */
int npt_nif_train(npt_ctx *ctx, const npt_train_params *p, npt_train_stats *out, void *stream);
/* Loss and gradient of training step `step`'s batch at the current weights,
 * without updating them: d_grad [n params] FP32 device, d_loss [1] FP32
 * device (caller-owned). */
int npt_nif_train_grad(npt_ctx *ctx, const npt_train_params *p, uint32_t step, float *d_grad,
                       float *d_loss, void *stream);
/* Evaluates the NIF at the centres of a gw x gh (u,v) grid against the
 * bilinear map: out[0] = mean log-radiance MSE (log1p domain), out[1] =
 * RGB PSNR in the log domain (peak = max log1p of the map).  Synchronous. */
int npt_nif_eval_grid(npt_ctx *ctx, uint32_t gw, uint32_t gh, float *out2, void *stream);
/* NIF radiance (or bilinear map if mode == NPT_ENV_MAP) for n world
 * directions d_dirs [n][3] FP32 device -> d_rgb [n][3] FP32 device. */
int npt_env_query(npt_ctx *ctx, int mode, const float *d_dirs, uint64_t n, float *d_rgb,
                  void *stream);

/* ---- rendering (Sec. 3.1, 3.3, 4) --------------------------------------------- */
/* Monte-Carlo path tracing: W*H pixels, spp samples, paths of at most
 * max_depth segments (1..64), Philox seed.  d_radiance: [H][W][3] FP32
 * device, caller-owned, overwritten with the per-pixel mean.
 * NPT_E_INVALID_ARG: W*H*spp overflows 2^40, zero sizes, max_depth 0 or > 64.
 * NPT_E_NO_SCENE / NPT_E_STATE: no geometry / BVH not built.
 * NPT_E_NO_ENV: environment mode without a map or NIF weights. */
int npt_render(npt_ctx *ctx, uint32_t width, uint32_t height, uint32_t spp, uint32_t max_depth,
               uint64_t seed, float *d_radiance, void *stream);
/* Progressive rendering and resume by sample index (the Monte-Carlo
 * estimate of Sec. 3.1 is a per-pixel mean over independent samples, each
 * drawn from its own Philox stream keyed by pixel and sample index):
 * adds samples [sample0, sample0 + samples) of every pixel to the running
 * sums d_sum [H][W][4] FP32 (RGB sums and an unused fourth word, zeroed
 * when sample0 == 0; device, caller-owned, 16-byte aligned), overwriting
 * them when sample0 == 0.  When d_radiance ([H][W][3] FP32 device) is not NULL the
 * mean over samples [0, sample0 + samples) is written there.  Each pixel's
 * samples are added in sample order whatever the split, so renders of
 * consecutive ranges on one d_sum give npt_render's image of
 * sample0 + samples spp bit for bit (same seed, depth and scene); d_sum may
 * be copied to host memory and back in between to checkpoint a render.
 * NPT_E_INVALID_ARG: null or misaligned d_sum, sample0 + samples >= 2^32,
 * and npt_render's argument errors with spp = samples.  Other errors and
 * statistics (paths = W*H*samples) as npt_render. */
int npt_render_samples(npt_ctx *ctx, uint32_t width, uint32_t height, uint32_t sample0, uint32_t samples,
                       uint32_t max_depth, uint64_t seed, float *d_sum, float *d_radiance, void *stream);

/* ---- allocation-free rendering ------------------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * render as npt_render, bit for bit, with the path pool, accumulator and
 * counters taken from a fixed scratch array of NPT_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that the library holds on every GPU it runs on until the process
 * ends.  Nothing is allocated on the device, and no hipMalloc / hipFree is
 * called.  Samples per pass are as many as fit (about 176 bytes per pixel per
 * sample of the pass, at most npt_render_options.samples_per_pass when set);
 * an image of more than about 380,000 pixels does not fit: NPT_E_INVALID_ARG.
 * Environment mode NPT_ENV_NIF needs a network shape with an LDS-resident
 * kernel (the layer-serial path allocates): NPT_E_UNSUPPORTED otherwise.
 * Other errors as npt_render.  Every call on one GPU shares that GPU's
 * array (the kernels clear the counters and the accumulator themselves), so
 * calls that overlap on one GPU -- other contexts, other threads, other
 * streams -- race and must be serialised by the caller.  No kernel timing:
 * npt_get_stats afterwards reports paths, passes and samples per pass. */
#define NPT_NOALLOC_SCRATCH_BYTES (64u << 20)
int npt_render_noalloc(npt_ctx *ctx, uint32_t width, uint32_t height, uint32_t spp, uint32_t max_depth,
                       uint64_t seed, float *d_radiance, void *stream);
/* Primary hits of sample `sample` (Table 3-style checks): d_prim / d_inst
 * [H*W] u32 (0xFFFFFFFF on miss), d_t [H*W] FP32 (+inf on miss), d_normal
 * [H*W][3] geometric normal (0 on miss).  Any output may be NULL. */
int npt_trace_primary(npt_ctx *ctx, uint32_t width, uint32_t height, uint32_t sample,
                      uint64_t seed, uint32_t *d_prim, uint32_t *d_inst, float *d_t,
                      float *d_normal, void *stream);
int npt_get_stats(npt_ctx *ctx, npt_stats *out);

#ifdef __cplusplus
}
#endif
#endif
