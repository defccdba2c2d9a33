/* Plain-C client of the library's C ABI (include/npt.h): compiled as C99
 * with every warning an error and linked against libnpt.so by
 * tests/test_abi_c.py.  A host-only context (device -1) needs no GPU: it
 * uploads a two-triangle quad, builds a 4-wide and a binary BVH on the host,
 * reads the summary back, and checks the documented status codes and error
 * messages of invalid calls.  Prints "ok" and returns 0 when every check
 * holds. */
#include <stdio.h>
#include <string.h>

#include "npt.h"

static int failures = 0;

static void expect(int got, int want, const char *what, npt_ctx *ctx) {
    if (got != want) {
        printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, ctx ? npt_last_error(ctx) : "");
        ++failures;
    }
}

int main(void) {
    npt_ctx *ctx = NULL;
    const float xyz[12] = {0, 0, 0, 1, 0, 0, 1, 1, 0, 0, 1, 0};
    const uint32_t tri[6] = {0, 1, 2, 0, 2, 3};
    const uint32_t bad_tri[3] = {0, 1, 7};
    const npt_material mat = {NPT_LAMBERT, {0.5f, 0.5f, 0.5f}, {0, 0, 0}, 1.0f};
    npt_bvh_params bp;
    uint64_t nodes = 0, leaves = 0, slots = 0;
    uint32_t depth = 0, width = 0;
    float out[3];
    const char *msg;

    expect(npt_create(&ctx, -1), NPT_OK, "create host-only", NULL);
    if (!ctx) return 1;
    expect(npt_build_bvh(ctx, NULL, NULL), NPT_E_NO_SCENE, "build without geometry", ctx);
    msg = npt_last_error(ctx);
    if (!msg || strlen(msg) == 0) {
        printf("FAIL empty error message\n");
        ++failures;
    }
    expect(npt_scene_triangles(ctx, xyz, 4, bad_tri, 1, NULL), NPT_E_INVALID_ARG, "vertex index out of range", ctx);
    expect(npt_scene_triangles(ctx, xyz, 4, tri, 2, NULL), NPT_OK, "triangles", ctx);
    expect(npt_scene_materials(ctx, &mat, 1), NPT_OK, "materials", ctx);

    memset(&bp, 0, sizeof bp);
    bp.max_leaf = 1;
    bp.width = 4;
    /* the host build happens; only the upload needs a device */
    expect(npt_build_bvh(ctx, &bp, NULL), NPT_E_NO_DEVICE, "build on a host-only context", ctx);
    expect(npt_bvh_info(ctx, &nodes, &leaves, &depth, &slots, &width), NPT_OK, "bvh info", ctx);
    if (leaves != 2 || slots != 2 || width != 4 || nodes < 1) {
        printf("FAIL bvh info: nodes %llu leaves %llu slots %llu width %u\n", (unsigned long long)nodes,
               (unsigned long long)leaves, (unsigned long long)slots, width);
        ++failures;
    }
    bp.width = 2;
    expect(npt_build_bvh(ctx, &bp, NULL), NPT_E_NO_DEVICE, "binary build on a host-only context", ctx);
    expect(npt_bvh_info(ctx, NULL, &leaves, NULL, NULL, &width), NPT_OK, "bvh info, some outputs NULL", ctx);
    if (leaves != 2 || width != 2) {
        printf("FAIL binary bvh info: leaves %llu width %u\n", (unsigned long long)leaves, width);
        ++failures;
    }
    bp.width = 3;
    expect(npt_build_bvh(ctx, &bp, NULL), NPT_E_INVALID_ARG, "width 3", ctx);

    expect(npt_render(ctx, 0, 4, 1, 1, 1, out, NULL), NPT_E_INVALID_ARG, "render width 0", ctx);
    expect(npt_set_env_mode(ctx, 9), NPT_E_INVALID_ARG, "unknown env mode", ctx);
    expect(npt_nif_set_precision(ctx, NPT_FP8), NPT_E_UNSUPPORTED, "FP8 without a device", ctx);
    expect(npt_destroy(ctx), NPT_OK, "destroy", NULL);
    expect(npt_create(NULL, -1), NPT_E_INVALID_ARG, "create without an output pointer", NULL);

    if (failures == 0) printf("ok\n");
    return failures == 0 ? 0 : 1;
}
