/*
 * A plain C client of include/vdi.h (no Python): create a VDI from host
 * arrays, render it exactly and as a preview into device memory, read the
 * image back and check it against the closed form, and check an error path.
 *
 * The VDI: 48 x 32 lists, N_S = 2, every list holding two supersegments of a
 * slab between constant V_O depths (Section 2.3).  Rendered from V_O itself,
 * each piece has length ratio l = 1 (Eq. 2), so every pixel is exactly
 * "first over second":
 *   C = a1 c1 + (1 - a1) a2 c2,  A = 1 - (1 - a1)(1 - a2).
 * Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "vdi.h"

#define W 48
#define H 32
#define NS 2

static int fail(const char *what)
{
    fprintf(stderr, "abi_client: %s (%s)\n", what, vdi_last_error());
    return 1;
}

int main(void)
{
    static uint8_t count[H * W];
    static float depth[NS * H * W * 2], rgba[NS * H * W * 4];
    const float f[NS] = {1.2f, 1.5f}, b[NS] = {1.4f, 1.8f}, a[NS] = {0.5f, 0.25f};
    const float c[NS][3] = {{0.9f, 0.1f, 0.1f}, {0.2f, 0.6f, 0.8f}};
    for (int li = 0; li < H * W; ++li) {
        count[li] = NS;
        for (int j = 0; j < NS; ++j) {
            const size_t o = (size_t)j * H * W + li;
            depth[2 * o] = f[j];
            depth[2 * o + 1] = b[j];
            rgba[4 * o] = c[j][0];
            rgba[4 * o + 1] = c[j][1];
            rgba[4 * o + 2] = c[j][2];
            rgba[4 * o + 3] = a[j];
        }
    }
    vdi_camera cam = {{0.0f, 0.0f, 1.5f}, {0.0f, 0.0f, 0.0f}, {0.0f, 1.0f, 0.0f}, 50.0f, 0.1f};
    vdi_desc d;
    memset(&d, 0, sizeof d);
    d.width = W;
    d.height = H;
    d.max_supersegments = NS;
    d.camera_VO = cam;
    for (int k = 0; k < 3; ++k) {
        d.aabb_min[k] = -2.0f;
        d.aabb_max[k] = 2.0f;
    }
    d.count = count;
    d.depth = depth;
    d.rgba = rgba;
    d.rgba_fmt_in = VDI_F32;
    d.rgba_fmt_store = VDI_F32;
    /* Depth slices whose faces are the supersegments' faces: the preview's
     * samples then tile each supersegment exactly (its exponents sum to 1). */
    static const float gz[6] = {1.0f, 1.2f, 1.4f, 1.5f, 1.8f, 2.0f};
    d.grid_k = 8;
    d.grid_nz = 5;
    d.grid_z = gz;
    d.validate = 1;

    vdi_t v = NULL;
    if (vdi_create(&d, &v) != VDI_OK) return fail("vdi_create");
    vdi_info_t info;
    if (vdi_get_info(v, &info) != VDI_OK || info.supersegments != (uint64_t)NS * H * W) return fail("vdi_get_info");

    float *dev = NULL;
    static float img[H * W * 4];
    if (hipMalloc((void **)&dev, sizeof img) != hipSuccess) return fail("hipMalloc");
    const float A = 1.0f - (1.0f - a[0]) * (1.0f - a[1]);
    float want[4];
    for (int m = 0; m < 3; ++m) want[m] = a[0] * c[0][m] + (1.0f - a[0]) * a[1] * c[1][m];
    want[3] = A;
    /* Exact, then the preview at D_R = 0.5 (point samples inside each supersegment). */
    const float modes[2] = {0.0f, 0.5f};
    for (int mi = 0; mi < 2; ++mi) {
        if (vdi_render(v, &cam, W, H, 1.0f, modes[mi], dev, NULL) != VDI_OK) return fail("vdi_render");
        if (hipMemcpy(img, dev, sizeof img, hipMemcpyDeviceToHost) != hipSuccess) return fail("hipMemcpy");
        double worst = 0.0;
        for (int i = 0; i < H * W * 4; ++i) {
            const double e = fabs((double)img[i] - (double)want[i % 4]);
            if (e > worst) worst = e;
        }
        printf("abi_client: D_R = %.1f: max |d| = %.3g against the closed form\n", modes[mi], worst);
        if (!(worst <= 1e-5)) return fail("image differs from the closed form");
    }
    /* Error path: a null camera is rejected before any device work, with a reason. */
    if (vdi_render(v, NULL, W, H, 1.0f, 0.0f, dev, NULL) != VDI_ERR_ARG || vdi_last_error()[0] == '\0')
        return fail("null camera not rejected");
    if (hipFree(dev) != hipSuccess) return fail("hipFree");
    if (vdi_destroy(v) != VDI_OK) return fail("vdi_destroy");
    printf("abi_client: ok\n");
    return 0;
}
