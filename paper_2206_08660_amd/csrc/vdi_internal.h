// Internal types shared by the libvdi host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vdi.h"

namespace vdi {

// Transmittance at which a ray stops (early ray termination).
constexpr float kTTerm = 1e-5f;
// |F_O . d| below this: the ray keeps a constant V_O depth.
constexpr double kFlatZ = 1e-12;

// A resident VDI as the kernels see it.  Planes are slot-major: slot j of
// list li lives at index j * plane + li, so one wavefront reading slot j of
// 64 neighbouring lists touches contiguous memory.
struct DevVDI {
    int32_t WO, HO, NS;
    int32_t fmt;
    uint64_t plane;            // WO * HO
    const uint8_t *count;      // [HO][WO]
    const float2 *depth;       // [NS][HO][WO] (f, b)
    const void *rgba;          // [NS][HO][WO] float4 or 4 x 16-bit
    const uint32_t *grid;      // [gnz][GH][GW]
    int32_t gk, gnz, GW, GH;
    const float *gz;           // [gnz + 1] slice boundaries (device)
    float tx_o, ty_o;          // tan(fov/2) * aspect, tan(fov/2) of V_O
    double dcx, dcy;           // 2 / WO, 2 / HO: spacing of the list grid lines in NDC
    float inv_gk;              // 1 / gk rounded up: (int)(i * inv_gk) == i / gk for i < 2^15
};

// Per-render constants, computed on the host in double precision.
struct Frame {
    // V_O basis and projection scales: x_ndc = X / Z with X = sx * R.(P - eye_O)
    double FO[3], RO[3], UO[3];
    double sx_o, sy_o, near_o;
    // V_N eye expressed in V_O's frame (constant for all rays of a frame)
    double X0, Y0, Z0;
    // V_N camera
    double eyeN[3], FN[3], RN[3], UN[3];
    double tx_n, ty_n, near_n;
    double bmin[3], bmax[3];
    int32_t W, H;              // rays cast
    int32_t ess, search;
    double DR;                 // > 0: along-ray subsampling
    float4 *out;               // [H][W]
    // counters (instrumented kernel only)
    uint8_t *touched_lists, *touched_slots;
    int32_t *ray_stats;
};

}  // namespace vdi

// A resident VDI (the object behind vdi_t).
struct vdi_s {
    vdi::DevVDI dev;
    vdi_camera cam_o;
    float bmin[3], bmax[3];
    int device;
    uint8_t *d_count = nullptr;
    float2 *d_depth = nullptr;
    void *d_rgba = nullptr;
    uint32_t *d_grid = nullptr;
    float *d_gz = nullptr;
    uint64_t device_bytes = 0, supersegments = 0;
};

namespace vdi {

// Host helpers shared by the render and serving entry points (vdi_api.hip).
// Each returns VDI_OK or an error code after recording the reason.
int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);
int check_render_args(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, const float *out);
// Ray-grid size for downsampling factor D_I.
void lowres_size(int32_t W, int32_t H, float D_I, int32_t *w, int32_t *h);
// Frame constants for rays on a w x h grid of camera `cam` with aspect `aspect`.
int make_frame(const vdi_s *v, const vdi_camera &cam, int w, int h, double aspect, Frame &f);

// Launchers (vdi_kernels.hip).  All run on `stream` and return the launch status.
hipError_t launch_render_exact(const DevVDI &v, const Frame &f, bool counters, hipStream_t stream);
hipError_t launch_render_preview(const DevVDI &v, const Frame &f, hipStream_t stream);
hipError_t launch_upsample(const float4 *lo, int32_t w, int32_t h, float4 *out, int32_t W, int32_t H,
                           hipStream_t stream);
hipError_t launch_grid_build(const DevVDI &v, uint32_t *grid, hipStream_t stream);
hipError_t launch_convert_rgba(const float4 *src, void *dst, uint64_t n, int32_t fmt, hipStream_t stream);

}  // namespace vdi
