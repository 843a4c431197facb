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

// Launchers (vdi_kernels.hip).  All run on `stream` and return the launch status.
hipError_t launch_render_exact(const DevVDI &v, const Frame &f, bool counters, hipStream_t stream);
hipError_t launch_render_preview(const DevVDI &v, const Frame &f, hipStream_t stream);
hipError_t launch_upsample(const float4 *lo, int32_t w, int32_t h, float4 *out, int32_t W, int32_t H,
                           hipStream_t stream);
hipError_t launch_grid_build(const DevVDI &v, uint32_t *grid, hipStream_t stream);
hipError_t launch_convert_rgba(const float4 *src, void *dst, uint64_t n, int32_t fmt, hipStream_t stream);

}  // namespace vdi
