/*
 * vdi.h -- C ABI of libvdi, a raycaster for Volumetric Depth Images (VDIs) on
 * AMD Instinct MI355X (gfx950).
 *
 * A VDI (Frey et al.; Gupta et al., "Efficient Raycasting of Volumetric Depth
 * Images for Remote Visualization of Large Volumes at High Frame Rates",
 * Section 2.3) stores, for every pixel i of the generating view V_O, a list L_i
 * of up to N_S supersegments S_ij, each with front and back depth f, b and
 * the colour and opacity accumulated between them.  This library keeps VDIs
 * resident in device memory and renders them from a new viewpoint V_N
 * (Section 4), either exactly or as the subsampled preview of Section 4.4.
 *
 * Conventions (all entry points):
 *   - World space is right-handed with y up.  Camera basis:
 *     F = normalize(target - eye), R = normalize(F x up), U = R x F; the field
 *     of view is vertical; aspect = image width / height.
 *   - NDC follows OpenGL: [-1, 1] on both axes; pixel (px, py) has its centre
 *     at (-1 + (2 px + 1)/w, -1 + (2 py + 1)/h); row 0 is the bottom row
 *     (y_ndc = -1).  Lists form a regular grid of 2/w x 2/h cells (Fig. 3).
 *   - Depths are linear view depth of V_O, z = F.(P - eye).  The paper
 *     compares NDC depths (supplement Alg. S2); NDC depth is monotone in z,
 *     so every comparison, and the result, is the same.
 *   - Every call returns VDI_OK (0) or a negative error code; the reason is
 *     available from vdi_last_error() on the calling thread.  No C++
 *     exception crosses this interface.
 */
#ifndef VDI_H
#define VDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define VDI_OK 0
#define VDI_ERR_ARG (-1)    /* invalid argument (null, size, range, non-finite, invalid VDI) */
#define VDI_ERR_OOM (-2)    /* device allocation failed */
#define VDI_ERR_HIP (-3)    /* a HIP runtime call failed */
#define VDI_ERR_BUDGET (-4) /* serving: request does not fit the memory budget or slots now */
#define VDI_ERR_STATE (-5)  /* call not valid in the object's current state */

/* Colour storage formats of supersegment RGBA. */
#define VDI_F32 0  /* 4 x float32, 16 bytes per supersegment */
#define VDI_F16 1  /* 4 x IEEE binary16 (round to nearest even), 8 bytes */
#define VDI_BF16 2 /* 4 x bfloat16 (round to nearest even), 8 bytes */

/* First-supersegment search (Section 4.2; all four give the same image). */
#define VDI_SEARCH_SEEDED 0 /* seeded by the index found in the previous list (supplement Alg. S2) */
#define VDI_SEARCH_BINARY 1 /* binary search over the whole list, from the middle */
#define VDI_SEARCH_LINEAR 2 /* linear scan from the list's near end */
#define VDI_SEARCH_WINDOW 3 /* seeded: 4 slots around the seed compared at once, then up to two
                               windows of 4 next to them, then the rest (default) */

#define VDI_MAX_SUPERSEGMENTS 255
#define VDI_MAX_GRID_NZ 64
#define VDI_MAX_GRID_K 16

typedef struct vdi_s *vdi_t;

/* Pinhole camera.  fov_y_deg in (0, 180); near_plane > 0. */
typedef struct {
    float eye[3];
    float target[3];
    float up[3];
    float fov_y_deg;
    float near_plane;
} vdi_camera;

/*
 * Description of a VDI in host or device memory (Section 2.3; Section 5 gives the
 * paper's texture layout, re-laid out here as slot-major planes).
 *   width, height       V_O viewport resolution = number of lists (N_L = w h).
 *   max_supersegments   N_S, 1..255.
 *   camera_VO           the generating view.
 *   aabb_min/max        volume bounding box; rays are clipped to it (Section 4.1).
 *   count   [height][width] uint8, supersegments in each list (<= N_S).
 *   depth   [N_S][height][width][2] float32, (f, b) of each slot, linear V_O depth.
 *   rgba    [N_S][height][width][4], straight (non-premultiplied) colour and the
 *           opacity accumulated over [f, b]; float32 when rgba_fmt_in == VDI_F32,
 *           16-bit values when VDI_F16 / VDI_BF16.
 *   rgba_fmt_store      format kept in device memory (conversion from float32
 *                       rounds to nearest even).
 *   grid_k, grid_nz     empty-space grid (Section 4.3): cells of grid_k x grid_k
 *                       lists by one depth slice; grid_k 1..16, grid_nz 1..64,
 *                       and fewer than 2^31 cells in all.
 *   grid_z  [grid_nz + 1] increasing float32 slice boundaries (linear V_O depth),
 *           or NULL to use grid_nz equal slices over the AABB corners' depth range.
 *   validate  non-zero: check every list (f < b, sorted, non-overlapping,
 *           count <= N_S, opacity in [0, 1], finite values) before upload.
 *   planes_on_device  0: count, depth and rgba are host arrays.  1: they are
 *           device arrays in the same layout (vdi_generate's output), copied
 *           device to device; only the count plane is read back to the host
 *           for the checks; validate must be 0.  grid_z stays a host array.
 * Slots at index >= count of their list are ignored.
 */
typedef struct {
    int32_t width, height, max_supersegments;
    vdi_camera camera_VO;
    float aabb_min[3], aabb_max[3];
    const uint8_t *count;
    const float *depth;
    const void *rgba;
    int32_t rgba_fmt_in, rgba_fmt_store;
    int32_t grid_k, grid_nz;
    const float *grid_z;
    int32_t validate;
    int32_t planes_on_device; /* 1: count, depth and rgba are DEVICE pointers (e.g. from vdi_generate) */
} vdi_desc;

/* Per-call options of vdi_render_ex.  Neither option changes the image. */
typedef struct {
    int32_t ess;    /* 1: empty-space skipping through the count grid (Section 4.3); 0: off */
    int32_t search; /* VDI_SEARCH_* */
} vdi_render_opts;

/* Sizes of a resident VDI. */
typedef struct {
    int32_t width, height, max_supersegments, rgba_fmt;
    int32_t grid_k, grid_nz, grid_w, grid_h;
    uint64_t device_bytes; /* count + depth + colour planes + grid and its occupancy bits (twice, plus staging, once a replacement was made) */
    uint64_t supersegments; /* sum of count */
} vdi_info_t;

/*
 * Upload a VDI and build its count grid (Section 4.3: per grid cell, the
 * number of supersegments of its lists whose [f, b] overlaps the cell's depth
 * slice with positive length).  Copies every array: the caller may free them
 * on return.  Synchronous for the calling thread: the upload runs on a stream
 * of its own, which is all it waits for, so work on the device's other
 * streams (a server's batches, renders of other VDIs) goes on meanwhile.
 * Device planes must be complete (their writers finished) when it is called.
 * Writes *out only on success.
 * Errors: VDI_ERR_ARG (null pointers, sizes, N_S or grid shape out of range,
 * non-finite camera or AABB, formats, and with validate != 0 an invalid list),
 * VDI_ERR_OOM, VDI_ERR_HIP.
 */
int vdi_create(const vdi_desc *desc, vdi_t *out);

/*
 * Render the VDI from camera cam_VN into out_rgba (Section 4; Eq. 2).
 *   width, height  output image; aspect = width/height.
 *   D_I >= 1       image downsampling factor: rays are cast on a
 *                  round(width/D_I) x round(height/D_I) grid with the same
 *                  camera and bilinearly upsampled (Section 4.4; the paper's
 *                  fraction D_I = 0.5 is factor 2 here).
 *   D_R            0: exact mode.  >= 1e-4: along-ray subsampling (Section 4.4):
 *                  in each non-empty grid cell a ray takes
 *                  ceil(((length in cell)/(slice depth)) (count/k^2) / D_R)
 *                  point samples at regular spacing (the paper's thinning
 *                  rate is 1/D_R).
 *   out_rgba       DEVICE pointer owned by the caller, >= width*height*16
 *                  bytes, receives premultiplied RGB and opacity (float32) over
 *                  transparent black, row-major, row 0 at the bottom.
 *   hip_stream     hipStream_t to run on (NULL: the null stream).
 * Asynchronous with respect to the host.  Reads but never writes the VDI, so
 * renders of one VDI on several streams may overlap.  The result is
 * deterministic: the same call gives the same bits.
 * Errors: VDI_ERR_ARG (null, width/height < 1 or > 16384, D_I < 1, D_R < 0,
 * 0 < D_R < 1e-4, non-finite values, fov out of range), VDI_ERR_OOM (preview
 * scratch), VDI_ERR_HIP.
 */
int vdi_render(vdi_t v, const vdi_camera *cam_VN, int32_t width, int32_t height, float D_I, float D_R,
               float *out_rgba, void *hip_stream);

/*
 * Render n frames in one call, frame i being what vdi_render(vdis[i],
 * &cams[i], widths[i], heights[i], D_I[i], D_R[i], outs[i], hip_stream)
 * would write, bit for bit (Section 4; Eq. 2; Section 4.4).  The frames are
 * independent: instead of one launch per frame, the tiles of all exact
 * frames of one colour format form one launch, those of all preview frames
 * another, and the upsampling of all downsampled frames a third, so the long
 * rays at the end of one frame run beside the next frame's tiles.  Frames may
 * name different VDIs, all resident on the device of hip_stream.
 *   n              1 .. VDI_BATCH_MAX_FRAMES.
 *   vdis, cams, widths, heights, D_I, D_R, outs
 *                  host arrays of n entries; outs[i] are DEVICE pointers
 *                  owned by the caller, laid out as for vdi_render, and must
 *                  not overlap each other.
 *   hip_stream     hipStream_t to run on (NULL: the null stream).
 * Asynchronous with respect to the host.  The job tables travel to the
 * device through pinned host memory of the library (a ring of 4 slots of
 * VDI_BATCH_MAX_FRAMES jobs per device, allocated at the first call): a call
 * waits only if the slot it takes is still being copied for a call 4 calls
 * earlier.  Device job tables and low-res images are stream-ordered
 * allocations of the library's pool, freed on hip_stream after the launches.
 * Errors: VDI_ERR_ARG (null arrays, n out of range, any frame's arguments as
 * for vdi_render, VDIs on different devices; nothing has been launched, and
 * the message names the first bad frame), VDI_ERR_OOM, VDI_ERR_HIP (some of
 * the frames may have been launched).
 */
#define VDI_BATCH_MAX_FRAMES 1024
int vdi_render_batch(int32_t n, const vdi_t *vdis, const vdi_camera *cams, const int32_t *widths,
                     const int32_t *heights, const float *D_I, const float *D_R, float *const *outs, void *hip_stream);

/*
 * vdi_render for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and image as vdi_render (bit for bit), but it calls no
 * hipMalloc, hipFree or pool allocation: the low-res image of a downsampled
 * render (D_I > 1) is kept in a static device array of the library,
 * VDI_NOALLOC_SCRATCH_TEXELS float4 texels (32 MiB), one copy per device,
 * held until the process ends.  The caller still owns out_rgba.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (other streams or threads, without ordering between them) race
 * on it and give undefined images; calls on one stream are ordered and safe.
 * The first call on a device looks the array's device address up
 * (hipGetSymbolAddress).
 * Errors: those of vdi_render, and VDI_ERR_ARG when the low-res image,
 * round(width/D_I) x round(height/D_I), exceeds VDI_NOALLOC_SCRATCH_TEXELS
 * (1920 x 1080 at any D_I > 1 fits).
 */
#define VDI_NOALLOC_SCRATCH_TEXELS (1u << 21)
int vdi_render_noalloc(vdi_t v, const vdi_camera *cam_VN, int32_t width, int32_t height, float D_I, float D_R,
                       float *out_rgba, void *hip_stream);

/* vdi_render with explicit options (opts NULL = defaults: ESS on, window search). */
int vdi_render_ex(vdi_t v, const vdi_camera *cam_VN, int32_t width, int32_t height, float D_I, float D_R,
                  const vdi_render_opts *opts, float *out_rgba, void *hip_stream);

/*
 * Instrumented exact render (same image as vdi_render with D_I = 1, D_R = 0)
 * that also records what the rays touched, to measure the algorithmic bytes
 * of a frame: touched_lists [H_O][W_O] uint8 and touched_slots [N_S][H_O][W_O]
 * uint8 (device pointers, zeroed by the caller) receive 1 for each list a ray
 * entered before terminating and each supersegment it composited;
 * ray_stats [height][width][2] int32 (device, may be NULL) receive per ray
 * (lists entered, supersegment pieces composited).  Slower than vdi_render.
 */
int vdi_render_counters(vdi_t v, const vdi_camera *cam_VN, int32_t width, int32_t height,
                        const vdi_render_opts *opts, float *out_rgba, uint8_t *touched_lists,
                        uint8_t *touched_slots, int32_t *ray_stats, void *hip_stream);

/*
 * Instrumented preview (Section 4.4 along-ray sampling) of the low-res ray
 * grid of a width x height, D_I, D_R render (D_R > 0): renders the
 * round(width/D_I) x round(height/D_I) image, with the display's aspect, into
 * lowres_out (device, float32 RGBA, that many pixels; the texels vdi_render
 * upsamples) and records what the samples read, to measure the algorithmic
 * bytes of a preview frame: touched_lists [H_O][W_O] uint8 (the list of every
 * sample), touched_slots [N_S][H_O][W_O] uint8 (every supersegment
 * composited) and touched_cells [grid_nz][grid_h][grid_w] uint8 (every grid
 * cell whose count was read); device pointers zeroed by the caller.
 * ray_stats [h][w][2] int32 (device, zeroed, may be NULL) receive per ray
 * (samples taken, supersegments composited).  Slower than vdi_render.
 * Errors: those of vdi_render, VDI_ERR_ARG for D_R = 0 or a null buffer.
 */
int vdi_preview_counters(vdi_t v, const vdi_camera *cam_VN, int32_t width, int32_t height, float D_I, float D_R,
                         float *lowres_out, uint8_t *touched_lists, uint8_t *touched_slots, uint8_t *touched_cells,
                         int32_t *ray_stats, void *hip_stream);

/* Copy the count grid, uint32 [grid_nz][grid_h][grid_w], to host memory. */
int vdi_get_grid(vdi_t v, uint32_t *host_out, size_t capacity_elems);

/* Sizes of a resident VDI. */
int vdi_get_info(vdi_t v, vdi_info_t *info);

/*
 * Wait for the work that reads the VDI, then free its device memory: the
 * last render of v on each stream that rendered it (tracked for up to eight
 * streams at a time; a ninth stream waits for the least recently used one
 * when it renders), a replacement upload in progress, and requests on v that
 * a server still holds (VDI_ERR_STATE, nothing freed, if they are not done
 * within 60 s).  No device-wide synchronization is requested; the runtime's
 * release of the device memory itself (hipFree) may still wait for the
 * device.  NULL is a no-op.  Destroying the same handle twice, or while
 * another thread renders it, is undefined.
 */
int vdi_destroy(vdi_t v);

/* ------------------------------------------------------------------------
 * Replacing a resident VDI while rendering (double buffering, the client
 * half of the paper's remote session, Section 5: a new VDI arrives from the
 * server while the client keeps rendering the old one).
 * ------------------------------------------------------------------------ */

/*
 * Start uploading `desc` into the back buffers of v: a VDI with the same
 * width, height, max_supersegments, stored colour format and grid shape,
 * possibly generated from another view (camera_VO, AABB and grid_z may
 * differ).  The upload runs on a stream of v's own, after the work already
 * enqueued on `stream` (the caller's render stream for v; NULL = default
 * stream), and the back buffers are allocated by the first call.  Renders of
 * v keep using the current VDI until vdi_replace_poll swaps the new one in.
 * Returns when the host arrays have been read: the caller may free them.
 * With device planes the call first waits for `stream` (the planes may be
 * written there, e.g. by vdi_generate) and the caller keeps them alive until
 * vdi_replace_poll reports the swap.
 * Renders of v on other streams and requests of a server that use v must be
 * complete before the call (their work may still read the back buffers, which
 * held the VDI before the last swap).
 * Errors: VDI_ERR_ARG (null arguments, an invalid descriptor as for
 * vdi_create, or another shape), VDI_ERR_STATE (a replacement is pending),
 * VDI_ERR_OOM, VDI_ERR_HIP.
 */
int vdi_replace_begin(vdi_t v, const vdi_desc *desc, void *stream);

/*
 * If the pending replacement's upload has finished, make the new VDI the one
 * later renders and queries use, and set *swapped = 1; otherwise (still
 * uploading, or nothing pending) set *swapped = 0.  Never waits.
 */
int vdi_replace_poll(vdi_t v, int32_t *swapped);

/* ------------------------------------------------------------------------
 * Frame-time control of preview rendering (Section 4.4; the application of
 * Section 5 holds a user-chosen frame rate with a PI controller on the image
 * downsampling D_I while the user keeps D_R).  Host-side only.
 *
 * The time of a downsampled frame is close to proportional to its number of
 * rays, (W/D_I)(H/D_I), so the controller acts on x = ln D_I with the error
 * e = ln(frame_ms / target_ms), in velocity form:
 *     x <- x + kp (e - e_prev) + ki e,   clamped to [ln D_I_min, ln D_I_max]
 * (the clamp also keeps the integral action from winding up).  With the
 * model plant ln(frame) = c - 2x, kp = 0.1 and ki = 0.3 place the error's
 * poles at 0.56 and -0.36.
 * ------------------------------------------------------------------------ */
typedef struct vdi_pace_s *vdi_pace_t;

/* target_ms > 0; kp, ki >= 0, finite; 1 <= D_I_min <= D_I_start <= D_I_max.
 * Errors: VDI_ERR_ARG, VDI_ERR_OOM. */
int vdi_pace_create(float target_ms, float kp, float ki, float D_I_min, float D_I_max, float D_I_start,
                    vdi_pace_t *out);

/* Feed the time of the frame just rendered (> 0, finite) and get the D_I for
 * the next one. */
int vdi_pace_update(vdi_pace_t p, float frame_ms, float *next_D_I);

/* NULL is a no-op. */
int vdi_pace_destroy(vdi_pace_t p);

/* Image size used for downsampling factor D_I (round half up, at least 1). */
int vdi_lowres_size(int32_t width, int32_t height, float D_I, int32_t *w, int32_t *h);

/* Device bytes of the count, depth and colour planes for a w x h x n_s VDI. */
uint64_t vdi_plane_bytes(int32_t width, int32_t height, int32_t n_s, int32_t rgba_fmt);

/* Reason for the last error on this thread ("" if none). */
const char *vdi_last_error(void);

/* ------------------------------------------------------------------------
 * VDI generation (Section 3: the server raycasts the volume from V_O and
 * splits each ray into supersegments with the homogeneity criterion of Eq. 1;
 * supplement Alg. S1: per ray, a bisection on the sensitivity gamma so that
 * the ray yields at most N_S supersegments and not many fewer).
 * ------------------------------------------------------------------------ */
#define VDI_VOXEL_F32 0 /* float32 voxels */
#define VDI_VOXEL_U16 1 /* uint16 voxels, value / 65535 */

#define VDI_TF_RAMP 0   /* colour (v, 0.25 + 0.5 v, 1 - v), opacity 0.2 clamp((v - 0.05)/0.95, 0, 1) */
#define VDI_TF_KNOTS4 1 /* piecewise linear through 4 knots at v = 0, 0.25, 0.55, 1:
                           colours (0.1,0.2,0.8) (0.1,0.7,0.9) (0.95,0.9,0.3) (0.9,0.15,0.1),
                           opacities 0, 0, 0.04, 0.12 (v clamped to [0, 1]) */

/* A scalar volume in DEVICE memory, [nz][ny][nx] with x fastest, spanning the
 * AABB with cell-centred voxels (voxel (i,j,k) sits at the centre of the
 * (i,j,k)-th of nx x ny x nz equal cells). 1 <= nx, ny, nz <= 16384. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t voxel_fmt; /* VDI_VOXEL_* */
    const void *data;
    double aabb_min[3], aabb_max[3];
} vdi_volume;

typedef struct {
    vdi_camera camera_VO;       /* the generating view; one ray per pixel centre */
    int32_t width, height;      /* V_O viewport = number of lists, 1..32768 each */
    int32_t max_supersegments;  /* N_S, 1..255 */
    int32_t tf;                 /* VDI_TF_* */
    double gamma;               /* > 0: fixed sensitivity; 0: per-ray bisection (Alg. S1) */
} vdi_gen_params;

/*
 * Generate a VDI on the device.  Per ray (all arithmetic FP64, no fused
 * multiply-adds; the per-call constants below are computed on the host):
 *   - clip to the AABB and to V_O's near plane (view depth >= near) -> [t0, t1];
 *   - N = ceil((t1 - t0)/ds - 1e-9) equal samples, clamped to
 *     [1, 2 max(nx,ny,nz) + 8], ds = longest AABB side / max(nx,ny,nz); each
 *     sample at its midpoint, trilinear with clamp to edge, transfer function
 *     tf, opacity a' = 1 - (1 - a)^(len/ds) for the sample length len;
 *   - front-to-back emission-absorption until the transmittance is <= 1e-5
 *     (early ray termination): the samples taken are the ones split;
 *   - gamma = params->gamma, or Alg. S1: start at 1e-5 in [0, sqrt 3],
 *     accept the first trial if it gives fewer than N_S supersegments,
 *     otherwise bisect until the count is in [N_S - floor(0.15 N_S), N_S]
 *     (or the interval is under 1e-6 wide, or after 25 trials: take its upper
 *     end, or its lower end if that gives none);
 *   - split with Eq. 1: a non-transparent sample joins the open supersegment
 *     unless the distance between the supersegment's premultiplied colour,
 *     with its opacity rescaled to one sample's length, and the sample's is
 *     >= gamma; a transparent sample closes it; once N_S - 1 are closed the
 *     last one takes every remaining non-transparent sample.
 * Outputs (DEVICE pointers, caller-owned, the vdi_desc host layout, so that
 * they can be copied to host arrays for vdi_create): count [height][width]
 * uint8; depth [N_S][height][width][2] float32 (f, b) as linear V_O depth
 * (b raised to the next float above f if they round equal); rgba
 * [N_S][height][width][4] float32 straight colour and accumulated opacity;
 * slots at index >= count are zero.  gamma_out [height][width] float64 (may be
 * NULL): the gamma each ray used (0 for rays that miss the volume).
 * Asynchronous on `stream` (NULL: the null stream).  Uses up to 4 GiB of
 * device scratch (each resident wavefront's cache of its rays' samples) from
 * the library's stream-ordered pool, which keeps freed blocks for reuse until
 * the process ends.
 * Errors: VDI_ERR_ARG (null pointers, sizes or formats out of range,
 * non-finite or degenerate camera, empty AABB, gamma < 0), VDI_ERR_OOM
 * (scratch), VDI_ERR_HIP.
 */
int vdi_generate(const vdi_volume *volume, const vdi_gen_params *params, uint8_t *count, float *depth, float *rgba,
                 double *gamma_out, void *stream);

/* ------------------------------------------------------------------------
 * Direct volume rendering and image quality (Section 6: VDI renderings are
 * compared with DVR of the volume from the same viewpoint by SSIM and PSNR,
 * and their frame rates with DVR's).
 * ------------------------------------------------------------------------ */
#define VDI_DVR_F64 0 /* every step in FP64, the generator's arithmetic (the quality reference) */
#define VDI_DVR_F32 1 /* FP64 ray set-up and sample positions; FP32 interpolation, transfer
                         function, opacity and compositing (the frame-rate baseline) */

typedef struct {
    vdi_camera camera;     /* the view rendered (V_N) */
    int32_t width, height; /* 1..16384 each */
    int32_t tf;            /* VDI_TF_* */
    int32_t precision;     /* VDI_DVR_* */
} vdi_dvr_params;

/*
 * Raycast the volume into out_rgba (DEVICE, caller-owned, width*height*16
 * bytes, the vdi_render layout: premultiplied RGB and opacity over
 * transparent black, row 0 at the bottom).  One ray per pixel centre, with
 * the clipping, samples, transfer function, opacity correction and early
 * termination (transmittance <= 1e-5) of vdi_generate's DVR pass, composited
 * front to back.  Asynchronous on `stream`.
 * Errors: VDI_ERR_ARG (as vdi_generate, and an unknown precision), VDI_ERR_HIP.
 */
int vdi_dvr(const vdi_volume *volume, const vdi_dvr_params *params, float *out_rgba, void *stream);

/*
 * SSIM and PSNR of `image` against `reference` (DEVICE RGBA float32 images of
 * width x height, the vdi_render layout; RGB compared, opacity ignored, data
 * range 1).  SSIM as Wang et al. (2004): 11 x 11 Gaussian window with
 * sigma 1.5, K1 = 0.01, K2 = 0.03, population moments, averaged over the
 * pixels whose window lies inside the image and over R, G and B.  PSNR =
 * 10 log10(1 / MSE) over all pixels and channels (+inf for equal images).
 * Sums run in FP64 in a fixed order (deterministic).  Allocates stream-ordered
 * scratch; waits for `stream` and returns the values in host memory.
 * Errors: VDI_ERR_ARG (null, images under 11 x 11 or over 16384), VDI_ERR_HIP.
 */
int vdi_image_quality(const float *image, const float *reference, int32_t width, int32_t height, double *ssim,
                      double *psnr, void *stream);

/* ------------------------------------------------------------------------
 * Serving (continuous batching; not part of the paper's method, whose client
 * renders one request at a time, Section 5).  A server renders requests for any
 * number of resident VDIs.  Requests are admitted while request slots and the
 * device-memory budget allow, and queued.  Everything queued is launched as
 * one batch as soon as one of the server's streams is free: by the
 * submitting thread within vdi_server_submit if a stream is free then,
 * otherwise by a scheduler thread owned by the server.  One kernel launch
 * per (mode, colour format) group covers
 * the tiles of all the group's requests, whatever their resolution,
 * viewpoint and preview level, and one more upsamples those with D_I > 1.
 * With two or more streams the next batches start while earlier ones
 * drain.  A request is done when its batch is.  A request's image is
 * identical to vdi_render's with the same arguments.
 * ------------------------------------------------------------------------ */
typedef struct vdi_server_s *vdi_server_t;

typedef struct {
    uint64_t submitted, completed, rejected_budget, rejected_slots;
    uint64_t bytes_in_flight, peak_bytes_in_flight;
    uint64_t batches;       /* batches launched so far */
    int32_t inflight, peak_inflight;  /* admitted and not yet done */
    int32_t queued;         /* admitted, waiting for a free stream */
    int32_t peak_batch;     /* most requests in one batch */
    uint64_t paced_completed;  /* requests of paced sessions done */
    uint64_t deadlines_met;    /* ... of them within their session's target frame time */
} vdi_server_stats;

/*
 * Create a server on the current device.
 *   hbm_budget_bytes  admission budget for the memory of requests in flight
 *                     (output images plus preview scratch), > 0.
 *   max_inflight      request slots, 1..4096.
 *   streams           batches in flight at once, each on a stream of the
 *                     server's own (0: three; at most 8).
 * Returns VDI_ERR_ARG for arguments out of range and VDI_ERR_HIP / VDI_ERR_OOM
 * when a stream, event, job table or the scheduler thread cannot be created.
 */
int vdi_server_create(uint64_t hbm_budget_bytes, int32_t max_inflight, int32_t streams, vdi_server_t *out);

/*
 * Create a server whose requests are rendered by one persistent kernel
 * instead of batched launches (same submit, poll, drain, stats and destroy
 * calls, same admission, same images).  The kernel stays resident while
 * requests come: every workgroup (one wavefront) takes the next render or
 * upsampling tile of the requests published to it, from a device-memory
 * queue that the server fills by two copies per request (the job record,
 * then the job count) on a stream of its own; a request is done when the
 * kernel has set its flag in host memory, after its results were written
 * through to device memory.  A launch serves one colour format and up to
 * 8192 requests, and takes requests only while no VDI has been created,
 * destroyed or replaced since it started (it reads VDIs through caches that
 * nothing invalidates while it runs).  The server ends a launch once the
 * requests published to it are done and the next request cannot be
 * published to it, or after 20 ms without requests, and starts a new one
 * for the next request.  While a launch is resident it holds
 * waves_per_simd wavefronts on every SIMD (0: as many as fit, 5), which
 * other kernels on the device then do not get, and work on a stream that
 * the runtime maps to the launch's hardware queue (a process has four by
 * default) waits until the launch ends: at the latest 20 ms after the
 * server runs out of requests.  A workgroup that waits
 * about 1.8 s for work flags the launch as failed (the server then reports
 * VDI_ERR_HIP).
 *   hbm_budget_bytes, max_inflight  as in vdi_server_create.
 *   waves_per_simd    0..16 (values above what fits take what fits).
 * Returns VDI_ERR_ARG for arguments out of range and VDI_ERR_HIP / VDI_ERR_OOM
 * when a stream, event, queue or the scheduler thread cannot be created.
 */
int vdi_server_create_persistent(uint64_t hbm_budget_bytes, int32_t max_inflight, int32_t waves_per_simd,
                                 vdi_server_t *out);

/*
 * Submit a render request (same arguments as vdi_render).  Returns VDI_OK with
 * *ticket set, or VDI_ERR_BUDGET when the request does not fit the budget or
 * the free slots right now (nothing is queued; submit again later).  `out` is
 * a device pointer the caller keeps alive until the request is done.  The
 * server's streams do not wait for other streams: the VDI and `out` must be
 * ready (their writers finished) when the request is submitted.  If one of
 * the server's streams is free, the call launches the queued requests itself
 * (on the server's device, restoring the caller's current device after).
 */
int vdi_server_submit(vdi_server_t s, vdi_t v, const vdi_camera *cam_VN, int32_t width, int32_t height, float D_I,
                      float D_R, float *out, uint64_t *ticket);

/*
 * Submit a request of a paced session (the frame-time control of Section
 * 4.4, which the paper's remote client runs with a PI controller on D_I,
 * Section 6): the request is rendered at the session's current D_I (written
 * to *D_I_used; D_R and the other arguments as in vdi_server_submit), and
 * when it is done the server feeds its latency, from submission to
 * completion in ms, to the session's controller, so that the session's next
 * request gets the next D_I.  The session's target frame time is the
 * request's deadline (counted in deadlines_met).  The session must outlive
 * its requests, and must not be updated by its owner while the server holds
 * one of them.  Errors: those of vdi_server_submit, VDI_ERR_ARG for a null
 * session or D_I_used.
 */
int vdi_server_submit_paced(vdi_server_t s, vdi_t v, const vdi_camera *cam_VN, int32_t width, int32_t height,
                            vdi_pace_t session, float D_R, float *out_rgba, uint64_t *ticket, float *D_I_used);

/* *done = 1 once the request's image is complete and visible to later work.
 * A call that finds the request's batch finished retires that batch itself,
 * without waiting for the scheduler thread.
 * A failed batch (a HIP error) makes this and every later call return VDI_ERR_HIP. */
int vdi_server_poll(vdi_server_t s, uint64_t ticket, int *done);

/* Block until all admitted requests are done (VDI_ERR_STATE after 60 s). */
int vdi_server_drain(vdi_server_t s);

int vdi_server_get_stats(vdi_server_t s, vdi_server_stats *stats);

/* Zero the counters (submitted, completed, rejections, batches) and restart
 * the peaks from the current in-flight state; requests in flight are kept. */
int vdi_server_reset_stats(vdi_server_t s);

/* Drain, stop the scheduler, free everything.  NULL is a no-op. */
int vdi_server_destroy(vdi_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* VDI_H */
