// Internal types shared by the libvdi host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "vdi.h"

namespace vdi {

// Transmittance at which a ray stops (early ray termination).
constexpr float kTTerm = 1e-5f;
// |F_O . d| below this: the ray keeps a constant V_O depth.
constexpr double kFlatZ = 1e-12;
// A workgroup renders a tile of kTileW x kTileH rays (one wavefront); MI355X
// has kXcds XCDs, which take the workgroups of a launch in turn.
#ifndef VDI_TILE_H
#define VDI_TILE_H 1
#endif
constexpr int kTileW = 64;
constexpr int kTileH = VDI_TILE_H;
// Exact renders use square tiles of kXTileW x kXTileH rays (one wavefront).
// Rays of vertically neighbouring pixels cross the same column of V_O lists
// in step, one list row apart and at nearly the same depth, where
// horizontal neighbours walk the same row of lists a list apart in time:
// an 8 x 8 tile keeps each column of 8 lanes in step (a 64 x 1 row tile:
// 17% slower on the 1080p sweep, 16 x 4: 4%, 4 x 16: 1%).
#ifndef VDI_EXACT_TW
#define VDI_EXACT_TW 8
#endif
constexpr int kXTileW = VDI_EXACT_TW;
constexpr int kXTileH = 64 / VDI_EXACT_TW;
constexpr int kXcds = 8;

// Preview rays are split over `parts` adjacent lanes when there are few of
// them: a preview frame lasts about as long as its longest ray's chain of
// dependent loads, and with fewer rays than about two wavefronts per SIMD
// nothing else hides it.  Each lane composites a contiguous block of the
// ray's grid cells; the partial results are combined in ray order.
#ifndef VDI_PREVIEW_LANES
#define VDI_PREVIEW_LANES 1000000  // lanes a preview launch should reach
#endif
__host__ __device__ inline int preview_parts(int w, int h)
{
    const long long rays = (long long)w * h;
    int p = 1;
    while (p < 8 && rays * p < VDI_PREVIEW_LANES) p <<= 1;
    return p;
}
// A preview wavefront renders a tile of 64 / parts rays, at most
// kPreviewTileH rows tall (the rays of a tile column cross neighbouring
// lists in step, as in exact tiles); the `parts` lanes of a ray are adjacent.
#ifndef VDI_PREVIEW_TH
#define VDI_PREVIEW_TH 8
#endif
__host__ __device__ inline void preview_tile_dims(int parts, int &tw, int &th)
{
    const int rays = kTileW * kTileH / parts;
    th = rays < VDI_PREVIEW_TH ? rays : VDI_PREVIEW_TH;
    tw = rays / th;
}
// Workgroups (one wavefront each) of a preview launch over a w x h ray grid.
__host__ __device__ inline uint32_t preview_tiles(int w, int h)
{
    int tw, th;
    preview_tile_dims(preview_parts(w, h), tw, th);
    return (uint32_t)(((w + tw - 1) / tw) * ((h + th - 1) / th));
}

// Storage order of the depth and colour planes on the device.  Lists are
// grouped in bricks of kBrickW x kBrickH neighbouring lists (2 x 2); a brick
// stores slot 0 of its lists, then slot 1, and so on.  Slot j of list
// (ix, iy) is element list_base_xy(ix, iy) + j * kBrick, and a 128-byte line
// holds four slots of depth pairs (two of colours) of a 2 x 2 block of
// lists: the supersegments a ray meets next whether it runs along its list or
// across neighbouring lists, and those the lanes of a tile column, which
// cross vertically neighbouring lists in step, read together.  kBrick = 0
// keeps whole slot planes (element j * WO * HO + li), the order of the input.
#ifndef VDI_BRICK
#define VDI_BRICK 4
#endif
constexpr int kBrick = VDI_BRICK;
static_assert(kBrick == 0 || (kBrick & (kBrick - 1)) == 0, "bricks must hold a power of two of lists");

#ifndef VDI_BRICK_W
#define VDI_BRICK_W 2
#endif
constexpr int kBrickW = kBrick == 0 ? 1 : VDI_BRICK_W;
constexpr int kBrickH = kBrick == 0 ? 1 : kBrick / kBrickW;

// Storage offset of slot 0 of list (ix, iy) of a WO-wide list grid.
__host__ __device__ inline uint64_t list_base_xy(int ix, int iy, int NS, int WO)
{
    if constexpr (kBrick == 0) return (uint64_t)iy * WO + ix;
    const uint32_t bw = (uint32_t)(WO + kBrickW - 1) / kBrickW;
    const uint64_t brick = (uint64_t)((uint32_t)iy / kBrickH) * bw + (uint32_t)ix / kBrickW;
    return brick * ((uint64_t)NS * kBrick) + ((uint32_t)iy % kBrickH) * kBrickW + (uint32_t)ix % kBrickW;
}
__host__ __device__ inline uint64_t list_base(uint64_t li, int NS, int WO)
{
    return list_base_xy((int)(li % (uint64_t)WO), (int)(li / (uint64_t)WO), NS, WO);
}
// Elements of one plane set (the list grid rounded up to whole bricks, times NS).
__host__ __device__ inline uint64_t plane_elems(int WO, int HO, int NS)
{
    if constexpr (kBrick == 0) return (uint64_t)WO * HO * (uint64_t)NS;
    return (uint64_t)((WO + kBrickW - 1) / kBrickW) * ((HO + kBrickH - 1) / kBrickH) * kBrick * (uint64_t)NS;
}

// A resident VDI as the kernels see it.
struct DevVDI {
    int32_t WO, HO, NS;
    int32_t fmt;
    uint64_t plane;            // WO * HO
    uint64_t sstride;          // element distance between slots j and j + 1 of a list
    const uint8_t *count;      // [HO][WO]
    const float2 *depth;       // (f, b), plane_elems(WO, HO, NS) in brick order
    const void *rgba;          // same order; float4 or 4 x 16-bit
    const uint32_t *grid;      // [gnz][GH][GW]
    const uint32_t *gbits;     // occupancy of the same cells, 32 per word: bit c % 32 of word c / 32 is (grid[c] != 0)
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
    int32_t parts;             // preview: lanes per ray (preview_parts)
    float4 *out;               // [H][W]
    // counters (instrumented kernels only)
    uint8_t *touched_lists, *touched_slots, *touched_cells;
    int32_t *ray_stats;
};

// One request of a batched launch (served form).  Blocks [tile0, tile0 +
// ntiles) of the launch render its tiles; tile0 is a multiple of the XCD
// count, so a block's XCD is the same as in a launch of its own.
struct BatchJob {
    DevVDI V;
    Frame F;                   // rays on F.W x F.H, writing F.out
    uint32_t tile0, ntiles;
};

// Bilinear upsampling of one request's low-resolution image in a batched launch.
struct UpsampleJob {
    const float4 *lo;          // [h][w]
    float4 *out;               // [H][W]
    int32_t w, h, W, H;
    uint32_t tile0, ntiles;    // blocks of 256 threads, 64 x 4 output pixels each
};

// Persistent served launch (vdi_server_create_persistent).  The launch's
// workgroups take tiles from per-XCD counters until the host stops them.
// The host publishes a job by writing its record, then the new job count,
// into coherent host memory (PHost); workgroup 0 of the launch copies new
// records into device memory and then publishes the count there (PQueue).
struct alignas(128) PCounter {
    unsigned long long v;
    unsigned long long pad[15];  // one 128-byte line per counter
};
struct PHost {
    PCounter tail;         // jobs written by the host
    PCounter stop;         // nonzero: the launch is to end
};
struct PQueue {
    PCounter next[kXcds];  // tiles taken by the workgroups of XCD x: its k-th is global tile k * kXcds + x
    PCounter tail;         // jobs whose records are in device memory
    PCounter stop;         // nonzero: leave once no published tile is left to take
    PCounter fault;        // nonzero: a workgroup gave up waiting (spin limit); the launch failed
    PCounter started;      // workgroups that have started
    PCounter exited;       // workgroups that have left
};
// Completion counters of one job in the persistent launch's table: word
// done_word(part, x) counts the finished tiles of XCD group x (x < kXcds) of
// part 0 (render) or 1 (upsampling), done_word(part, kXcds) the groups that
// have finished that part; every counter on a 128-byte line of its own.
constexpr int kDoneWords = 2 * (kXcds + 1) * 32;
__host__ __device__ inline int done_word(int part, int x) { return (part * (kXcds + 1) + x) * 32; }
// Tiles of XCD group x among n tiles from a multiple of kXcds.
__host__ __device__ inline uint32_t group_tiles(uint32_t n, uint32_t x) { return n / kXcds + (x < n % kXcds ? 1u : 0u); }

// One published request.  Global tiles [R.tile0, R.tile0 + R.ntiles) render
// it (on the low-res grid when D_I > 1), then, when U.ntiles > 0, tiles
// [U.tile0, U.tile0 + U.ntiles) upsample it (64 x 4 output pixels each).
struct alignas(256) PJob {
    BatchJob R;
    UpsampleJob U;
    uint32_t end;     // global tile after the job's last (the next job starts at or after it)
    uint32_t slot;    // position in the launch's job table: its counters and completion flag
    int32_t preview;  // D_R > 0
    int32_t pad;
};

}  // namespace vdi

namespace vdi {
// One set of device buffers of a resident VDI, with the metadata of the view
// it was generated from.
struct VdiSet {
    DevVDI dev{};
    vdi_camera cam_o{};
    float bmin[3]{}, bmax[3]{};
    uint8_t *d_count = nullptr;
    float2 *d_depth = nullptr;
    void *d_rgba = nullptr;
    uint32_t *d_grid = nullptr;
    uint32_t *d_gbits = nullptr;
    float *d_gz = nullptr;
    uint64_t supersegments = 0;
};
}  // namespace vdi

// A resident VDI (the object behind vdi_t).  Renders use `cur`; a
// replacement uploads into `back` on the copy stream and the two are swapped
// once the upload has finished (vdi_replace_begin / vdi_replace_poll).
struct vdi_s {
    vdi::VdiSet cur, back;
    int device = 0;
    uint64_t set_bytes = 0;          // device bytes of one set
    std::mutex mu;                   // guards cur, back and the replacement state
    hipStream_t copy = nullptr;      // the VDI's own stream: uploads (create, replacement) and its stream-ordered memory
    hipEvent_t start = nullptr;      // caller's stream reached vdi_replace_begin
    hipEvent_t ready = nullptr;      // the pending upload has finished
    void *stage = nullptr;           // staging buffer of replacement uploads
    uint64_t stage_bytes = 0;
    bool pending = false;            // a replacement was started and not yet swapped in
    bool enqueued = false;           // ... and all of its work is on the copy stream
    std::vector<float> gz_host;      // slice boundaries of the pending upload
    // Renders in flight, for vdi_destroy: an event recorded after the last
    // render of v on each of up to kUseSlots streams (created with v, so a
    // render allocates nothing), and the requests a server holds on v.
    static constexpr int kUseSlots = 8;
    hipEvent_t use_ev[kUseSlots] = {};
    hipStream_t use_st[kUseSlots] = {};
    uint64_t use_tick[kUseSlots] = {};
    uint64_t use_clock = 0;
    int use_n = 0;
    std::atomic<int> server_refs{0};
};

// Frame-time controller of a session (vdi_pace_*): its state is shared
// between the caller and a server's scheduler thread, hence the lock.
struct vdi_pace_s {
    double target, kp, ki, xmin, xmax, x, e_prev;
    bool first;
    std::mutex mu;
};

namespace vdi {

// Feed a frame time (ms) to a pace controller; returns the next D_I.
double pace_feed(vdi_pace_s *p, double frame_ms);
// The controller's current D_I.
double pace_d_i(vdi_pace_s *p);

// Count of changes to the device memory VDIs occupy (a VDI created or
// destroyed, a replacement swapped in).  A persistent served launch reads
// VDIs through caches that nothing invalidates while it runs, so it only
// takes requests while this count is what it was at its start.
extern std::atomic<uint64_t> g_mem_epoch;

// Host helpers shared by the render and serving entry points (vdi_api.hip).
// Each returns VDI_OK or an error code after recording the reason.
int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);
int check_render_args(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, const float *out);
// Record that v's buffers are read by work enqueued on `stream` (see vdi_s).
hipError_t note_use(vdi_s *v, hipStream_t stream);
// Ray-grid size for downsampling factor D_I.
void lowres_size(int32_t W, int32_t H, float D_I, int32_t *w, int32_t *h);
// The library's stream-ordered memory pool on `device` (freed blocks are kept
// for reuse until the process ends).
hipError_t library_pool(int device, hipMemPool_t *out);
// Frame constants for rays on a w x h grid of camera `cam` with aspect `aspect`.
int make_frame(const VdiSet &s, const vdi_camera &cam, int w, int h, double aspect, Frame &f);
// Copy of v's current set, taken under its lock.
VdiSet current(vdi_s *v);

// Launchers (vdi_kernels.hip).  All run on `stream` and return the launch status.
hipError_t launch_render_exact(const DevVDI &v, const Frame &f, bool counters, hipStream_t stream);
hipError_t launch_render_preview(const DevVDI &v, const Frame &f, bool counters, hipStream_t stream);
hipError_t launch_upsample(const float4 *lo, int32_t w, int32_t h, float4 *out, int32_t W, int32_t H,
                           hipStream_t stream);
hipError_t launch_grid_build(const DevVDI &v, uint32_t *grid, hipStream_t stream);
// Occupancy bits of the count grid (see DevVDI::gbits).
hipError_t launch_grid_bits(const DevVDI &v, uint32_t *bits, hipStream_t stream);
// n elements of slot-major input planes, starting at slot j0 (n a multiple of
// v.plane), into v's storage order; colour converted from fmt_in to fmt_store.
hipError_t launch_scatter_slots(const void *src, int32_t fmt_in, void *dst, int32_t fmt_store, bool depth, uint64_t n,
                                const DevVDI &v, int32_t j0, hipStream_t stream);
// Batched launches: `jobs` is a device array of njobs records sorted by
// tile0, all of colour format fmt; nblocks covers the last job's tiles.
// Exact jobs use the window search with empty-space skipping.
hipError_t launch_batch_render(const BatchJob *jobs, int32_t njobs, uint32_t nblocks, int32_t fmt, bool preview,
                               hipStream_t stream);
hipError_t launch_batch_upsample(const UpsampleJob *jobs, int32_t njobs, uint32_t nblocks, hipStream_t stream);
// Persistent served launch of `blocks` workgroups (see PHost, PQueue; jobs
// gets the records of host_jobs), for VDIs whose colour is stored in format
// fmt.  done + kDoneWords * slot holds a job's completion counters
// (done_word); host_done[slot] (host memory) is set once the job's output is
// in device memory.  A workgroup that waits longer than about spin_limit
// sleeps of ~27 us for a tile to be published, or for a job's render tiles
// before upsampling it, sets q->fault and leaves.
hipError_t launch_persist(int32_t fmt, const PHost *ctl, const PJob *host_jobs, PQueue *q, PJob *jobs, uint32_t *done,
                          uint32_t *host_done, uint32_t blocks, uint32_t spin_limit, hipStream_t stream);
// Workgroups of the persistent kernel that can be resident on the device at
// `waves` per SIMD (at most its occupancy), or 0 on error.
uint32_t persist_blocks(int device, int waves);

}  // namespace vdi
