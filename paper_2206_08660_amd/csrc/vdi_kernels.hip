// One-shot HIP kernels of libvdi for gfx950 (MI355X): raycasting a VDI from
// a new viewpoint (Gupta et al., Section 4), its preview mode (Section 4.4),
// bilinear upsampling, the count grid (Section 4.3) and colour storage
// conversion.  The per-ray code they run is in vdi_trace.h.
//
// Execution model.  One lane per ray; a workgroup is one wavefront, so a CU
// slot is freed as soon as its 64 rays are done (with four wavefronts per
// workgroup the finished ones wait for the slowest: 6% slower).  An exact
// wavefront covers an 8 x 8 tile of pixels (kXTileW x kXTileH): their
// projected lines in V_O are near-parallel, and the 8 lanes of a tile column
// cross vertically neighbouring lists in step, at nearly the same depth,
// while the columns follow each other along the same lists a step apart.
// The planes are stored in bricks of 2 x 2 neighbouring lists (see
// list_base_xy), so one 128-byte line holds several slots of the lists a
// tile column reads together, and lists revisited by neighbouring rays are
// served from L1/L2 (the paper's spatial smoothness).  Preview wavefronts
// cover 64 x 1 tiles of the low-res grid, split by lanes per ray.  Tiles are
// dealt to the 8 XCDs in interleaved bands of rows (xcd_tile), so
// neighbouring tiles share an L2 and every XCD gets part of the image
// centre.
//
// Precision.  Ray set-up, list crossings and supersegment overlaps run in
// FP64 (the crossing depth of a ray with a list edge is ill-conditioned near
// the generating view: an FP32 error of 1e-7 in NDC moves it by ~1e-5 in
// depth); opacity correction (Eq. 2) and compositing run in FP32.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "vdi_trace.h"

namespace vdi {
namespace {

// The exact kernel is bound by the latency of its dependent loads (count ->
// depth pair -> colour per list crossed): it is compiled for at least 6
// wavefronts per SIMD (at most 80 VGPRs), which it reaches without spilling.
#ifndef VDI_EXACT_WAVES
#define VDI_EXACT_WAVES 6
#endif
#define VDI_EXACT_OCC __attribute__((amdgpu_waves_per_eu(VDI_EXACT_WAVES)))

template <int FMT, int SEARCH, bool ESS, bool COUNT>
__global__ __launch_bounds__(kBlock) VDI_EXACT_OCC void k_render_exact(DevVDI V, Frame F)
{
    __shared__ float s_gz[VDI_MAX_GRID_NZ + 1];
    if constexpr (ESS) {
        for (int i = threadIdx.x; i <= V.gnz; i += kBlock) s_gz[i] = V.gz[i];
        __syncthreads();
    }
    const int tiles_x = (F.W + kXTileW - 1) / kXTileW, tiles_y = (F.H + kXTileH - 1) / kXTileH;
    const int tile = xcd_tile(blockIdx.x, tiles_x, tiles_y, kXBandRows);
    const int px = (tile % tiles_x) * kXTileW + (threadIdx.x % kXTileW);
    const int py = (tile / tiles_x) * kXTileH + (threadIdx.x / kXTileW);
    if (px >= F.W || py >= F.H) return;
    Counters cnt = {0, 0};
    F.out[(uint64_t)py * F.W + px] = trace_exact<FMT, SEARCH, ESS, COUNT>(V, F, s_gz, px, py, cnt);
    if constexpr (COUNT) {
        if (F.ray_stats) {
            F.ray_stats[2 * ((uint64_t)py * F.W + px)] = cnt.lists;
            F.ray_stats[2 * ((uint64_t)py * F.W + px) + 1] = cnt.pieces;
        }
    }
}

// Store of an output pixel: plain, or (WT) written through to device memory
// as two relaxed system-scope atomic stores of 8 bytes, for the persistent
// kernel, whose results are read by other workgroups and by the host with no
// kernel boundary in between (no dirty line is left in an XCD's L2).
template <bool WT>
__device__ __forceinline__ void store_px(float4 *p, float4 v)
{
    if constexpr (WT) {
        auto *u = reinterpret_cast<unsigned long long *>(p);
        const unsigned long long lo = (unsigned long long)__float_as_uint(v.y) << 32 | __float_as_uint(v.x);
        const unsigned long long hi = (unsigned long long)__float_as_uint(v.w) << 32 | __float_as_uint(v.z);
        __hip_atomic_store(u, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(u + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
        *p = v;
    }
}

// One preview tile (preview_tile_dims): tw x th rays, F.parts adjacent lanes
// per ray.  Lanes outside the image take part in the combination with an
// empty result.
template <int FMT, bool COUNT = false, bool WT = false>
__device__ __forceinline__ void preview_tile(const DevVDI &V, const Frame &F, const float *s_gz, int tile_index)
{
    const int parts = F.parts;
    int tw, th;
    preview_tile_dims(parts, tw, th);
    const int tiles_x = (F.W + tw - 1) / tw, tiles_y = (F.H + th - 1) / th;
    const int tile = xcd_tile(tile_index, tiles_x, tiles_y, VDI_BAND_ROWS / th > 0 ? VDI_BAND_ROWS / th : 1);
    const int lane = threadIdx.x, ray = lane / parts;
    const int px = (tile % tiles_x) * tw + ray % tw;
    const int py = (tile / tiles_x) * th + ray / tw;
    const bool in = px < F.W && py < F.H;
    Accum a = {0.0f, 0.0f, 0.0f, 1.0f};
    Counters cnt = {0, 0};
    if (in) a = trace_preview<FMT, COUNT>(V, F, s_gz, px, py, lane % parts, parts, &cnt);
    a = combine_parts(a, parts, lane);
    if (in && lane % parts == 0) store_px<WT>(&F.out[(uint64_t)py * F.W + px], to_rgba(a));
    if constexpr (COUNT) {
        if (in && F.ray_stats) {
            atomicAdd(&F.ray_stats[2 * ((uint64_t)py * F.W + px)], cnt.lists);
            atomicAdd(&F.ray_stats[2 * ((uint64_t)py * F.W + px) + 1], cnt.pieces);
        }
    }
}

template <int FMT, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_render_preview(DevVDI V, Frame F)
{
    __shared__ float s_gz[VDI_MAX_GRID_NZ + 1];
    for (int i = threadIdx.x; i <= V.gnz; i += kBlock) s_gz[i] = V.gz[i];
    __syncthreads();
    preview_tile<FMT, COUNT>(V, F, s_gz, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Batched launches (served form).  Block b belongs to the last job whose
// tile0 <= b; the job table is read-only for the launch, so its uniform
// loads go through the scalar cache like kernel arguments.  Inside a job the
// block renders exactly what k_render_exact / k_render_preview would.
// ---------------------------------------------------------------------------
template <typename J>
__device__ __forceinline__ const J &job_of(const J *__restrict__ jobs, int njobs, uint32_t b)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return jobs[lo];
}

template <int FMT, bool PREVIEW>
__device__ __forceinline__ void batch_tile(const BatchJob *__restrict__ jobs, int njobs)
{
    __shared__ float s_gz[VDI_MAX_GRID_NZ + 1];
    const BatchJob &J = job_of(jobs, njobs, blockIdx.x);
    const uint32_t local = blockIdx.x - J.tile0;
    if (local >= J.ntiles) return;  // padding block: the whole workgroup leaves
    for (int i = threadIdx.x; i <= J.V.gnz; i += kBlock) s_gz[i] = J.V.gz[i];
    __syncthreads();
    if constexpr (PREVIEW) {
        preview_tile<FMT>(J.V, J.F, s_gz, (int)local);
    } else {
        const int tiles_x = (J.F.W + kXTileW - 1) / kXTileW, tiles_y = (J.F.H + kXTileH - 1) / kXTileH;
        const int tile = xcd_tile((int)local, tiles_x, tiles_y, kXBandRows);
        const int px = (tile % tiles_x) * kXTileW + (threadIdx.x % kXTileW);
        const int py = (tile / tiles_x) * kXTileH + (threadIdx.x / kXTileW);
        if (px >= J.F.W || py >= J.F.H) return;
        Counters cnt = {0, 0};
        J.F.out[(uint64_t)py * J.F.W + px] = trace_exact<FMT, VDI_SEARCH_WINDOW, true, false>(J.V, J.F, s_gz, px, py, cnt);
    }
}

// Exact tiles at the exact kernel's occupancy (6 wavefronts per SIMD);
// preview tiles at the preview kernel's (its registers, 5 wavefronts): held
// to 80 VGPRs the preview loop spilled, and the benchmark step took
// 9.95-10.09 ms against 9.74-9.83 ms.
template <int FMT>
__global__ __launch_bounds__(kBlock) VDI_EXACT_OCC void k_render_batch(const BatchJob *__restrict__ jobs, int njobs)
{
    batch_tile<FMT, false>(jobs, njobs);
}
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_render_batch_preview(const BatchJob *__restrict__ jobs, int njobs)
{
    batch_tile<FMT, true>(jobs, njobs);
}

__global__ __launch_bounds__(256) void k_upsample_batch(const UpsampleJob *__restrict__ jobs, int njobs)
{
    const UpsampleJob &J = job_of(jobs, njobs, blockIdx.x);
    const uint32_t local = blockIdx.x - J.tile0;
    if (local >= J.ntiles) return;
    const int tiles_x = (J.W + 63) / 64;
    const int x = (int)(local % (uint32_t)tiles_x) * 64 + (int)(threadIdx.x & 63);
    const int y = (int)(local / (uint32_t)tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= J.W || y >= J.H) return;
    J.out[(uint64_t)y * J.W + x] = upsample_px(J.lo, J.w, J.h, J.W, J.H, x, y);
}

// ---------------------------------------------------------------------------
// Persistent served launch (served form; see PQueue).  Every workgroup (one
// wavefront) loops: it takes the next tile of its XCD group (global tiles
// x, x + 8, x + 16, ... for blockIdx.x % 8 == x, so a tile lands on the XCD
// it would get in a launch of its own), finds the published job that holds
// it, waiting while the tile lies beyond the published jobs, and renders or
// upsamples it exactly as k_render_batch / k_upsample_batch would.
// Workgroup 0 takes no tiles: it publishes the jobs the host writes.
//
// Coherence without kernel boundaries, and without L2 write-back or
// invalidation per tile.  The host writes a job's record, then the job
// count, to coherent host memory; workgroup 0 copies new records into
// device memory with stores written through to memory and only then
// publishes their count there (persist_mirror).  Every word another agent
// or workgroup writes during the launch (counts, stop word, records, tile
// counters) is read with system-scope atomic loads, which no cache answers
// with an old copy.  A job record is read with plain (scalar) loads, but
// only once its count is published, that is once it is in memory, and no
// cache holds its lines before: records are 256-byte aligned, written once
// per launch, and the launch starts with invalidated caches.  (Two copies on
// one stream, record then count, were not seen in that order by all XCDs
// while the launch filled the device: hence the mirror.)  The
// VDIs are not written while a launch reads them: the host ends the launch
// before a VDI is created, destroyed or replaced.  Results are written
// through to memory (store_px<true>); after its stores have completed
// (s_waitcnt) lane 0 counts the tile in the job's counter, and the
// workgroup that finishes a job's last tile sets its flag in host memory.
// Upsampling tiles wait until every XCD group has finished the job's render
// tiles, then read the low-res texels through the caches: the server gives
// each request of a launch a low-res image in memory that no cache has held
// during the launch.  A job's tiles are counted per XCD group, each counter
// on a line of its own, so that its tiles do not all update one word.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long load_host_word(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Count a finished tile of XCD group x in part `part` of a job with n tiles
// in that part (counters D, see done_word); true for the tile that finishes
// the part, whose last group counts itself in the part's group count.
__device__ __forceinline__ bool tile_done(uint32_t *D, int part, uint32_t x, uint32_t n)
{
    const uint32_t c = __hip_atomic_fetch_add(&D[done_word(part, (int)x)], 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_SYSTEM) + 1u;
    if (c != group_tiles(n, x)) return false;
    const uint32_t groups = n < (uint32_t)kXcds ? n : (uint32_t)kXcds;
    return __hip_atomic_fetch_add(&D[done_word(part, kXcds)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) + 1u ==
           groups;
}

// Sleep of a waiting wavefront: short at first, then about 27 us, so that
// thousands of idle wavefronts polling a word in memory do not load the
// memory system the working ones use.
__device__ __forceinline__ void nap(uint32_t spins)
{
    if (spins < 64) {
        __builtin_amdgcn_s_sleep(2);
    } else {
        for (int i = 0; i < 8; ++i) __builtin_amdgcn_s_sleep(127);
    }
}

// Workgroup 0 of a persistent launch: copies the records the host has
// written into device memory (written through), then publishes their count
// to the other workgroups; passes the host's stop on.
__device__ __forceinline__ void persist_mirror(const PHost *ctl, const PJob *host_jobs, PQueue *q, PJob *jobs,
                                               uint32_t spin_limit)
{
    const int lane = (int)threadIdx.x;
    uint32_t have = 0;
    for (uint32_t spins = 0;; ++spins) {
        const uint32_t t = (uint32_t)load_host_word(const_cast<unsigned long long *>(&ctl->tail.v));
        if (t > have) {
            for (uint32_t j = have; j < t; ++j) {
                auto *src = reinterpret_cast<unsigned long long *>(const_cast<PJob *>(host_jobs + j));
                auto *dst = reinterpret_cast<unsigned long long *>(jobs + j);
                for (int i = lane; i < (int)(sizeof(PJob) / 8); i += kBlock)
                    __hip_atomic_store(dst + i, __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            __builtin_amdgcn_s_waitcnt(0);  // the records are in device memory
            __syncthreads();
            if (lane == 0) __hip_atomic_store(&q->tail.v, (unsigned long long)t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            have = t;
            spins = 0;
            continue;
        }
        const bool stop = load_host_word(const_cast<unsigned long long *>(&ctl->stop.v)) != 0;
        if (stop || spins >= spin_limit) {
            if (lane == 0) {
                if (!stop) __hip_atomic_store(&q->fault.v, 3ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&q->stop.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_fetch_add(&q->exited.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            return;
        }
        nap(spins);
    }
}

// Compiled for 5 wavefronts per SIMD (96 VGPRs): with both walkers in one
// loop it spilled 18-48 VGPRs per lane at 6.
#define VDI_PERSIST_OCC __attribute__((amdgpu_waves_per_eu(5)))

// `mirror_jobs` and `jobs` are the same table: workgroup 0 writes it through
// the first, the others only read it through the second (scalar loads of a
// record that no cache holds before it is published).
template <int FMT>
__global__ __launch_bounds__(kBlock) VDI_PERSIST_OCC void k_persist(const PHost *ctl, const PJob *host_jobs, PQueue *q,
                                                                  PJob *mirror_jobs, const PJob *__restrict__ jobs,
                                                                  uint32_t *done, uint32_t *host_done,
                                                                  uint32_t spin_limit)
{
    __shared__ float s_gz[VDI_MAX_GRID_NZ + 1];
    const int lane = (int)threadIdx.x;
    if (blockIdx.x == 0) {
        if (lane == 0) __hip_atomic_fetch_add(&q->started.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        persist_mirror(ctl, host_jobs, q, mirror_jobs, spin_limit);
        return;
    }
    const uint32_t x = blockIdx.x % kXcds;
    uint32_t j = 0;            // the jobs before j end at or before every tile this workgroup has still to take
    uint32_t tail = 0;         // jobs known to be published
    if (lane == 0) __hip_atomic_fetch_add(&q->started.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (;;) {
        unsigned long long k = 0;
        if (lane == 0) k = __hip_atomic_fetch_add(&q->next[x].v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint32_t khi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)__shfl((int)(uint32_t)(k >> 32), 0));
        const uint32_t klo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)__shfl((int)(uint32_t)k, 0));
        const unsigned long long g = (((unsigned long long)khi << 32) | klo) * kXcds + x;
        // The published job holding tile g; wait while there is none (the
        // job count is read only when g lies beyond the jobs known).
        for (uint32_t spins = 0;; ++spins) {
            while (j < tail && g >= jobs[j].end) ++j;
            if (j < tail) break;
            tail = (uint32_t)load_host_word(&q->tail.v);
            while (j < tail && g >= jobs[j].end) ++j;
            if (j < tail) break;
            if (load_host_word(&q->stop.v) || spins >= spin_limit) {
                if (lane == 0) {
                    if (spins >= spin_limit)
                        __hip_atomic_store(&q->fault.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_fetch_add(&q->exited.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                return;
            }
            nap(spins);
        }
        const PJob &J = jobs[j];
        const uint32_t slot = J.slot;
        if (g < J.R.tile0) continue;  // alignment gap before the job
        if (g < (unsigned long long)J.R.tile0 + J.R.ntiles) {
            const uint32_t local = (uint32_t)(g - J.R.tile0);
            for (int i = lane; i <= J.R.V.gnz; i += kBlock) s_gz[i] = J.R.V.gz[i];
            __syncthreads();
            if (J.preview) {
                preview_tile<FMT, false, true>(J.R.V, J.R.F, s_gz, (int)local);
            } else {
                const int tiles_x = (J.R.F.W + kXTileW - 1) / kXTileW, tiles_y = (J.R.F.H + kXTileH - 1) / kXTileH;
                const int tile = xcd_tile((int)local, tiles_x, tiles_y, kXBandRows);
                const int px = (tile % tiles_x) * kXTileW + (lane % kXTileW);
                const int py = (tile / tiles_x) * kXTileH + (lane / kXTileW);
                if (px < J.R.F.W && py < J.R.F.H) {
                    Counters cnt = {0, 0};
                    store_px<true>(&J.R.F.out[(uint64_t)py * J.R.F.W + px],
                                   trace_exact<FMT, VDI_SEARCH_WINDOW, true, false>(J.R.V, J.R.F, s_gz, px, py, cnt));
                }
            }
            __builtin_amdgcn_s_waitcnt(0);  // this wavefront's stores have completed
            __syncthreads();                // and s_gz is free for the next tile
            if (lane == 0 && tile_done(done + (size_t)kDoneWords * slot, 0, x, J.R.ntiles) && J.U.ntiles == 0)
                __hip_atomic_store(&host_done[slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            continue;
        }
        if (g < J.U.tile0) continue;  // alignment gap before the upsampling tiles
        // Upsampling tile: once every render tile of the job is done.
        const uint32_t groups = J.R.ntiles < (uint32_t)kXcds ? J.R.ntiles : (uint32_t)kXcds;
        for (uint32_t spins = 0;; ++spins) {
            if (__hip_atomic_load(&done[(size_t)kDoneWords * slot + done_word(0, kXcds)], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_SYSTEM) >= groups)
                break;
            if (spins >= spin_limit) {
                if (lane == 0) {
                    __hip_atomic_store(&q->fault.v, 2ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_fetch_add(&q->exited.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                return;
            }
            nap(spins);
        }
        const uint32_t local = (uint32_t)(g - J.U.tile0);
        const UpsampleJob &U = J.U;
        const int tiles_x = (U.W + 63) / 64;
        const int px = (int)(local % (uint32_t)tiles_x) * 64 + lane;
        for (int r = 0; r < 4; ++r) {
            const int py = (int)(local / (uint32_t)tiles_x) * 4 + r;
            // The low-res image lies in memory no cache has held in this launch.
            if (px < U.W && py < U.H)
                store_px<true>(&U.out[(uint64_t)py * U.W + px], upsample_px(U.lo, U.w, U.h, U.W, U.H, px, py));
        }
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0 && tile_done(done + (size_t)kDoneWords * slot, 1, x, U.ntiles))
            __hip_atomic_store(&host_done[slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ---------------------------------------------------------------------------
// Bilinear upsampling, half-pixel centres, clamped (Section 4.4, Fig. 7)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_upsample(const float4 *__restrict__ lo, int w, int h,
                                                  float4 *__restrict__ out, int W, int H)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    out[(uint64_t)y * W + x] = upsample_px(lo, w, h, W, H, x, y);
}

// ---------------------------------------------------------------------------
// Count grid (Section 4.3).  One workgroup per k x k column of lists; each
// lane walks one list and counts, in LDS, the depth slices its supersegments
// overlap with positive length.  No global atomics; deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grid_build(DevVDI V, uint32_t *__restrict__ grid)
{
    __shared__ uint32_t s_cnt[VDI_MAX_GRID_NZ];
    __shared__ float s_gz[VDI_MAX_GRID_NZ + 1];
    const int k = V.gk;
    const int cx = blockIdx.x % V.GW, cy = blockIdx.x / V.GW;
    for (int i = threadIdx.x; i < V.gnz; i += blockDim.x) s_cnt[i] = 0u;
    for (int i = threadIdx.x; i <= V.gnz; i += blockDim.x) s_gz[i] = V.gz[i];
    __syncthreads();
    const int lx = cx * k + (int)threadIdx.x % k, ly = cy * k + (int)threadIdx.x / k;
    if ((int)threadIdx.x < k * k && lx < V.WO && ly < V.HO) {
        const uint64_t li = (uint64_t)ly * V.WO + lx, lb = list_base_xy(lx, ly, V.NS, V.WO);
        const int n = V.count[li];
        for (int j = 0; j < n; ++j) {
            const float2 fb = V.depth[(uint64_t)j * V.sstride + lb];
            for (int c = 0; c < V.gnz; ++c)
                if (fb.x < s_gz[c + 1] && fb.y > s_gz[c]) atomicAdd(&s_cnt[c], 1u);
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < V.gnz; c += blockDim.x)
        grid[((uint64_t)c * V.GH + cy) * V.GW + cx] = s_cnt[c];
}

// Occupancy bits of the count grid, one 32-cell word per lane.  The exact
// walker only asks whether a cell is empty: the bits (81 KB for the 1080p
// VDI's 648,000 cells) are 32 times denser than the 2.6 MB of counts, so a
// cache line answers for 1024 cells instead of 32.
__global__ __launch_bounds__(256) void k_grid_bits(const uint32_t *__restrict__ grid, uint32_t *__restrict__ bits,
                                                   uint32_t ncells)
{
    const uint32_t w = blockIdx.x * 256u + threadIdx.x;
    if (w >= (ncells + 31u) / 32u) return;
    uint32_t b = 0u;
    for (uint32_t i = 0; i < 32u; ++i) {
        const uint32_t c = w * 32u + i;
        if (c < ncells && grid[c] != 0u) b |= 1u << i;
    }
    bits[w] = b;
}

// ---------------------------------------------------------------------------
// Upload: slots [j0, j0 + n / plane) of slot-major input planes are scattered
// into the device's brick order, converting colour float32 -> binary16 /
// bfloat16 (round to nearest even) where asked.
// ---------------------------------------------------------------------------
__device__ inline uint2 to16(float4 v, int fmt)
{
    uint2 o;
    if (fmt == VDI_F16) {
        const __half2 rg = __floats2half2_rn(v.x, v.y), ba = __floats2half2_rn(v.z, v.w);
        o.x = *reinterpret_cast<const uint32_t *>(&rg);
        o.y = *reinterpret_cast<const uint32_t *>(&ba);
    } else {
        const __hip_bfloat16 r = __float2bfloat16(v.x), g = __float2bfloat16(v.y);
        const __hip_bfloat16 b = __float2bfloat16(v.z), a = __float2bfloat16(v.w);
        o.x = (uint32_t)(*reinterpret_cast<const uint16_t *>(&r)) | ((uint32_t)(*reinterpret_cast<const uint16_t *>(&g)) << 16);
        o.y = (uint32_t)(*reinterpret_cast<const uint16_t *>(&b)) | ((uint32_t)(*reinterpret_cast<const uint16_t *>(&a)) << 16);
    }
    return o;
}

// S -> D element by element; CONV: store S as is, or a float4 as 16-bit format CONV.
template <typename S, typename D, int CONV>
__global__ __launch_bounds__(256) void k_scatter(const S *__restrict__ src, D *__restrict__ dst, uint64_t n,
                                                 uint64_t plane, int NS, int j0, uint64_t sstride, int WO)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = j0 + i / plane, li = i % plane;
        const uint64_t o = list_base(li, NS, WO) + j * sstride;
        if constexpr (CONV == 0) dst[o] = src[i];
        else dst[o] = to16(src[i], CONV);
    }
}

template <int FMT, bool COUNT>
hipError_t launch_exact_fmt(const DevVDI &v, const Frame &f, dim3 grid, hipStream_t s)
{
    const bool ess = f.ess != 0;
    switch (f.search) {
    case VDI_SEARCH_BINARY:
        if (ess) k_render_exact<FMT, VDI_SEARCH_BINARY, true, COUNT><<<grid, kBlock, 0, s>>>(v, f);
        else k_render_exact<FMT, VDI_SEARCH_BINARY, false, COUNT><<<grid, kBlock, 0, s>>>(v, f);
        break;
    case VDI_SEARCH_LINEAR:
        if (ess) k_render_exact<FMT, VDI_SEARCH_LINEAR, true, COUNT><<<grid, kBlock, 0, s>>>(v, f);
        else k_render_exact<FMT, VDI_SEARCH_LINEAR, false, COUNT><<<grid, kBlock, 0, s>>>(v, f);
        break;
    case VDI_SEARCH_WINDOW:
        if (ess) k_render_exact<FMT, VDI_SEARCH_WINDOW, true, COUNT><<<grid, kBlock, 0, s>>>(v, f);
        else k_render_exact<FMT, VDI_SEARCH_WINDOW, false, COUNT><<<grid, kBlock, 0, s>>>(v, f);
        break;
    default:
        if (ess) k_render_exact<FMT, VDI_SEARCH_SEEDED, true, COUNT><<<grid, kBlock, 0, s>>>(v, f);
        else k_render_exact<FMT, VDI_SEARCH_SEEDED, false, COUNT><<<grid, kBlock, 0, s>>>(v, f);
    }
    return hipGetLastError();
}

inline dim3 tile_grid(int W, int H)
{
    return dim3((unsigned)(((W + kXTileW - 1) / kXTileW) * ((H + kXTileH - 1) / kXTileH)));
}

}  // namespace

hipError_t launch_render_exact(const DevVDI &v, const Frame &f, bool counters, hipStream_t s)
{
    const dim3 g = tile_grid(f.W, f.H);
    if (counters) {
        switch (v.fmt) {
        case VDI_F16: return launch_exact_fmt<VDI_F16, true>(v, f, g, s);
        case VDI_BF16: return launch_exact_fmt<VDI_BF16, true>(v, f, g, s);
        default: return launch_exact_fmt<VDI_F32, true>(v, f, g, s);
        }
    }
    switch (v.fmt) {
    case VDI_F16: return launch_exact_fmt<VDI_F16, false>(v, f, g, s);
    case VDI_BF16: return launch_exact_fmt<VDI_BF16, false>(v, f, g, s);
    default: return launch_exact_fmt<VDI_F32, false>(v, f, g, s);
    }
}

hipError_t launch_render_preview(const DevVDI &v, const Frame &f, bool counters, hipStream_t s)
{
    if (f.parts != preview_parts(f.W, f.H)) return hipErrorInvalidValue;
    const dim3 g(preview_tiles(f.W, f.H));
    if (counters) {
        switch (v.fmt) {
        case VDI_F16: k_render_preview<VDI_F16, true><<<g, kBlock, 0, s>>>(v, f); break;
        case VDI_BF16: k_render_preview<VDI_BF16, true><<<g, kBlock, 0, s>>>(v, f); break;
        default: k_render_preview<VDI_F32, true><<<g, kBlock, 0, s>>>(v, f); break;
        }
        return hipGetLastError();
    }
    switch (v.fmt) {
    case VDI_F16: k_render_preview<VDI_F16, false><<<g, kBlock, 0, s>>>(v, f); break;
    case VDI_BF16: k_render_preview<VDI_BF16, false><<<g, kBlock, 0, s>>>(v, f); break;
    default: k_render_preview<VDI_F32, false><<<g, kBlock, 0, s>>>(v, f); break;
    }
    return hipGetLastError();
}

hipError_t launch_upsample(const float4 *lo, int32_t w, int32_t h, float4 *out, int32_t W, int32_t H, hipStream_t s)
{
    const dim3 g((unsigned)((W + 63) / 64), (unsigned)((H + 3) / 4));
    k_upsample<<<g, 256, 0, s>>>(lo, w, h, out, W, H);
    return hipGetLastError();
}

hipError_t launch_batch_render(const BatchJob *jobs, int32_t njobs, uint32_t nblocks, int32_t fmt, bool preview,
                               hipStream_t s)
{
    const dim3 g(nblocks);
    if (preview) {
        switch (fmt) {
        case VDI_F16: k_render_batch_preview<VDI_F16><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        case VDI_BF16: k_render_batch_preview<VDI_BF16><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        default: k_render_batch_preview<VDI_F32><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        }
    } else {
        switch (fmt) {
        case VDI_F16: k_render_batch<VDI_F16><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        case VDI_BF16: k_render_batch<VDI_BF16><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        default: k_render_batch<VDI_F32><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_batch_upsample(const UpsampleJob *jobs, int32_t njobs, uint32_t nblocks, hipStream_t s)
{
    k_upsample_batch<<<dim3(nblocks), 256, 0, s>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_grid_build(const DevVDI &v, uint32_t *grid, hipStream_t s)
{
    const int threads = ((v.gk * v.gk + 63) / 64) * 64;
    k_grid_build<<<dim3((unsigned)(v.GW * v.GH)), threads, 0, s>>>(v, grid);
    return hipGetLastError();
}

hipError_t launch_grid_bits(const DevVDI &v, uint32_t *bits, hipStream_t s)
{
    const uint32_t ncells = (uint32_t)v.gnz * (uint32_t)v.GH * (uint32_t)v.GW;
    const uint32_t words = (ncells + 31u) / 32u;
    k_grid_bits<<<dim3((words + 255u) / 256u), 256, 0, s>>>(v.grid, bits, ncells);
    return hipGetLastError();
}

hipError_t launch_persist(int32_t fmt, const PHost *ctl, const PJob *host_jobs, PQueue *q, PJob *jobs, uint32_t *done,
                          uint32_t *host_done, uint32_t blocks, uint32_t spin_limit, hipStream_t s)
{
    if (fmt == VDI_F32)
        k_persist<VDI_F32><<<dim3(blocks), kBlock, 0, s>>>(ctl, host_jobs, q, jobs, jobs, done, host_done, spin_limit);
    else if (fmt == VDI_F16)
        k_persist<VDI_F16><<<dim3(blocks), kBlock, 0, s>>>(ctl, host_jobs, q, jobs, jobs, done, host_done, spin_limit);
    else
        k_persist<VDI_BF16><<<dim3(blocks), kBlock, 0, s>>>(ctl, host_jobs, q, jobs, jobs, done, host_done, spin_limit);
    return hipGetLastError();
}

uint32_t persist_blocks(int device, int waves)
{
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<VDI_F32>, kBlock, 0) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    const int simd_waves = per_cu / 4;  // four SIMDs per CU, one wavefront per workgroup
    const int w = waves > 0 && waves < simd_waves ? waves : simd_waves;
    return (uint32_t)(w * 4 * cus);
}

hipError_t launch_scatter_slots(const void *src, int32_t fmt_in, void *dst, int32_t fmt_store, bool depth, uint64_t n,
                                const DevVDI &v, int32_t j0, hipStream_t s)
{
    const uint64_t blocks = (n + 255) / 256;
    const dim3 g((unsigned)(blocks < 65536 ? blocks : 65536));
    const uint64_t plane = v.plane, st = v.sstride;
    const int NS = v.NS;
    if (depth)
        k_scatter<float2, float2, 0><<<g, 256, 0, s>>>(static_cast<const float2 *>(src), static_cast<float2 *>(dst), n,
                                                       plane, NS, j0, st, v.WO);
    else if (fmt_store == VDI_F32)
        k_scatter<float4, float4, 0><<<g, 256, 0, s>>>(static_cast<const float4 *>(src), static_cast<float4 *>(dst), n,
                                                       plane, NS, j0, st, v.WO);
    else if (fmt_in != VDI_F32)
        k_scatter<uint2, uint2, 0><<<g, 256, 0, s>>>(static_cast<const uint2 *>(src), static_cast<uint2 *>(dst), n,
                                                     plane, NS, j0, st, v.WO);
    else if (fmt_store == VDI_F16)
        k_scatter<float4, uint2, VDI_F16><<<g, 256, 0, s>>>(static_cast<const float4 *>(src), static_cast<uint2 *>(dst),
                                                            n, plane, NS, j0, st, v.WO);
    else
        k_scatter<float4, uint2, VDI_BF16><<<g, 256, 0, s>>>(static_cast<const float4 *>(src), static_cast<uint2 *>(dst),
                                                             n, plane, NS, j0, st, v.WO);
    return hipGetLastError();
}

}  // namespace vdi
