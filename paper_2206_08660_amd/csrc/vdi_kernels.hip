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

// One preview tile (preview_tile_dims): tw x th rays, F.parts adjacent lanes
// per ray.  Lanes outside the image take part in the combination with an
// empty result.
template <int FMT, bool COUNT = false>
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
    if (in && lane % parts == 0) F.out[(uint64_t)py * F.W + px] = to_rgba(a);
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
__global__ __launch_bounds__(kBlock) VDI_EXACT_OCC void k_render_batch(const BatchJob *__restrict__ jobs, int njobs)
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
        case VDI_F16: k_render_batch<VDI_F16, true><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        case VDI_BF16: k_render_batch<VDI_BF16, true><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        default: k_render_batch<VDI_F32, true><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        }
    } else {
        switch (fmt) {
        case VDI_F16: k_render_batch<VDI_F16, false><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        case VDI_BF16: k_render_batch<VDI_BF16, false><<<g, kBlock, 0, s>>>(jobs, njobs); break;
        default: k_render_batch<VDI_F32, false><<<g, kBlock, 0, s>>>(jobs, njobs); break;
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
