// Served form of libvdi: continuous batching of render requests in one
// persistent kernel (build addition; the paper's client renders one request
// at a time, Section 5).
//
// Work is a stream of 64 x 4 pixel tiles numbered 0, 1, 2, ...  A request's
// tiles occupy a contiguous range: first the tiles of its ray grid (exact or
// along-ray preview), then, for D_I > 1, the tiles of its bilinear upsampling.
// The host publishes a request by writing its descriptor and a job record
// into host-coherent memory and then advancing `published_tiles`.  Every
// workgroup of the kernel repeatedly takes the next tile number from a device
// atomic, waits until it is published, finds its request, renders the tile,
// and counts it; the workgroup finishing a request's last tile writes the
// request's ticket to its completion word.  Requests that arrive while others
// run are therefore spread over the same running kernel as soon as they are
// published.  An upsampling tile waits until its request's ray tiles are all
// done; those have smaller numbers, so they were taken by running workgroups
// that never wait themselves, and the wait ends.
//
// Every wait is bounded: on shutdown, or after kIdleSeconds without work, the
// workgroups exit.  A request's image is bit-identical to vdi_render's: the
// same per-ray functions and the same frame constants are used.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "vdi_trace.h"

namespace vdi {
namespace {

constexpr int kServeBlock = 256;  // 4 wavefronts: one 64 x 4 tile
constexpr int kJobRing = 16384;   // job records kept in the ring
constexpr int kMaxSlots = 4096;
constexpr double kIdleSeconds = 20.0;
constexpr uint64_t kClockHz = 100000000ull;  // s_memrealtime ticks per second

// One request as the kernel sees it.
struct Job {
    DevVDI V;
    Frame F;              // phase 1: rays on a w x h grid writing F.out
    float4 *out;          // final image, W x H
    int32_t W, H, w, h;
    int32_t preview;      // phase 1 is the along-ray preview
    int32_t tiles_x1;     // tiles per row of phase 1
    int32_t ntiles1, ntiles2;
    uint64_t ticket;
};

struct JobRec {
    uint64_t base;        // first tile number
    uint64_t jobno;       // sequence number of the record
    uint64_t ticket;
    uint32_t ntiles;
    uint32_t slot;
};

// Control block in host-coherent memory.
struct Ctl {
    uint64_t published_tiles;
    uint64_t published_jobs;
    uint32_t shutdown;
    uint32_t error;       // set by the kernel when a wait times out
    uint64_t pad[6];
    JobRec rec[kJobRing];
    uint64_t done[kMaxSlots];  // ticket of the last request completed in each slot
};

// Device-only counters.
struct DevCtr {
    uint64_t cursor;
    uint32_t tiles_done[kMaxSlots];
    uint32_t phase1_done[kMaxSlots];
};

__device__ __forceinline__ uint64_t ld_sys(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_sys32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

template <int FMT>
__device__ void render_tile(const Job &J, const float *s_gz, uint32_t local)
{
    const int tx = (int)(local % (uint32_t)J.tiles_x1), ty = (int)(local / (uint32_t)J.tiles_x1);
    const int px = tx * kTileW + (int)(threadIdx.x % kTileW);
    const int py = ty * kTileH + (int)(threadIdx.x / kTileW);
    if (px >= J.w || py >= J.h) return;
    float4 o;
    if (J.preview) {
        o = trace_preview<FMT>(J.V, J.F, s_gz, px, py);
    } else {
        Counters cnt = {0, 0};
        o = trace_exact<FMT, VDI_SEARCH_SEEDED, true, false>(J.V, J.F, s_gz, px, py, cnt);
    }
    J.F.out[(uint64_t)py * J.w + px] = o;
}

__global__ __launch_bounds__(kServeBlock) void k_serve(Ctl *ctl, const Job *desc, DevCtr *dc)
{
    __shared__ Job s_job;
    __shared__ float s_gz[VDI_MAX_GRID_NZ + 1];
    __shared__ uint64_t s_g, s_base, s_ticket;
    __shared__ uint32_t s_slot, s_ntiles;
    __shared__ int s_cmd;
    uint64_t k = 0;          // thread 0: index of the job record last used
    uint64_t have_ticket = 0;
    uint32_t have_slot = 0xffffffffu;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint64_t g = atomicAdd((unsigned long long *)&dc->cursor, 1ull);
            int cmd = 0;
            const uint64_t t0 = now_ticks();
            for (;;) {
                if (g < ld_sys(&ctl->published_tiles)) break;
                if (ld_sys32(&ctl->shutdown)) {
                    cmd = 1;
                    break;
                }
                if (now_ticks() - t0 > (uint64_t)(kIdleSeconds * kClockHz)) {
                    __hip_atomic_store(&ctl->error, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                    cmd = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(20);
            }
            if (cmd == 0) {
                // Find the job holding tile g: records are published in tile
                // order, so scan forward from the last one used.
                const uint64_t nj = ld_sys(&ctl->published_jobs);
                if (k + kJobRing <= nj) k = nj - kJobRing + 1;
                for (; k < nj; ++k) {
                    const JobRec *r = &ctl->rec[k % kJobRing];
                    const uint64_t jn = __hip_atomic_load(&r->jobno, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    const uint64_t base = __hip_atomic_load(&r->base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    const uint32_t nt = __hip_atomic_load(&r->ntiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    // A record overwritten by a newer job belongs to a finished job: skip it.
                    if (jn == k && g >= base && g < base + nt) {
                        s_base = base;
                        s_ntiles = nt;
                        s_slot = __hip_atomic_load(&r->slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        s_ticket = __hip_atomic_load(&r->ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        break;
                    }
                }
                if (k >= nj) cmd = 1;  // cannot happen: a published tile always has a record
            }
            s_g = g;
            s_cmd = cmd;
        }
        __syncthreads();
        if (s_cmd) break;
        const uint32_t slot = s_slot;
        if (slot != have_slot || s_ticket != have_ticket) {
            // Copy the request's descriptor from host-coherent memory.
            const uint32_t *src = reinterpret_cast<const uint32_t *>(desc + slot);
            uint32_t *dst = reinterpret_cast<uint32_t *>(&s_job);
            for (int i = threadIdx.x; i < (int)(sizeof(Job) / 4); i += kServeBlock)
                dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __syncthreads();
            for (int i = threadIdx.x; i <= s_job.V.gnz; i += kServeBlock) s_gz[i] = s_job.V.gz[i];
            __syncthreads();
            have_slot = slot;
            have_ticket = s_ticket;
        }
        const uint32_t local = (uint32_t)(s_g - s_base);
        const bool phase1 = local < (uint32_t)s_job.ntiles1;
        if (phase1) {
            render_tile<kFmtRuntime>(s_job, s_gz, local);
        } else {
            if (threadIdx.x == 0) {
                const uint64_t t0 = now_ticks();
                while (__hip_atomic_load(&dc->phase1_done[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
                       (uint32_t)s_job.ntiles1) {
                    if (now_ticks() - t0 > (uint64_t)(kIdleSeconds * kClockHz)) {
                        __hip_atomic_store(&ctl->error, 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
            }
            __syncthreads();
            const uint32_t u = local - (uint32_t)s_job.ntiles1;
            const int tiles_x = (s_job.W + kTileW - 1) / kTileW;
            const int x = (int)(u % (uint32_t)tiles_x) * kTileW + (int)(threadIdx.x % kTileW);
            const int y = (int)(u / (uint32_t)tiles_x) * kTileH + (int)(threadIdx.x / kTileW);
            if (x < s_job.W && y < s_job.H)
                s_job.out[(uint64_t)y * s_job.W + x] = upsample_px(s_job.F.out, s_job.w, s_job.h, s_job.W, s_job.H, x, y);
        }
        // Each wavefront's stores must reach device scope before thread 0
        // counts the tile: the barrier alone does not wait for other
        // wavefronts' stores, and readers of this tile may sit on another XCD.
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            if (phase1)
                __hip_atomic_fetch_add(&dc->phase1_done[slot], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t d =
                __hip_atomic_fetch_add(&dc->tiles_done[slot], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
            if (d == s_ntiles) {
                // Last tile: reset the slot's counters, then publish completion.
                __hip_atomic_store(&dc->tiles_done[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&dc->phase1_done[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __threadfence_system();
                __hip_atomic_store(&ctl->done[slot], s_ticket, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

int tiles_of(int w, int h) { return ((w + kTileW - 1) / kTileW) * ((h + kTileH - 1) / kTileH); }

}  // namespace
}  // namespace vdi

using vdi::Job;
using vdi::JobRec;

struct vdi_server_s {
    int device = 0;
    hipStream_t stream = nullptr;
    vdi::Ctl *ctl = nullptr;
    Job *desc = nullptr;
    vdi::DevCtr *dc = nullptr;
    uint64_t budget = 0;
    int max_inflight = 0, workers = 0;
    bool running = false;
    uint64_t next_ticket = 1;
    struct Slot {
        bool busy = false;
        uint64_t ticket = 0, bytes = 0, lowres_bytes = 0;
        float4 *lowres = nullptr;
    };
    std::vector<Slot> slots;
    int next_slot = 0;
    std::map<uint64_t, int> pending;                  // ticket -> slot
    std::multimap<uint64_t, float4 *> free_lowres;    // bytes -> buffer
    vdi_server_stats st{};
    std::mutex mu;
};

namespace {

// Release a finished request's slot (caller holds the lock).
void finish(vdi_server_s *s, std::map<uint64_t, int>::iterator it)
{
    vdi_server_s::Slot &sl = s->slots[it->second];
    if (sl.lowres) s->free_lowres.emplace(sl.lowres_bytes, sl.lowres);
    s->st.bytes_in_flight -= sl.bytes;
    s->st.inflight--;
    s->st.completed++;
    sl = vdi_server_s::Slot();
    s->pending.erase(it);
}

// Collect completed requests (caller holds the lock).
void reap(vdi_server_s *s)
{
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        const uint64_t d = __atomic_load_n(&s->ctl->done[it->second], __ATOMIC_ACQUIRE);
        if (d == it->first) {
            auto nx = std::next(it);
            finish(s, it);
            it = nx;
        } else {
            ++it;
        }
    }
}

bool kernel_alive(vdi_server_s *s)
{
    if (!s->running) return false;
    const hipError_t q = hipStreamQuery(s->stream);
    if (q == hipErrorNotReady) return true;
    s->running = false;
    return false;
}

}  // namespace

extern "C" {

int vdi_server_create(uint64_t hbm_budget_bytes, int32_t max_inflight, int32_t workers, vdi_server_t *out)
{
    if (!out) return vdi::set_error(VDI_ERR_ARG, "null output");
    if (hbm_budget_bytes == 0) return vdi::set_error(VDI_ERR_ARG, "hbm_budget_bytes must be > 0");
    if (max_inflight < 1 || max_inflight > vdi::kMaxSlots)
        return vdi::set_error(VDI_ERR_ARG, "max_inflight must be in [1, %d]", vdi::kMaxSlots);
    if (workers < 0) return vdi::set_error(VDI_ERR_ARG, "workers must be >= 0");
    vdi_server_s *s = new (std::nothrow) vdi_server_s();
    if (!s) return vdi::set_error(VDI_ERR_OOM, "host allocation");
    hipError_t e = hipGetDevice(&s->device);
    auto bail = [&](hipError_t err, const char *what) {
        const int code = vdi::hip_error(err, what);
        if (s->ctl) (void)hipHostFree(s->ctl);
        if (s->desc) (void)hipHostFree(s->desc);
        if (s->dc) (void)hipFree(s->dc);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return code;
    };
    if (e != hipSuccess) return bail(e, "hipGetDevice");
    if ((e = hipHostMalloc((void **)&s->ctl, sizeof(vdi::Ctl), hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess)
        return bail(e, "control block");
    if ((e = hipHostMalloc((void **)&s->desc, sizeof(Job) * max_inflight, hipHostMallocCoherent | hipHostMallocMapped)) !=
        hipSuccess)
        return bail(e, "descriptors");
    memset(s->ctl, 0, sizeof(vdi::Ctl));
    memset(s->desc, 0, sizeof(Job) * max_inflight);
    if ((e = hipMalloc((void **)&s->dc, sizeof(vdi::DevCtr))) != hipSuccess) return bail(e, "device counters");
    if ((e = hipMemset(s->dc, 0, sizeof(vdi::DevCtr))) != hipSuccess) return bail(e, "device counters");
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    int occ = 0, cus = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, vdi::k_serve, vdi::kServeBlock, 0)) != hipSuccess)
        return bail(e, "occupancy");
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device)) != hipSuccess)
        return bail(e, "CU count");
    s->workers = workers > 0 ? workers : std::max(1, occ) * cus;
    s->budget = hbm_budget_bytes;
    s->max_inflight = max_inflight;
    s->slots.resize(max_inflight);
    vdi::k_serve<<<dim3((unsigned)s->workers), dim3(vdi::kServeBlock), 0, s->stream>>>(s->ctl, s->desc, s->dc);
    if ((e = hipGetLastError()) != hipSuccess) return bail(e, "serving kernel launch");
    s->running = true;
    s->st.kernel_running = 1;
    *out = s;
    return VDI_OK;
}

int vdi_server_submit(vdi_server_t s, vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R,
                      float *out, uint64_t *ticket)
{
    if (!s || !ticket) return vdi::set_error(VDI_ERR_ARG, "null argument");
    int rc = vdi::check_render_args(v, cam, W, H, D_I, D_R, out);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(s->mu);
    if (!kernel_alive(s)) return vdi::set_error(VDI_ERR_STATE, "the serving kernel is not running");
    reap(s);
    int32_t w, h;
    vdi::lowres_size(W, H, D_I, &w, &h);
    const bool down = (w != W || h != H);
    const uint64_t lowres_bytes = down ? (uint64_t)w * h * sizeof(float4) : 0;
    const uint64_t bytes = (uint64_t)W * H * sizeof(float4) + lowres_bytes;
    if (s->st.inflight >= s->max_inflight) {
        s->st.rejected_slots++;
        return vdi::set_error(VDI_ERR_BUDGET, "all %d request slots are in use", s->max_inflight);
    }
    if (s->st.bytes_in_flight + bytes > s->budget) {
        s->st.rejected_budget++;
        return vdi::set_error(VDI_ERR_BUDGET, "request needs %llu bytes; %llu of %llu in flight",
                              (unsigned long long)bytes, (unsigned long long)s->st.bytes_in_flight,
                              (unsigned long long)s->budget);
    }
    // The oldest pending request must keep its job record in the ring
    // (ticket t is job number t - 1).
    if (!s->pending.empty() && s->ctl->published_jobs - (s->pending.begin()->first - 1) >= (uint64_t)vdi::kJobRing) {
        s->st.rejected_slots++;
        return vdi::set_error(VDI_ERR_BUDGET, "job ring full");
    }
    vdi::Frame f;
    rc = vdi::make_frame(v, *cam, w, h, (double)W / (double)H, f);
    if (rc) return rc;
    float4 *lo = nullptr;
    if (down) {
        auto it = s->free_lowres.find(lowres_bytes);
        if (it != s->free_lowres.end()) {
            lo = it->second;
            s->free_lowres.erase(it);
        } else {
            const hipError_t e = hipMalloc((void **)&lo, lowres_bytes);
            if (e != hipSuccess) return vdi::hip_error(e, "preview scratch");
        }
    }
    int slot = -1;
    for (int i = 0; i < s->max_inflight; ++i) {
        const int c = (s->next_slot + i) % s->max_inflight;
        if (!s->slots[c].busy) {
            slot = c;
            break;
        }
    }
    s->next_slot = (slot + 1) % s->max_inflight;
    const uint64_t t = s->next_ticket++;
    Job &J = s->desc[slot];
    J.V = v->dev;
    J.F = f;
    J.F.out = down ? lo : reinterpret_cast<float4 *>(out);
    J.F.DR = D_R;
    J.F.ess = 1;
    J.F.search = VDI_SEARCH_SEEDED;
    J.out = reinterpret_cast<float4 *>(out);
    J.W = W;
    J.H = H;
    J.w = w;
    J.h = h;
    J.preview = D_R > 0.0f ? 1 : 0;
    J.tiles_x1 = (w + vdi::kTileW - 1) / vdi::kTileW;
    J.ntiles1 = vdi::tiles_of(w, h);
    J.ntiles2 = down ? vdi::tiles_of(W, H) : 0;
    J.ticket = t;
    const uint64_t jobno = s->ctl->published_jobs;
    JobRec &r = s->ctl->rec[jobno % vdi::kJobRing];
    r.base = s->ctl->published_tiles;
    r.jobno = jobno;
    r.ticket = t;
    r.ntiles = (uint32_t)(J.ntiles1 + J.ntiles2);
    r.slot = (uint32_t)slot;
    __atomic_store_n(&s->ctl->published_jobs, jobno + 1, __ATOMIC_RELEASE);
    __atomic_store_n(&s->ctl->published_tiles, r.base + r.ntiles, __ATOMIC_RELEASE);
    vdi_server_s::Slot &sl = s->slots[slot];
    sl.busy = true;
    sl.ticket = t;
    sl.bytes = bytes;
    sl.lowres = lo;
    sl.lowres_bytes = lowres_bytes;
    s->pending.emplace(t, slot);
    s->st.submitted++;
    s->st.inflight++;
    s->st.peak_inflight = std::max(s->st.peak_inflight, s->st.inflight);
    s->st.bytes_in_flight += bytes;
    s->st.peak_bytes_in_flight = std::max(s->st.peak_bytes_in_flight, s->st.bytes_in_flight);
    *ticket = t;
    return VDI_OK;
}

int vdi_server_poll(vdi_server_t s, uint64_t ticket, int *done)
{
    if (!s || !done) return vdi::set_error(VDI_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lock(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket) return vdi::set_error(VDI_ERR_ARG, "unknown ticket");
    auto it = s->pending.find(ticket);
    if (it == s->pending.end()) {
        *done = 1;
        return VDI_OK;
    }
    if (__atomic_load_n(&s->ctl->done[it->second], __ATOMIC_ACQUIRE) == ticket) {
        finish(s, it);
        *done = 1;
        return VDI_OK;
    }
    *done = 0;
    if (!kernel_alive(s)) return vdi::set_error(VDI_ERR_STATE, "the serving kernel stopped with requests pending");
    return VDI_OK;
}

int vdi_server_drain(vdi_server_t s)
{
    if (!s) return vdi::set_error(VDI_ERR_ARG, "null server");
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        {
            std::lock_guard<std::mutex> lock(s->mu);
            reap(s);
            if (s->pending.empty()) return VDI_OK;
            if (!kernel_alive(s)) return vdi::set_error(VDI_ERR_STATE, "the serving kernel stopped with requests pending");
        }
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
            return vdi::set_error(VDI_ERR_STATE, "drain timed out");
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

int vdi_server_get_stats(vdi_server_t s, vdi_server_stats *out)
{
    if (!s || !out) return vdi::set_error(VDI_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lock(s->mu);
    s->st.kernel_running = kernel_alive(s) ? 1 : 0;
    *out = s->st;
    return VDI_OK;
}

int vdi_server_destroy(vdi_server_t s)
{
    if (!s) return VDI_OK;
    int rc = vdi_server_drain(s);
    __atomic_store_n(&s->ctl->shutdown, 1u, __ATOMIC_RELEASE);
    hipError_t e = hipStreamSynchronize(s->stream);
    const uint32_t kerr = s->ctl->error;
    for (auto &kv : s->free_lowres) (void)hipFree(kv.second);
    for (auto &sl : s->slots)
        if (sl.lowres) (void)hipFree(sl.lowres);
    (void)hipStreamDestroy(s->stream);
    (void)hipFree(s->dc);
    (void)hipHostFree(s->desc);
    (void)hipHostFree(s->ctl);
    delete s;
    if (rc) return rc;
    if (e != hipSuccess) return vdi::hip_error(e, "serving kernel");
    if (kerr) return vdi::set_error(VDI_ERR_STATE, "the serving kernel timed out waiting (code %u)", kerr);
    return VDI_OK;
}

}  // extern "C"
