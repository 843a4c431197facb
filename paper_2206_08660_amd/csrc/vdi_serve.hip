// Served form of libvdi: continuous batching of render requests (not part
// of the paper's method, whose client renders one request at a time,
// Section 5).
//
// Requests are admitted while request slots and the device-memory budget
// allow, and queued.  Everything queued is launched as one batch as soon as
// one of the server's streams is free, by the submitting thread if a stream
// is free when it submits, otherwise by a scheduler thread: one launch per
// (mode, colour format) group renders the tiles of all of the group's
// requests (k_render_batch for exact tiles, k_render_batch_preview for
// preview tiles), and one more upsamples those with D_I > 1
// (k_upsample_batch).  With two or more streams the next batch starts while
// the previous one drains, so the tail of one batch is filled with the next
// one's tiles and the GPU does not idle between requests.  A request is done
// when its batch is; the scheduler thread, or a poll of one of its tickets,
// retires a batch once its completion event has passed.
//
// Each batch's job table is copied to device memory before its launches and
// stays unchanged until they finish, so the kernels read it like kernel
// arguments; no kernel waits on another or on the host.  The per-ray
// functions, frame constants and tile order are those of vdi_render, so a
// request's image is bit-identical to vdi_render's.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vdi_internal.h"

namespace vdi {
namespace {

constexpr int kMaxStreams = 8;
constexpr int kDefaultStreams = 3;
constexpr int kMaxSlots = 4096;
constexpr int kMaxBatch = 256;                 // requests per batch
// Render tiles per batch (8M rays, about four 1920 x 1080 frames): enough to
// fill the tail of each launch, small enough that a request does not wait
// long for the rest of its batch.  A larger single request forms a batch of
// its own.
#ifndef VDI_BATCH_TILES
#define VDI_BATCH_TILES ((1ull << 23) / (kTileW * kTileH))
#endif
constexpr uint64_t kBatchTiles = VDI_BATCH_TILES;
// Upsampling tiles per batch: keeps every launch far below 2^32 work-items.
constexpr uint64_t kBatchUpTiles = 1ull << 22;

// An admitted request.
struct Request {
    vdi_s *owner = nullptr;  // the VDI rendered (its server_refs counts this request)
    vdi_pace_s *pace = nullptr;  // session fed the request's latency when it is done (paced requests)
    std::chrono::steady_clock::time_point t_submit;
    BatchJob job;       // tile0 is set when its batch is built
    int32_t fmt = VDI_F32;
    bool preview = false, down = false;
    UpsampleJob up{};
    uint64_t bytes = 0, lowres_bytes = 0;
    float4 *lowres = nullptr;
    uint32_t slot = 0;  // persistent engine: the request's position in its launch's job table
};

// One stream and the buffers of the batch running on it.
struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    BatchJob *h_jobs = nullptr, *d_jobs = nullptr;    // kMaxBatch records, pinned host / device
    UpsampleJob *h_up = nullptr, *d_up = nullptr;
    std::vector<uint64_t> tickets;
    bool busy = false;
};

// Persistent engine (vdi_server_create_persistent): one resident launch of
// k_persist takes the tiles of every request published to it.  A request is
// published by writing its job record and then the new job count to
// coherent host memory, from which the launch's first workgroup copies it
// to device memory; the launch flags it done in host memory.  A launch serves
// one colour format and up to kPersistJobs requests, and only while no VDI
// has been created, destroyed or replaced since it started; otherwise, and
// after kPersistIdle with nothing to do, the host stops it once its
// published requests are done, and the next request starts a new one.
constexpr uint32_t kPersistJobs = 8192;
// Low-res images of a launch's D_I > 1 requests are carved in turn from one
// device buffer that is reused only by the next launch, so that upsampling
// tiles can read them through the caches (no cache holds an older copy of a
// line within a launch).  A request that does not fit ends the launch.
constexpr uint64_t kPersistLowresBytes = 2ull << 30;
// Completion counters: per job and part (render, upsampling), one counter per
// XCD group (the tiles k * kXcds + x of XCD x), each on a 128-byte line of
// its own, and one count of finished groups: the tiles of a job do not all
// update one word.
constexpr auto kPersistIdle = std::chrono::milliseconds(20);
// Sleeps (about 27 us each) a workgroup waits for work before it gives up
// and flags the launch as failed (about 1.8 s): far beyond kPersistIdle.
constexpr uint32_t kPersistSpins = 1u << 16;
struct Persist {
    hipStream_t kstream = nullptr;                     // the launches
    hipEvent_t end = nullptr;
    PQueue *d_q = nullptr;
    PJob *d_jobs = nullptr, *h_jobs = nullptr;          // kPersistJobs records, device / coherent host
    PHost *h_ctl = nullptr;                            // job count and stop word (coherent host memory)
    uint32_t *d_done = nullptr;                        // kPersistJobs * kDoneWords tile counters
    float4 *d_lowres = nullptr;                        // kPersistLowresBytes of low-res images
    uint64_t lowres_used = 0;                          // bytes of it given out in this launch
    uint32_t *h_done = nullptr;                        // kPersistJobs completion flags (coherent host memory)
    uint32_t blocks = 0;
    bool running = false, ending = false;
    int32_t fmt = VDI_F32;                             // colour format of the running launch
    uint32_t used = 0;                                 // jobs published to it
    uint64_t tiles = 0;                                // global tiles given out by it
    uint64_t mem_epoch = 0;                            // g_mem_epoch at its start
    std::vector<uint64_t> published;                   // its tickets not yet retired
    std::chrono::steady_clock::time_point idle_since;
};

// Workgroups of an exact render of w x h rays.
uint32_t exact_tiles(int w, int h)
{
    return (uint32_t)(((w + kXTileW - 1) / kXTileW) * ((h + kXTileH - 1) / kXTileH));
}
// Workgroups of 256 threads upsampling a W x H image (64 x 4 pixels each).
uint32_t upsample_tiles(int W, int H) { return (uint32_t)(((W + 63) / 64) * ((H + 3) / 4)); }
// Job starts are multiples of the XCD count.
uint64_t align_up(uint64_t x) { return (x + kXcds - 1) / kXcds * kXcds; }

}  // namespace
}  // namespace vdi

struct vdi_server_s {
    int device = 0;
    uint64_t budget = 0;
    int max_inflight = 0;
    std::vector<vdi::Lane> lanes;
    vdi::Persist *P = nullptr;                             // persistent engine (else batched launches on lanes)
    std::deque<uint64_t> queue;                            // admitted, not yet launched (FIFO)
    std::unordered_map<uint64_t, vdi::Request> requests;   // ticket -> request, until done
    std::multimap<uint64_t, float4 *> free_lowres;         // bytes -> pooled preview scratch
    std::vector<float4 *> all_lowres;
    vdi_server_stats st{};
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable wake;      // scheduler: new work or stop
    std::condition_variable progress;  // drain: a batch finished or failed
    std::thread scheduler;
    bool stop = false;
    int err = VDI_OK;
    std::string err_msg;
};

namespace vdi {
namespace {

// Record a failure of the scheduler: every later call reports it.
void fail(vdi_server_s *s, hipError_t e, const char *what)
{
    if (s->err) return;
    s->err = VDI_ERR_HIP;
    s->err_msg = std::string(what) + ": " + hipGetErrorString(e);
}

int report(vdi_server_s *s) { return set_error(s->err, "serving: %s", s->err_msg.c_str()); }

// Build the next batch from the queue and launch it on lane L (lock held).
void launch_batch(vdi_server_s *s, Lane &L)
{
    // Take requests in arrival order while the batch has room.
    std::vector<uint64_t> take;
    uint64_t tiles = 0, up_tiles = 0;
    while (!s->queue.empty() && (int)take.size() < kMaxBatch) {
        const Request &r = s->requests.at(s->queue.front());
        const uint64_t ut = r.down ? r.up.ntiles : 0;
        if (!take.empty() && (tiles + r.job.ntiles > kBatchTiles || up_tiles + ut > kBatchUpTiles)) break;
        tiles += r.job.ntiles;
        up_tiles += ut;
        take.push_back(s->queue.front());
        s->queue.pop_front();
    }
    // Job tables: one group per (mode, format), each sorted by tile0.
    int nj = 0, nu = 0;
    int group_start[2][3], group_count[2][3];
    uint32_t group_blocks[2][3];
    for (int p = 0; p < 2; ++p)
        for (int f = 0; f < 3; ++f) {
            group_start[p][f] = nj;
            uint64_t t = 0;
            for (uint64_t tk : take) {
                Request &r = s->requests.at(tk);
                if (r.preview != (p == 1) || r.fmt != f) continue;
                t = align_up(t);
                r.job.tile0 = (uint32_t)t;
                t += r.job.ntiles;
                L.h_jobs[nj++] = r.job;
            }
            group_count[p][f] = nj - group_start[p][f];
            group_blocks[p][f] = (uint32_t)t;
        }
    uint64_t tu = 0;
    for (uint64_t tk : take) {
        Request &r = s->requests.at(tk);
        if (!r.down) continue;
        tu = align_up(tu);
        r.up.tile0 = (uint32_t)tu;
        tu += r.up.ntiles;
        L.h_up[nu++] = r.up;
    }
    hipError_t e = hipMemcpyAsync(L.d_jobs, L.h_jobs, sizeof(BatchJob) * nj, hipMemcpyHostToDevice, L.stream);
    if (e == hipSuccess && nu)
        e = hipMemcpyAsync(L.d_up, L.h_up, sizeof(UpsampleJob) * nu, hipMemcpyHostToDevice, L.stream);
    for (int p = 0; p < 2 && e == hipSuccess; ++p)
        for (int f = 0; f < 3 && e == hipSuccess; ++f)
            if (group_count[p][f])
                e = launch_batch_render(L.d_jobs + group_start[p][f], group_count[p][f], group_blocks[p][f], f, p == 1,
                                        L.stream);
    if (e == hipSuccess && nu) e = launch_batch_upsample(L.d_up, nu, (uint32_t)tu, L.stream);
    if (e == hipSuccess) e = hipEventRecord(L.done, L.stream);
    L.tickets = std::move(take);
    L.busy = true;
    s->st.batches++;
    s->st.queued = (int32_t)s->queue.size();
    s->st.peak_batch = std::max(s->st.peak_batch, (int32_t)L.tickets.size());
    if (e != hipSuccess) fail(s, e, "batch launch");
}

// Retire a finished request (lock held).
void finish_request(vdi_server_s *s, uint64_t tk)
{
    {
        auto it = s->requests.find(tk);
        Request &r = it->second;
        if (r.lowres) s->free_lowres.emplace(r.lowres_bytes, r.lowres);
        r.owner->server_refs--;
        if (r.pace) {
            // The request's latency is the session's frame time.
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                         r.t_submit).count();
            s->st.paced_completed++;
            if (ms <= r.pace->target) s->st.deadlines_met++;
            pace_feed(r.pace, std::max(ms, 1e-3));
        }
        s->st.bytes_in_flight -= r.bytes;
        s->st.inflight--;
        s->st.completed++;
        s->requests.erase(it);
    }
}

// Retire the requests of lane L's finished batch (lock held).
void finish_batch(vdi_server_s *s, Lane &L)
{
    for (uint64_t tk : L.tickets) finish_request(s, tk);
    L.tickets.clear();
    L.busy = false;
}

// ---------------------------------------------------------------------------
// Persistent engine (lock held in all of these)
// ---------------------------------------------------------------------------
// Start a launch for colour format fmt: clear its queue and counters on the
// launch stream, let the feed stream copy only after that, launch.
void persist_launch(vdi_server_s *s, int32_t fmt)
{
    Persist &P = *s->P;
    // No launch is running: the host words can be cleared directly.
    memset(P.h_done, 0, sizeof(uint32_t) * kPersistJobs);
    __atomic_store_n(&P.h_ctl->tail.v, 0ull, __ATOMIC_RELEASE);
    __atomic_store_n(&P.h_ctl->stop.v, 0ull, __ATOMIC_RELEASE);
    hipError_t e = hipMemsetAsync(P.d_q, 0, sizeof(PQueue), P.kstream);
    if (e == hipSuccess) e = hipMemsetAsync(P.d_done, 0, sizeof(uint32_t) * kDoneWords * kPersistJobs, P.kstream);
    if (e == hipSuccess)
        e = launch_persist(fmt, P.h_ctl, P.h_jobs, P.d_q, P.d_jobs, P.d_done, P.h_done, P.blocks, kPersistSpins,
                           P.kstream);
    if (e == hipSuccess) e = hipEventRecord(P.end, P.kstream);
    if (e != hipSuccess) {
        fail(s, e, "persistent launch");
        return;
    }
    P.running = true;
    P.ending = false;
    P.fmt = fmt;
    P.used = 0;
    P.tiles = 0;
    P.lowres_used = 0;
    P.mem_epoch = g_mem_epoch.load();
    P.idle_since = std::chrono::steady_clock::now();
    s->st.batches++;
}

// Publish queued requests to the running launch, starting one if none runs;
// a request the launch cannot take marks it to be ended.
void persist_pump(vdi_server_s *s)
{
    Persist &P = *s->P;
    while (!s->queue.empty() && !s->err && !P.ending) {
        const uint64_t tk = s->queue.front();
        Request &r = s->requests.at(tk);
        if (!P.running) persist_launch(s, r.fmt);
        if (s->err) return;
        const uint64_t t0 = align_up(P.tiles);
        const uint64_t u0 = align_up(t0 + r.job.ntiles);
        const uint64_t end = r.down ? u0 + r.up.ntiles : t0 + r.job.ntiles;
        const uint64_t lowres = (r.lowres_bytes + 255) / 256 * 256;
        if (r.fmt != P.fmt || P.used >= kPersistJobs || end >= (1ull << 31) || g_mem_epoch.load() != P.mem_epoch ||
            P.lowres_used + lowres > kPersistLowresBytes) {
            P.ending = true;
            return;
        }
        const uint32_t j = P.used++;
        r.slot = j;
        r.job.tile0 = (uint32_t)t0;
        if (r.down) {
            r.job.F.out = P.d_lowres + P.lowres_used / sizeof(float4);
            r.up.lo = r.job.F.out;
            P.lowres_used += lowres;
        }
        PJob &J = P.h_jobs[j];
        J.R = r.job;
        J.U = r.up;
        J.U.tile0 = (uint32_t)u0;
        if (!r.down) J.U.ntiles = 0;
        J.end = (uint32_t)end;
        J.slot = j;
        J.preview = r.preview ? 1 : 0;
        J.pad = 0;
        P.tiles = end;
        // The record is written before the count that publishes it (x86 keeps store order).
        __atomic_store_n(&P.h_ctl->tail.v, (unsigned long long)(j + 1), __ATOMIC_RELEASE);
        s->queue.pop_front();
        P.published.push_back(tk);
        s->st.queued = (int32_t)s->queue.size();
    }
}

// Retire published requests whose flag the launch has set; true if any.
bool persist_retire(vdi_server_s *s)
{
    Persist &P = *s->P;
    bool any = false;
    for (size_t i = 0; i < P.published.size();) {
        const uint64_t tk = P.published[i];
        if (__atomic_load_n(&P.h_done[s->requests.at(tk).slot], __ATOMIC_ACQUIRE) != 0u) {
            finish_request(s, tk);
            P.published[i] = P.published.back();
            P.published.pop_back();
            any = true;
        } else {
            ++i;
        }
    }
    if (any || !P.published.empty() || !s->queue.empty()) P.idle_since = std::chrono::steady_clock::now();
    return any;
}

// State of an ended launch that left requests unfinished: its fault word,
// job count and tile counters, and the tile counts and flags of the first
// unfinished requests.
std::string persist_diagnose(vdi_server_s *s)
{
    Persist &P = *s->P;
    PQueue q{};
    std::string d;
    if (hipMemcpy(&q, P.d_q, sizeof q, hipMemcpyDeviceToHost) != hipSuccess) return "(queue unreadable)";
    char buf[256];
    snprintf(buf, sizeof buf, "fault %llu, workgroups %u started %llu exited %llu, jobs %llu/%u published, tiles given %llu; taken per XCD:",
             q.fault.v, P.blocks, q.started.v, q.exited.v, q.tail.v, P.used, (unsigned long long)P.tiles);
    d += buf;
    for (int x = 0; x < kXcds; ++x) d += " " + std::to_string(q.next[x].v);
    for (size_t i = 0; i < P.published.size() && i < 3; ++i) {
        const Request &r = s->requests.at(P.published[i]);
        std::vector<uint32_t> c(kDoneWords);
        (void)hipMemcpy(c.data(), P.d_done + (size_t)kDoneWords * r.slot, sizeof(uint32_t) * kDoneWords,
                        hipMemcpyDeviceToHost);
        uint32_t rt = 0, ut = 0;
        for (int x = 0; x < kXcds; ++x) rt += c[done_word(0, x)], ut += c[done_word(1, x)];
        const PJob &J = P.h_jobs[r.slot];
        snprintf(buf, sizeof buf, "; slot %u: render %u/%u (groups %u) from tile %u, upsample %u/%u (groups %u) from %u, end %u, flag %u",
                 r.slot, rt, J.R.ntiles, c[done_word(0, kXcds)], J.R.tile0, ut, J.U.ntiles, c[done_word(1, kXcds)],
                 J.U.tile0, J.end,
                 __atomic_load_n(&P.h_done[r.slot], __ATOMIC_ACQUIRE));
        d += buf;
    }
    return d;
}

// Write the stop word and wait for the launch to end; *fault gets its fault word.
hipError_t persist_halt(vdi_server_s *s, unsigned long long *fault)
{
    Persist &P = *s->P;
    __atomic_store_n(&P.h_ctl->stop.v, 1ull, __ATOMIC_RELEASE);
    hipError_t e = hipEventSynchronize(P.end);
    *fault = 0;
    if (e == hipSuccess) e = hipMemcpy(fault, &P.d_q->fault.v, sizeof *fault, hipMemcpyDeviceToHost);
    P.running = false;
    P.ending = false;
    return e;
}

// Stop the running launch when it has nothing left in flight and must end
// (it cannot take the next request, the server stops, or it has idled for
// kPersistIdle); also notice a launch that ended by itself (a fault).
void persist_check_end(vdi_server_s *s)
{
    Persist &P = *s->P;
    if (!P.running || s->err) return;
    if (!P.published.empty()) {
        if (hipEventQuery(P.end) == hipSuccess) {
            const std::string d = "persistent launch ended with work in flight (" + persist_diagnose(s) + ")";
            fail(s, hipErrorLaunchFailure, d.c_str());
        }
        return;
    }
    const bool idle = s->queue.empty() && std::chrono::steady_clock::now() - P.idle_since > kPersistIdle;
    if (!P.ending && !s->stop && !idle) return;
    unsigned long long fault = 0;
    const hipError_t e = persist_halt(s, &fault);
    if (e != hipSuccess) fail(s, e, "stopping the persistent launch");
    else if (fault) fail(s, hipErrorLaunchTimeOut, "persistent launch gave up waiting for work");
}

void run_scheduler(vdi_server_s *s)
{
    (void)hipSetDevice(s->device);
    // The 20 us polls below would otherwise sleep for Linux's default timer
    // slack of 50 us on top, which an idle-GPU request pays once or twice.
    (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(s->mu);
    while (s->P) {
        Persist &P = *s->P;
        bool retired = false;
        if (!s->err) {
            retired = persist_retire(s);
            persist_pump(s);
            persist_check_end(s);
            persist_pump(s);  // into a new launch, if the last one ended for the next request
        }
        if (s->err && P.running) {
            unsigned long long fault = 0;
            (void)persist_halt(s, &fault);
        }
        if (retired || s->err) s->progress.notify_all();
        if (s->stop && !P.running && (s->queue.empty() || s->err)) return;
        if (s->err) {
            s->wake.wait(lk, [&] { return s->stop; });
            continue;
        }
        if (!P.published.empty() || !s->queue.empty()) s->wake.wait_for(lk, std::chrono::microseconds(20));
        else if (P.running || s->stop) s->wake.wait_for(lk, std::chrono::milliseconds(2));
        else s->wake.wait(lk, [&] { return s->stop || !s->queue.empty() || !P.published.empty() || P.running; });
    }
    for (;;) {
        bool busy = false, retired = false;
        for (Lane &L : s->lanes) {
            if (!L.busy) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipSuccess) {
                finish_batch(s, L);
                retired = true;
            } else if (q == hipErrorNotReady) {
                busy = true;
            } else {
                fail(s, q, "batch");
                L.busy = false;
            }
        }
        if (!s->err)
            for (Lane &L : s->lanes)
                if (!L.busy && !s->queue.empty()) {
                    launch_batch(s, L);
                    busy = true;
                }
        if (retired || s->err) s->progress.notify_all();
        if (s->stop && !busy && (s->queue.empty() || s->err)) return;
        if (busy) {
            s->wake.wait_for(lk, std::chrono::microseconds(20));
        } else {
            // Also woken by a batch that a submitter launched itself.
            s->wake.wait(lk, [&] {
                if (s->stop || (!s->queue.empty() && !s->err)) return true;
                for (const Lane &L : s->lanes)
                    if (L.busy) return true;
                return false;
            });
        }
    }
}

// Free everything a server owns (its scheduler is not running).
void release(vdi_server_s *s)
{
    for (Lane &L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.h_jobs) (void)hipHostFree(L.h_jobs);
        if (L.h_up) (void)hipHostFree(L.h_up);
        if (L.d_jobs) (void)hipFree(L.d_jobs);
        if (L.d_up) (void)hipFree(L.d_up);
    }
    if (s->P) {
        vdi::Persist &P = *s->P;
        if (P.kstream) (void)hipStreamSynchronize(P.kstream);
        if (P.end) (void)hipEventDestroy(P.end);
        if (P.kstream) (void)hipStreamDestroy(P.kstream);
        if (P.d_q) (void)hipFree(P.d_q);
        if (P.d_jobs) (void)hipFree(P.d_jobs);
        if (P.d_done) (void)hipFree(P.d_done);
        if (P.d_lowres) (void)hipFree(P.d_lowres);
        if (P.h_jobs) (void)hipHostFree(P.h_jobs);
        if (P.h_ctl) (void)hipHostFree(P.h_ctl);
        if (P.h_done) (void)hipHostFree(P.h_done);
        delete s->P;
    }
    for (float4 *p : s->all_lowres) (void)hipFree(p);
    // Requests never retired (the server failed): their VDIs are not read any more.
    for (auto &kv : s->requests) kv.second.owner->server_refs--;
    delete s;
}

}  // namespace
}  // namespace vdi

namespace vdi {
namespace {
int submit(vdi_server_t s, vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, float *out,
           uint64_t *ticket, vdi_pace_s *pace)
{
    if (!s || !ticket) return vdi::set_error(VDI_ERR_ARG, "null argument");
    int rc = vdi::check_render_args(v, cam, W, H, D_I, D_R, out);
    if (rc) return rc;
    int32_t w, h;
    vdi::lowres_size(W, H, D_I, &w, &h);
    const bool down = (w != W || h != H);
    const uint64_t lowres_bytes = down ? (uint64_t)w * h * sizeof(float4) : 0;
    const uint64_t bytes = (uint64_t)W * H * sizeof(float4) + lowres_bytes;
    vdi::Request r;
    const vdi::VdiSet S = vdi::current(v);
    rc = vdi::make_frame(S, *cam, w, h, (double)W / (double)H, r.job.F);
    if (rc) return rc;
    std::unique_lock<std::mutex> lock(s->mu);
    if (s->err) return vdi::report(s);
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
    if (down && s->P && lowres_bytes > vdi::kPersistLowresBytes)
        return vdi::set_error(VDI_ERR_ARG, "low-res image of %llu bytes exceeds the persistent server's %llu",
                              (unsigned long long)lowres_bytes, (unsigned long long)vdi::kPersistLowresBytes);
    if (down && !s->P) {
        auto it = s->free_lowres.find(lowres_bytes);
        if (it != s->free_lowres.end()) {
            r.lowres = it->second;
            s->free_lowres.erase(it);
        } else {
            // A new scratch buffer: allocated without the lock, so that the
            // scheduler keeps launching and retiring batches meanwhile.
            lock.unlock();
            const hipError_t e = hipMalloc((void **)&r.lowres, lowres_bytes);
            if (e != hipSuccess) return vdi::hip_error(e, "preview scratch");
            lock.lock();
            s->all_lowres.push_back(r.lowres);
            if (s->err) {
                s->free_lowres.emplace(lowres_bytes, r.lowres);
                return vdi::report(s);
            }
            // Admission is checked again: other requests may have been admitted meanwhile.
            if (s->st.inflight >= s->max_inflight || s->st.bytes_in_flight + bytes > s->budget) {
                s->free_lowres.emplace(lowres_bytes, r.lowres);
                if (s->st.inflight >= s->max_inflight) s->st.rejected_slots++;
                else s->st.rejected_budget++;
                return vdi::set_error(VDI_ERR_BUDGET, "no room after allocating preview scratch; submit again");
            }
        }
    }
    r.job.V = S.dev;
    r.job.F.out = down ? r.lowres : reinterpret_cast<float4 *>(out);
    r.job.F.DR = D_R;
    r.job.F.ess = 1;
    r.job.F.search = VDI_SEARCH_WINDOW;
    r.job.tile0 = 0;
    r.job.ntiles = D_R > 0.0f ? vdi::preview_tiles(w, h) : vdi::exact_tiles(w, h);
    r.fmt = S.dev.fmt;
    r.preview = D_R > 0.0f;
    r.down = down;
    if (down) r.up = vdi::UpsampleJob{r.lowres, reinterpret_cast<float4 *>(out), w, h, W, H, 0, vdi::upsample_tiles(W, H)};
    r.bytes = bytes;
    r.lowres_bytes = lowres_bytes;
    r.owner = v;
    r.pace = pace;
    r.t_submit = std::chrono::steady_clock::now();
    v->server_refs++;
    const uint64_t t = s->next_ticket++;
    s->requests.emplace(t, r);
    s->queue.push_back(t);
    s->st.submitted++;
    s->st.inflight++;
    s->st.queued = (int32_t)s->queue.size();
    s->st.peak_inflight = std::max(s->st.peak_inflight, s->st.inflight);
    s->st.bytes_in_flight += bytes;
    s->st.peak_bytes_in_flight = std::max(s->st.peak_bytes_in_flight, s->st.bytes_in_flight);
    // Persistent engine: the submitter publishes the request itself.
    if (s->P) {
        int prev = -1;
        if (hipGetDevice(&prev) == hipSuccess && prev != s->device) (void)hipSetDevice(s->device);
        vdi::persist_pump(s);
        if (prev >= 0 && prev != s->device) (void)hipSetDevice(prev);
    }
    // A free stream: the submitter launches the queue itself, so that a
    // request on an idle server does not wait for the scheduler thread to
    // wake up; the scheduler then only watches the batch for completion.
    for (Lane &L : s->lanes) {
        if (L.busy || s->err) continue;
        int prev = -1;
        if (hipGetDevice(&prev) == hipSuccess && prev != s->device) (void)hipSetDevice(s->device);
        launch_batch(s, L);
        if (prev >= 0 && prev != s->device) (void)hipSetDevice(prev);
        break;
    }
    s->wake.notify_one();
    *ticket = t;
    return VDI_OK;
}
}  // namespace
}  // namespace vdi

// ---------------------------------------------------------------------------
// Many frames in one call on the caller's stream (vdi_render_batch): the same
// batched launches as a server batch, without the scheduler.
// ---------------------------------------------------------------------------
namespace vdi {
namespace {

constexpr int kRingSlots = 4;
// Blocks per launch of a batched render (far below 2^32 work-items).
constexpr uint64_t kLaunchBlocks = 1ull << 24;

// Pinned host job tables of one device, reused in turn once their copy to
// the device has finished.
struct JobRing {
    std::mutex mu;
    BatchJob *jobs[kRingSlots] = {};
    UpsampleJob *up[kRingSlots] = {};
    hipEvent_t copied[kRingSlots] = {};
    int next = 0;
    bool ready = false;
};
std::mutex g_rings_mu;
std::map<int, JobRing *> g_rings;  // one per device, kept until the process ends

hipError_t job_ring(int device, JobRing **out)
{
    JobRing *R;
    {
        std::lock_guard<std::mutex> lock(g_rings_mu);
        JobRing *&r = g_rings[device];
        if (!r) r = new (std::nothrow) JobRing();
        if (!r) return hipErrorOutOfMemory;
        R = r;
    }
    std::lock_guard<std::mutex> lock(R->mu);
    hipError_t e = hipSuccess;
    for (int k = 0; k < kRingSlots && !R->ready && e == hipSuccess; ++k) {
        if (!R->jobs[k]) e = hipHostMalloc((void **)&R->jobs[k], sizeof(BatchJob) * VDI_BATCH_MAX_FRAMES, 0);
        if (e == hipSuccess && !R->up[k])
            e = hipHostMalloc((void **)&R->up[k], sizeof(UpsampleJob) * VDI_BATCH_MAX_FRAMES, 0);
        if (e == hipSuccess && !R->copied[k]) e = hipEventCreateWithFlags(&R->copied[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) R->ready = true;
    *out = R;
    return e;
}

struct BatchItem {
    BatchJob job;
    UpsampleJob up{};
    int fmt = VDI_F32;
    bool preview = false, down = false;
    size_t lo_bytes = 0;
};

// One launch: jobs [start, start + count) of the device table, nblocks blocks.
struct Launch {
    int start, count;
    uint32_t nblocks;
    int fmt;
    bool preview;
};

int render_batch(int32_t n, const vdi_t *vdis, const vdi_camera *cams, const int32_t *widths, const int32_t *heights,
                 const float *D_I, const float *D_R, float *const *outs, hipStream_t st)
{
    if (n < 1 || n > VDI_BATCH_MAX_FRAMES)
        return set_error(VDI_ERR_ARG, "n must be in [1, %d] (got %d)", VDI_BATCH_MAX_FRAMES, n);
    if (!vdis || !cams || !widths || !heights || !D_I || !D_R || !outs) return set_error(VDI_ERR_ARG, "null array");
    std::vector<BatchItem> items((size_t)n);
    int device = -1;
    for (int i = 0; i < n; ++i) {
        int rc = check_render_args(vdis[i], &cams[i], widths[i], heights[i], D_I[i], D_R[i], outs[i]);
        if (rc) return set_error(rc, "frame %d: %s", i, vdi_last_error());
        if (i == 0) device = vdis[0]->device;
        else if (vdis[i]->device != device)
            return set_error(VDI_ERR_ARG, "frame %d renders a VDI of device %d, frame 0 one of device %d", i,
                             vdis[i]->device, device);
        int32_t w, h;
        lowres_size(widths[i], heights[i], D_I[i], &w, &h);
        BatchItem &it = items[(size_t)i];
        const VdiSet S = current(vdis[i]);
        rc = make_frame(S, cams[i], w, h, (double)widths[i] / (double)heights[i], it.job.F);
        if (rc) return set_error(rc, "frame %d: %s", i, vdi_last_error());
        it.job.V = S.dev;
        it.job.F.DR = D_R[i];
        it.job.F.ess = 1;
        it.job.F.search = VDI_SEARCH_WINDOW;
        it.fmt = S.dev.fmt;
        it.preview = D_R[i] > 0.0f;
        it.down = (w != widths[i] || h != heights[i]);
        it.job.ntiles = it.preview ? preview_tiles(w, h) : exact_tiles(w, h);
        if (it.down) {
            // Rounded up to a power of two (at least 1 MiB), as for vdi_render.
            it.lo_bytes = (size_t)1 << 20;
            while (it.lo_bytes < (size_t)w * h * sizeof(float4)) it.lo_bytes <<= 1;
            it.up = UpsampleJob{nullptr, reinterpret_cast<float4 *>(outs[i]), w, h, widths[i], heights[i], 0,
                                upsample_tiles(widths[i], heights[i])};
        } else {
            it.job.F.out = reinterpret_cast<float4 *>(outs[i]);
        }
    }
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_error(e, "hipSetDevice");
    hipMemPool_t pool = nullptr;
    e = library_pool(device, &pool);
    if (e != hipSuccess) return hip_error(e, "memory pool");
    // Stream-ordered allocations: low-res images, then the device job tables.
    std::vector<void *> allocs;
    auto release = [&]() {
        for (void *p : allocs) (void)hipFreeAsync(p, st);
    };
    for (BatchItem &it : items) {
        if (!it.down) continue;
        void *lo = nullptr;
        e = hipMallocFromPoolAsync(&lo, it.lo_bytes, pool, st);
        if (e != hipSuccess) {
            release();
            return hip_error(e, "preview scratch");
        }
        allocs.push_back(lo);
        it.job.F.out = static_cast<float4 *>(lo);
        it.up.lo = static_cast<float4 *>(lo);
    }
    BatchJob *d_jobs = nullptr;
    UpsampleJob *d_up = nullptr;
    e = hipMallocFromPoolAsync((void **)&d_jobs, sizeof(BatchJob) * (size_t)n, pool, st);
    if (e == hipSuccess) {
        allocs.push_back(d_jobs);
        e = hipMallocFromPoolAsync((void **)&d_up, sizeof(UpsampleJob) * (size_t)n, pool, st);
        if (e == hipSuccess) allocs.push_back(d_up);
    }
    if (e != hipSuccess) {
        release();
        return hip_error(e, "job tables");
    }
    JobRing *R = nullptr;
    e = job_ring(device, &R);
    if (e != hipSuccess) {
        release();
        return hip_error(e, "pinned job tables");
    }
    // Job tables: one group per (mode, format), cut into launches of at most
    // kLaunchBlocks blocks; a job starts at a multiple of the XCD count.
    std::vector<Launch> launches, up_launches;
    {
        std::lock_guard<std::mutex> lock(R->mu);
        const int k = R->next;
        R->next = (k + 1) % kRingSlots;
        e = hipEventSynchronize(R->copied[k]);
        int nj = 0, nu = 0;
        for (int p = 0; p < 2 && e == hipSuccess; ++p)
            for (int f = 0; f < 3; ++f) {
                uint64_t t = 0;
                int start = nj;
                for (const BatchItem &it : items) {
                    if (it.preview != (p == 1) || it.fmt != f) continue;
                    if (nj > start && align_up(t) + it.job.ntiles > kLaunchBlocks) {
                        launches.push_back({start, nj - start, (uint32_t)t, f, p == 1});
                        start = nj;
                        t = 0;
                    }
                    t = align_up(t);
                    R->jobs[k][nj] = it.job;
                    R->jobs[k][nj].tile0 = (uint32_t)t;
                    t += it.job.ntiles;
                    ++nj;
                }
                if (nj > start) launches.push_back({start, nj - start, (uint32_t)t, f, p == 1});
            }
        uint64_t tu = 0;
        int ustart = 0;
        for (const BatchItem &it : items) {
            if (!it.down) continue;
            if (nu > ustart && align_up(tu) + it.up.ntiles > kLaunchBlocks) {
                up_launches.push_back({ustart, nu - ustart, (uint32_t)tu, 0, false});
                ustart = nu;
                tu = 0;
            }
            tu = align_up(tu);
            R->up[k][nu] = it.up;
            R->up[k][nu].tile0 = (uint32_t)tu;
            tu += it.up.ntiles;
            ++nu;
        }
        if (nu > ustart) up_launches.push_back({ustart, nu - ustart, (uint32_t)tu, 0, false});
        if (e == hipSuccess) e = hipMemcpyAsync(d_jobs, R->jobs[k], sizeof(BatchJob) * nj, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && nu)
            e = hipMemcpyAsync(d_up, R->up[k], sizeof(UpsampleJob) * nu, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(R->copied[k], st);
    }
    for (const Launch &L : launches) {
        if (e != hipSuccess) break;
        e = launch_batch_render(d_jobs + L.start, L.count, L.nblocks, L.fmt, L.preview, st);
    }
    for (const Launch &L : up_launches) {
        if (e != hipSuccess) break;
        e = launch_batch_upsample(d_up + L.start, L.count, L.nblocks, st);
    }
    release();
    if (e != hipSuccess) return hip_error(e, "batched render");
    for (int i = 0; i < n; ++i) {
        bool seen = false;
        for (int j = 0; j < i && !seen; ++j) seen = vdis[j] == vdis[i];
        if (seen) continue;
        e = note_use(vdis[i], st);
        if (e != hipSuccess) return hip_error(e, "render event");
    }
    return VDI_OK;
}

}  // namespace
}  // namespace vdi

extern "C" {

int vdi_server_create_persistent(uint64_t hbm_budget_bytes, int32_t max_inflight, int32_t waves_per_simd,
                                 vdi_server_t *out)
{
    if (!out) return vdi::set_error(VDI_ERR_ARG, "null output");
    *out = nullptr;
    if (hbm_budget_bytes == 0) return vdi::set_error(VDI_ERR_ARG, "hbm_budget_bytes must be > 0");
    if (max_inflight < 1 || max_inflight > vdi::kMaxSlots)
        return vdi::set_error(VDI_ERR_ARG, "max_inflight must be in [1, %d]", vdi::kMaxSlots);
    if (waves_per_simd < 0 || waves_per_simd > 16) return vdi::set_error(VDI_ERR_ARG, "waves_per_simd must be in [0, 16]");
    vdi_server_s *s = new (std::nothrow) vdi_server_s();
    if (!s) return vdi::set_error(VDI_ERR_OOM, "host allocation");
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return vdi::hip_error(e, "hipGetDevice");
    }
    s->budget = hbm_budget_bytes;
    s->max_inflight = max_inflight;
    s->P = new (std::nothrow) vdi::Persist();
    if (!s->P) {
        delete s;
        return vdi::set_error(VDI_ERR_OOM, "host allocation");
    }
    vdi::Persist &P = *s->P;
    const char *what = "streams";
    e = hipStreamCreateWithFlags(&P.kstream, hipStreamNonBlocking);
    if (e == hipSuccess) what = "event", e = hipEventCreateWithFlags(&P.end, hipEventDisableTiming);
    if (e == hipSuccess) what = "job queue", e = hipMalloc((void **)&P.d_q, sizeof(vdi::PQueue));
    if (e == hipSuccess) e = hipMalloc((void **)&P.d_jobs, sizeof(vdi::PJob) * vdi::kPersistJobs);
    if (e == hipSuccess) e = hipMalloc((void **)&P.d_done, sizeof(uint32_t) * vdi::kDoneWords * vdi::kPersistJobs);
    if (e == hipSuccess) what = "low-res images", e = hipMalloc((void **)&P.d_lowres, vdi::kPersistLowresBytes);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&P.h_jobs, sizeof(vdi::PJob) * vdi::kPersistJobs, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void **)&P.h_ctl, sizeof(vdi::PHost), hipHostMallocCoherent);
    if (e == hipSuccess)
        what = "completion flags",
        e = hipHostMalloc((void **)&P.h_done, sizeof(uint32_t) * vdi::kPersistJobs, hipHostMallocCoherent);
    if (e == hipSuccess) {
        memset(P.h_ctl, 0, sizeof(vdi::PHost));
        // Workgroup 0 copies the records; the others take tiles.
        P.blocks = vdi::persist_blocks(s->device, waves_per_simd);
        if (P.blocks == 0) what = "occupancy query", e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) {
        const int rc = vdi::hip_error(e, what);
        vdi::release(s);
        return rc;
    }
    try {
        s->scheduler = std::thread(vdi::run_scheduler, s);
    } catch (...) {
        vdi::release(s);
        return vdi::set_error(VDI_ERR_OOM, "scheduler thread");
    }
    *out = s;
    return VDI_OK;
}

int vdi_server_create(uint64_t hbm_budget_bytes, int32_t max_inflight, int32_t streams, vdi_server_t *out)
{
    if (!out) return vdi::set_error(VDI_ERR_ARG, "null output");
    *out = nullptr;
    if (hbm_budget_bytes == 0) return vdi::set_error(VDI_ERR_ARG, "hbm_budget_bytes must be > 0");
    if (max_inflight < 1 || max_inflight > vdi::kMaxSlots)
        return vdi::set_error(VDI_ERR_ARG, "max_inflight must be in [1, %d]", vdi::kMaxSlots);
    if (streams < 0 || streams > vdi::kMaxStreams)
        return vdi::set_error(VDI_ERR_ARG, "streams must be in [0, %d]", vdi::kMaxStreams);
    vdi_server_s *s = new (std::nothrow) vdi_server_s();
    if (!s) return vdi::set_error(VDI_ERR_OOM, "host allocation");
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return vdi::hip_error(e, "hipGetDevice");
    }
    s->budget = hbm_budget_bytes;
    s->max_inflight = max_inflight;
    s->lanes.resize(streams ? streams : vdi::kDefaultStreams);
    for (vdi::Lane &L : s->lanes) {
        const char *what = "stream";
        e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) what = "event", e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e == hipSuccess)
            what = "job table", e = hipHostMalloc((void **)&L.h_jobs, sizeof(vdi::BatchJob) * vdi::kMaxBatch, 0);
        if (e == hipSuccess)
            what = "job table", e = hipHostMalloc((void **)&L.h_up, sizeof(vdi::UpsampleJob) * vdi::kMaxBatch, 0);
        if (e == hipSuccess) what = "job table", e = hipMalloc((void **)&L.d_jobs, sizeof(vdi::BatchJob) * vdi::kMaxBatch);
        if (e == hipSuccess)
            what = "job table", e = hipMalloc((void **)&L.d_up, sizeof(vdi::UpsampleJob) * vdi::kMaxBatch);
        if (e != hipSuccess) {
            const int rc = vdi::hip_error(e, what);
            vdi::release(s);
            return rc;
        }
    }
    try {
        s->scheduler = std::thread(vdi::run_scheduler, s);
    } catch (...) {
        vdi::release(s);
        return vdi::set_error(VDI_ERR_OOM, "scheduler thread");
    }
    *out = s;
    return VDI_OK;
}


int vdi_server_submit(vdi_server_t s, vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R,
                      float *out, uint64_t *ticket)
{
    return vdi::submit(s, v, cam, W, H, D_I, D_R, out, ticket, nullptr);
}

int vdi_server_submit_paced(vdi_server_t s, vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, vdi_pace_t session,
                            float D_R, float *out, uint64_t *ticket, float *D_I_used)
{
    if (!session || !D_I_used) return vdi::set_error(VDI_ERR_ARG, "null argument");
    const float D_I = (float)vdi::pace_d_i(session);
    const int rc = vdi::submit(s, v, cam, W, H, D_I, D_R, out, ticket, session);
    if (rc == VDI_OK) *D_I_used = D_I;
    return rc;
}

int vdi_render_batch(int32_t n, const vdi_t *vdis, const vdi_camera *cams, const int32_t *widths,
                     const int32_t *heights, const float *D_I, const float *D_R, float *const *outs, void *hip_stream)
{
    return vdi::render_batch(n, vdis, cams, widths, heights, D_I, D_R, outs, static_cast<hipStream_t>(hip_stream));
}

int vdi_server_poll(vdi_server_t s, uint64_t ticket, int *done)
{
    if (!s || !done) return vdi::set_error(VDI_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lock(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket) return vdi::set_error(VDI_ERR_ARG, "unknown ticket");
    if (s->P && s->requests.count(ticket) && !s->err) {
        if (vdi::persist_retire(s)) {
            s->progress.notify_all();
            s->wake.notify_one();
        }
    } else if (s->requests.count(ticket) && !s->err) {
        // Retire the ticket's batch here if it has finished, rather than at
        // the scheduler's next look at it.
        for (vdi::Lane &L : s->lanes) {
            if (!L.busy || std::find(L.tickets.begin(), L.tickets.end(), ticket) == L.tickets.end()) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipSuccess) {
                vdi::finish_batch(s, L);
                s->progress.notify_all();
                s->wake.notify_one();
            } else if (q != hipErrorNotReady) {
                vdi::fail(s, q, "batch");
                L.busy = false;
                s->progress.notify_all();
            }
            break;
        }
    }
    *done = s->requests.count(ticket) ? 0 : 1;
    if (!*done && s->err) return vdi::report(s);
    return VDI_OK;
}

int vdi_server_drain(vdi_server_t s)
{
    if (!s) return vdi::set_error(VDI_ERR_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->progress.wait_for(lk, std::chrono::seconds(60), [&] { return s->requests.empty() || s->err; });
    if (s->err) return vdi::report(s);
    if (!ok) return vdi::set_error(VDI_ERR_STATE, "drain timed out with %d requests in flight", s->st.inflight);
    return VDI_OK;
}

int vdi_server_get_stats(vdi_server_t s, vdi_server_stats *out)
{
    if (!s || !out) return vdi::set_error(VDI_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->st;
    return VDI_OK;
}

int vdi_server_reset_stats(vdi_server_t s)
{
    if (!s) return vdi::set_error(VDI_ERR_ARG, "null server");
    std::lock_guard<std::mutex> lock(s->mu);
    vdi_server_stats &st = s->st;
    st.submitted = st.completed = st.rejected_budget = st.rejected_slots = st.batches = 0;
    st.paced_completed = st.deadlines_met = 0;
    st.peak_bytes_in_flight = st.bytes_in_flight;
    st.peak_inflight = st.inflight;
    st.peak_batch = 0;
    return VDI_OK;
}

int vdi_server_destroy(vdi_server_t s)
{
    if (!s) return VDI_OK;
    const int rc = vdi_server_drain(s);
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->wake.notify_all();
    }
    s->scheduler.join();
    vdi::release(s);
    return rc;
}

}  // extern "C"
