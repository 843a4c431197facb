// Host side of the libvdi C ABI (include/vdi.h): argument checking, device
// residency of VDIs, per-frame set-up in double precision, kernel launches.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "vdi_internal.h"

namespace vdi {
std::atomic<uint64_t> g_mem_epoch{0};
}

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? VDI_ERR_OOM : VDI_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_OR_FAIL(expr, what)                   \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool finite3(const float *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

struct Basis {
    double eye[3], F[3], R[3], U[3], th;
};

void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

double norm(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

// Camera basis F = normalize(target - eye), R = normalize(F x up), U = R x F.
int make_basis(const vdi_camera &c, Basis &b)
{
    if (!finite3(c.eye) || !finite3(c.target) || !finite3(c.up) || !isfinite(c.fov_y_deg) || !isfinite(c.near_plane))
        return fail(VDI_ERR_ARG, "camera has a non-finite value");
    if (!(c.fov_y_deg > 0.0f && c.fov_y_deg < 180.0f)) return fail(VDI_ERR_ARG, "fov_y_deg must be in (0, 180)");
    if (!(c.near_plane > 0.0f)) return fail(VDI_ERR_ARG, "near_plane must be > 0");
    double up[3];
    for (int a = 0; a < 3; ++a) {
        b.eye[a] = c.eye[a];
        b.F[a] = (double)c.target[a] - (double)c.eye[a];
        up[a] = c.up[a];
    }
    double n = norm(b.F);
    if (!(n > 0.0)) return fail(VDI_ERR_ARG, "camera target equals eye");
    for (double &x : b.F) x /= n;
    cross(b.F, up, b.R);
    n = norm(b.R);
    if (!(n > 1e-12)) return fail(VDI_ERR_ARG, "camera up is parallel to the view direction");
    for (double &x : b.R) x /= n;
    cross(b.R, b.F, b.U);
    b.th = tan((double)c.fov_y_deg * M_PI / 360.0);
    return VDI_OK;
}

double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Frame constants for rays on a w x h grid with aspect `aspect`, for the VDI set S.
int build_frame(const vdi::VdiSet &S, const vdi_camera &cam, int w, int h, double aspect, vdi::Frame &f)
{
    Basis o, n;
    int rc = make_basis(S.cam_o, o);
    if (rc) return rc;
    rc = make_basis(cam, n);
    if (rc) return rc;
    memset(&f, 0, sizeof f);
    const double aspect_o = (double)S.dev.WO / (double)S.dev.HO;
    for (int a = 0; a < 3; ++a) {
        f.FO[a] = o.F[a];
        f.RO[a] = o.R[a];
        f.UO[a] = o.U[a];
        f.eyeN[a] = n.eye[a];
        f.FN[a] = n.F[a];
        f.RN[a] = n.R[a];
        f.UN[a] = n.U[a];
        f.bmin[a] = S.bmin[a];
        f.bmax[a] = S.bmax[a];
    }
    f.sx_o = 1.0 / (o.th * aspect_o);
    f.sy_o = 1.0 / o.th;
    f.near_o = S.cam_o.near_plane;
    double rel[3];
    for (int a = 0; a < 3; ++a) rel[a] = n.eye[a] - o.eye[a];
    f.X0 = dot(o.R, rel) * f.sx_o;
    f.Y0 = dot(o.U, rel) * f.sy_o;
    f.Z0 = dot(o.F, rel);
    f.tx_n = n.th * aspect;
    f.ty_n = n.th;
    f.near_n = cam.near_plane;
    f.W = w;
    f.H = h;
    f.ess = 1;
    f.search = VDI_SEARCH_WINDOW;
    f.parts = vdi::preview_parts(w, h);
    return VDI_OK;
}

int check_opts(const vdi_render_opts *opts, vdi::Frame &f)
{
    if (!opts) return VDI_OK;
    if (opts->ess != 0 && opts->ess != 1) return fail(VDI_ERR_ARG, "opts.ess must be 0 or 1");
    if (opts->search < VDI_SEARCH_SEEDED || opts->search > VDI_SEARCH_WINDOW)
        return fail(VDI_ERR_ARG, "opts.search must be a VDI_SEARCH_* value");
    f.ess = opts->ess;
    f.search = opts->search;
    return VDI_OK;
}

int lowres_dims(int32_t W, int32_t H, float D_I, int32_t *w, int32_t *h)
{
    *w = std::max(1, (int32_t)floor((double)W / (double)D_I + 0.5));
    *h = std::max(1, (int32_t)floor((double)H / (double)D_I + 0.5));
    return VDI_OK;
}

int check_args(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, const float *out)
{
    if (!v) return fail(VDI_ERR_ARG, "null VDI handle");
    if (!cam) return fail(VDI_ERR_ARG, "null camera");
    if (!out) return fail(VDI_ERR_ARG, "null output pointer");
    if (W < 1 || H < 1 || W > 16384 || H > 16384) return fail(VDI_ERR_ARG, "image size %dx%d out of range", W, H);
    if (!isfinite(D_I) || D_I < 1.0f) return fail(VDI_ERR_ARG, "D_I must be a finite value >= 1");
    if (!isfinite(D_R) || D_R < 0.0f || (D_R > 0.0f && D_R < 1e-4f))
        return fail(VDI_ERR_ARG, "D_R must be 0 or a finite value >= 1e-4");
    return VDI_OK;
}

// Stream-ordered memory pool of the library on `device`, for the low-res
// scratch of downsampled renders.  Freed blocks stay in the pool (release
// threshold unlimited): a session whose D_I changes every frame, with a
// synchronisation per frame, would otherwise map fresh memory for most
// frames.  Created on first use and kept until the process ends.
hipError_t scratch_pool(int device, hipMemPool_t *out)
{
    static std::mutex mu;
    static std::vector<hipMemPool_t> pools;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((int)pools.size() <= device) pools.resize(device + 1, nullptr);
    if (!pools[device]) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        hipMemPool_t p = nullptr;
        hipError_t e = hipMemPoolCreate(&p, &props);
        if (e != hipSuccess) return e;
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(p);
            return e;
        }
        pools[device] = p;
    }
    *out = pools[device];
    return hipSuccess;
}

// Allocation-free downsampled renders (vdi_render_noalloc) keep their
// low-res image in this library-owned array, one copy per device, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address on each device comes from
// hipGetSymbolAddress (noalloc_scratch), and only that address is passed on.
constexpr size_t kNoAllocTexels = VDI_NOALLOC_SCRATCH_TEXELS;  // 32 MiB of float4
static __device__ __align__(256) float4 scratch[kNoAllocTexels];

// Device address of `scratch` on `device` (current), looked up once per device.
hipError_t noalloc_scratch(int device, float4 **out)
{
    static std::mutex mu;
    static std::vector<float4 *> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
    if (!addr[device]) {
        float4 *p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

// Renders into `out` (W x H).  For D_I > 1 the low-res image goes to
// stream-ordered scratch from the library's pool, or, with noalloc, to the
// library's static array (no allocation of any kind).
int render_impl(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R,
                const vdi_render_opts *opts, float *out, hipStream_t s, bool noalloc = false)
{
    int rc = check_args(v, cam, W, H, D_I, D_R, out);
    if (rc) return rc;
    int32_t w, h;
    lowres_dims(W, H, D_I, &w, &h);
    const bool down = (w != W || h != H);
    if (noalloc && down && (size_t)w * (size_t)h > kNoAllocTexels)
        return fail(VDI_ERR_ARG, "low-res image %dx%d exceeds the allocation-free scratch (%zu texels)", w, h,
                    kNoAllocTexels);
    const vdi::VdiSet S = vdi::current(v);
    vdi::Frame f;
    rc = build_frame(S, *cam, w, h, (double)W / (double)H, f);
    if (rc) return rc;
    rc = check_opts(opts, f);
    if (rc) return rc;
    HIP_OR_FAIL(hipSetDevice(v->device), "hipSetDevice");
    float4 *lo = nullptr;
    if (down && noalloc) {
        HIP_OR_FAIL(noalloc_scratch(v->device, &lo), "hipGetSymbolAddress(scratch)");
    } else if (down) {
        hipMemPool_t pool = nullptr;
        HIP_OR_FAIL(scratch_pool(v->device, &pool), "scratch pool");
        // Sizes rounded up to a power of two (at least 1 MiB): a D_I that
        // changes every frame then reuses a few pooled blocks.
        size_t bytes = (size_t)1 << 20;
        while (bytes < (size_t)w * h * sizeof(float4)) bytes <<= 1;
        HIP_OR_FAIL(hipMallocFromPoolAsync((void **)&lo, bytes, pool, s), "preview scratch");
    }
    f.out = down ? lo : reinterpret_cast<float4 *>(out);
    f.DR = D_R;
    hipError_t e = D_R > 0.0f ? vdi::launch_render_preview(S.dev, f, false, s) : vdi::launch_render_exact(S.dev, f, false, s);
    if (e == hipSuccess && down) e = vdi::launch_upsample(lo, w, h, reinterpret_cast<float4 *>(out), W, H, s);
    if (down && !noalloc) {
        hipError_t e2 = hipFreeAsync(lo, s);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = vdi::note_use(v, s);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return VDI_OK;
}

// Host-side validation of every list (optional at create).
int validate_lists(const vdi_desc *d)
{
    const uint64_t plane = (uint64_t)d->width * d->height;
    for (uint64_t li = 0; li < plane; ++li) {
        const int n = d->count[li];
        if (n > d->max_supersegments) return fail(VDI_ERR_ARG, "list %llu: count %d > N_S", (unsigned long long)li, n);
        float prev_b = -INFINITY;
        for (int j = 0; j < n; ++j) {
            const uint64_t o = (uint64_t)j * plane + li;
            const float f = d->depth[2 * o], b = d->depth[2 * o + 1];
            if (!isfinite(f) || !isfinite(b) || !(f < b))
                return fail(VDI_ERR_ARG, "list %llu slot %d: need finite f < b", (unsigned long long)li, j);
            if (f < prev_b)
                return fail(VDI_ERR_ARG, "list %llu slot %d: supersegments unsorted or overlapping",
                            (unsigned long long)li, j);
            prev_b = b;
            if (d->rgba_fmt_in == VDI_F32) {
                const float *c = static_cast<const float *>(d->rgba) + 4 * o;
                if (!isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2]) || !(c[3] >= 0.0f && c[3] <= 1.0f))
                    return fail(VDI_ERR_ARG, "list %llu slot %d: colour not finite or opacity outside [0, 1]",
                                (unsigned long long)li, j);
            }
        }
    }
    return VDI_OK;
}

void free_set(vdi::VdiSet &S)
{
    // Errors are ignored: every pointer was allocated here or is null.
    (void)hipFree(S.d_count);
    (void)hipFree(S.d_depth);
    (void)hipFree(S.d_rgba);
    (void)hipFree(S.d_grid);
    (void)hipFree(S.d_gbits);
    (void)hipFree(S.d_gz);
    S = vdi::VdiSet();
}

void free_vdi(vdi_s *v)
{
    if (!v) return;
    if (v->copy) (void)hipStreamSynchronize(v->copy);
    free_set(v->cur);
    free_set(v->back);
    if (v->stage) (void)hipFreeAsync(v->stage, v->copy);
    if (v->copy) (void)hipStreamSynchronize(v->copy);
    for (int i = 0; i < vdi_s::kUseSlots; ++i)
        if (v->use_ev[i]) (void)hipEventDestroy(v->use_ev[i]);
    if (v->start) (void)hipEventDestroy(v->start);
    if (v->ready) (void)hipEventDestroy(v->ready);
    if (v->copy) (void)hipStreamDestroy(v->copy);
    delete v;
}

// Checks of a descriptor common to vdi_create and vdi_replace_begin; on
// success fills the V_O basis and the grid slice boundaries.
// The count plane in host memory: d->count itself, or a copy of it in
// `copy` when the planes are in device memory (they must be complete).
int host_counts(const vdi_desc *d, std::vector<uint8_t> &copy, const uint8_t **out)
{
    if (!d->planes_on_device) {
        *out = d->count;
        return VDI_OK;
    }
    copy.resize((size_t)d->width * d->height);
    const hipError_t e = hipMemcpy(copy.data(), d->count, copy.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "count plane download");
    *out = copy.data();
    return VDI_OK;
}

int check_desc(const vdi_desc *d, Basis &ob, std::vector<float> &gz, const uint8_t **counts, std::vector<uint8_t> &count_copy)
{
    if (d->width < 1 || d->height < 1 || d->width > 32768 || d->height > 32768)
        return fail(VDI_ERR_ARG, "VDI size %dx%d out of range", d->width, d->height);
    if (d->max_supersegments < 1 || d->max_supersegments > VDI_MAX_SUPERSEGMENTS)
        return fail(VDI_ERR_ARG, "max_supersegments must be in [1, 255]");
    if (!d->count || !d->depth || !d->rgba) return fail(VDI_ERR_ARG, "null VDI plane");
    if (d->rgba_fmt_in < VDI_F32 || d->rgba_fmt_in > VDI_BF16 || d->rgba_fmt_store < VDI_F32 ||
        d->rgba_fmt_store > VDI_BF16)
        return fail(VDI_ERR_ARG, "unknown colour format");
    if (d->rgba_fmt_in != VDI_F32 && d->rgba_fmt_in != d->rgba_fmt_store)
        return fail(VDI_ERR_ARG, "16-bit colour input must be stored in the same format");
    if (d->grid_k < 1 || d->grid_k > VDI_MAX_GRID_K || d->grid_nz < 1 || d->grid_nz > VDI_MAX_GRID_NZ)
        return fail(VDI_ERR_ARG, "grid shape out of range (k 1..16, nz 1..64)");
    // Cell indices are 32-bit in the kernels.
    if ((uint64_t)d->grid_nz * ((d->width + d->grid_k - 1) / d->grid_k) * ((d->height + d->grid_k - 1) / d->grid_k) >=
        (1ull << 31))
        return fail(VDI_ERR_ARG, "count grid too large (needs fewer than 2^31 cells)");
    if (!finite3(d->aabb_min) || !finite3(d->aabb_max)) return fail(VDI_ERR_ARG, "non-finite AABB");
    for (int a = 0; a < 3; ++a)
        if (!(d->aabb_max[a] > d->aabb_min[a])) return fail(VDI_ERR_ARG, "empty AABB");
    int rc = make_basis(d->camera_VO, ob);
    if (rc) return rc;
    if (d->planes_on_device != 0 && d->planes_on_device != 1) return fail(VDI_ERR_ARG, "planes_on_device must be 0 or 1");
    if (d->planes_on_device && d->validate)
        return fail(VDI_ERR_ARG, "list validation reads the planes on the host: not available for device planes");
    rc = host_counts(d, count_copy, counts);
    if (rc) return rc;
    const uint64_t plane = (uint64_t)d->width * d->height;
    for (uint64_t li = 0; li < plane; ++li)
        if ((*counts)[li] > d->max_supersegments) return fail(VDI_ERR_ARG, "a list count exceeds max_supersegments");
    if (d->validate) {
        rc = validate_lists(d);
        if (rc) return rc;
    }
    // Grid slice boundaries.
    gz.assign(d->grid_nz + 1, 0.0f);
    if (d->grid_z) {
        for (int c = 0; c <= d->grid_nz; ++c) {
            gz[c] = d->grid_z[c];
            if (!isfinite(gz[c]) || (c > 0 && !(gz[c] > gz[c - 1])))
                return fail(VDI_ERR_ARG, "grid_z must be finite and strictly increasing");
        }
    } else {
        double lo = INFINITY, hi = -INFINITY;
        for (int m = 0; m < 8; ++m) {
            double p[3] = {(m & 1) ? d->aabb_max[0] : d->aabb_min[0], (m & 2) ? d->aabb_max[1] : d->aabb_min[1],
                           (m & 4) ? d->aabb_max[2] : d->aabb_min[2]};
            double rel[3] = {p[0] - ob.eye[0], p[1] - ob.eye[1], p[2] - ob.eye[2]};
            const double z = dot(ob.F, rel);
            lo = std::min(lo, z);
            hi = std::max(hi, z);
        }
        lo -= 1e-3;
        hi += 1e-3;
        for (int c = 0; c <= d->grid_nz; ++c) gz[c] = (float)(lo + (hi - lo) * c / d->grid_nz);
    }
    return VDI_OK;
}

uint64_t set_bytes_of(const vdi_desc *d)
{
    const uint64_t plane = (uint64_t)d->width * d->height;
    const uint64_t colour = d->rgba_fmt_store == VDI_F32 ? 16 : 8;
    const uint64_t gw = (d->width + d->grid_k - 1) / d->grid_k, gh = (d->height + d->grid_k - 1) / d->grid_k;
    const uint64_t cells = (uint64_t)d->grid_nz * gw * gh;
    return plane + vdi::plane_elems(d->width, d->height, d->max_supersegments) * (8 + colour) + cells * sizeof(uint32_t) +
           (cells + 31) / 32 * sizeof(uint32_t) + (uint64_t)(d->grid_nz + 1) * sizeof(float);
}

// Host-to-device copies of a VDI's arrays.  A copy from pageable host memory
// waits for the device's other streams (measured: a create stalled behind a
// server's running batch); copies from pinned memory are ordered on their
// stream only.  Host arrays therefore go through two pinned halves of the
// library, taken in turn: a half is refilled once the copy that last read it
// has completed.  The halves are allocated on first use and kept.
constexpr size_t kPinHalf = (size_t)32 << 20;
std::mutex g_pin_mu;
void *g_pin[2] = {nullptr, nullptr};
hipEvent_t g_pin_ev[2] = {nullptr, nullptr};

hipError_t h2d(void *dst, const void *src, size_t n, hipStream_t st)
{
    std::lock_guard<std::mutex> lock(g_pin_mu);
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        if (!g_pin[k]) e = hipHostMalloc(&g_pin[k], kPinHalf, hipHostMallocDefault);
        if (e == hipSuccess && !g_pin_ev[k]) e = hipEventCreateWithFlags(&g_pin_ev[k], hipEventDisableTiming);
    }
    static int k = 0;
    for (size_t off = 0; off < n && e == hipSuccess; off += kPinHalf, k ^= 1) {
        const size_t m = std::min(n - off, kPinHalf);
        e = hipEventSynchronize(g_pin_ev[k]);
        if (e != hipSuccess) break;
        memcpy(g_pin[k], static_cast<const char *>(src) + off, m);
        e = hipMemcpyAsync(static_cast<char *>(dst) + off, g_pin[k], m, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(g_pin_ev[k], st);
    }
    return e;
}

// A copy of a VDI array: device to device when the planes are on the device.
hipError_t copy_in(void *dst, const void *src, size_t n, bool on_device, hipStream_t st)
{
    if (on_device) return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, st);
    return h2d(dst, src, n, st);
}

// Upload d into the set S on stream st: allocate S's buffers if it has none,
// copy the count plane and slice boundaries, stage whole slot planes through
// `stage` (stage_bytes) and scatter them into storage order (colour
// converted on the way), then build the count grid.  Enqueues only; the
// caller synchronises.  `gz` must stay valid until the work has run.
hipError_t upload_set(vdi::VdiSet &S, const vdi_desc *d, const uint8_t *counts, const Basis &ob,
                      const std::vector<float> &gz, hipStream_t st, void *stage, uint64_t stage_bytes, const char **what)
{
    const uint64_t plane = (uint64_t)d->width * d->height;
    const uint64_t ns = (uint64_t)d->max_supersegments;
    const size_t colour = d->rgba_fmt_store == VDI_F32 ? 16 : 8;
    vdi::DevVDI &D = S.dev;
    D.WO = d->width;
    D.HO = d->height;
    D.NS = d->max_supersegments;
    D.fmt = d->rgba_fmt_store;
    D.plane = plane;
    D.sstride = vdi::kBrick ? (uint64_t)vdi::kBrick : plane;
    D.gk = d->grid_k;
    D.gnz = d->grid_nz;
    D.GW = (d->width + d->grid_k - 1) / d->grid_k;
    D.GH = (d->height + d->grid_k - 1) / d->grid_k;
    D.tx_o = (float)(ob.th * ((double)d->width / d->height));
    D.ty_o = (float)ob.th;
    D.dcx = 2.0 / d->width;
    D.dcy = 2.0 / d->height;
    D.inv_gk = nextafterf(1.0f / (float)d->grid_k, INFINITY);
    S.cam_o = d->camera_VO;
    memcpy(S.bmin, d->aabb_min, sizeof S.bmin);
    memcpy(S.bmax, d->aabb_max, sizeof S.bmax);
    const uint64_t elems = vdi::plane_elems(d->width, d->height, (int)ns);
    const size_t grid_bytes = (size_t)D.gnz * D.GH * D.GW * sizeof(uint32_t);
    const size_t gbits_bytes = ((size_t)D.gnz * D.GH * D.GW + 31) / 32 * sizeof(uint32_t);
    hipError_t e = hipSuccess;
    if (!S.d_count) {
        *what = "device allocation";
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_count, plane);
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_depth, elems * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&S.d_rgba, elems * colour);
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_grid, grid_bytes);
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_gbits, gbits_bytes);
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_gz, gz.size() * sizeof(float));
        if (e != hipSuccess) return e;
    }
    D.count = S.d_count;
    D.depth = S.d_depth;
    D.rgba = S.d_rgba;
    D.grid = S.d_grid;
    D.gbits = S.d_gbits;
    D.gz = S.d_gz;
    *what = "upload";
    const bool on_dev = d->planes_on_device != 0;
    e = copy_in(S.d_count, d->count, plane, on_dev, st);
    if (e == hipSuccess) e = h2d(S.d_gz, gz.data(), gz.size() * sizeof(float), st);
    const size_t colour_in = d->rgba_fmt_in == VDI_F32 ? 16 : 8;
    const uint64_t slots = std::max<uint64_t>(1, std::min<uint64_t>(ns, stage_bytes / (plane * 16)));
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        const bool dep = pass == 0;
        const size_t esz = dep ? sizeof(float2) : colour_in;
        const char *src = static_cast<const char *>(dep ? (const void *)d->depth : d->rgba);
        for (uint64_t j0 = 0; j0 < ns && e == hipSuccess; j0 += slots) {
            const uint64_t nj = std::min(slots, ns - j0);
            // Stream order keeps the staging buffer from being refilled before it is scattered.
            e = copy_in(stage, src + j0 * plane * esz, nj * plane * esz, on_dev, st);
            if (e == hipSuccess)
                e = vdi::launch_scatter_slots(stage, d->rgba_fmt_in, dep ? (void *)S.d_depth : S.d_rgba, d->rgba_fmt_store,
                                              dep, nj * plane, D, (int32_t)j0, st);
        }
    }
    if (e != hipSuccess) return e;
    *what = "grid build";
    e = vdi::launch_grid_build(D, S.d_grid, st);
    if (e == hipSuccess) e = vdi::launch_grid_bits(D, S.d_gbits, st);
    uint64_t total = 0;
    for (uint64_t li = 0; li < plane; ++li) total += counts[li];
    S.supersegments = total;
    return e;
}

}  // namespace

namespace vdi {
// PI control of x = ln D_I on the error e = ln(frame / target), velocity
// form: x += kp (e - e_prev) + ki e, clamped to [ln D_I_min, ln D_I_max].
double pace_feed(vdi_pace_s *p, double frame_ms)
{
    std::lock_guard<std::mutex> lock(p->mu);
    const double e = log(frame_ms / p->target);
    const double de = p->first ? 0.0 : e - p->e_prev;
    p->x = std::min(p->xmax, std::max(p->xmin, p->x + p->kp * de + p->ki * e));
    p->e_prev = e;
    p->first = false;
    return exp(p->x);
}

double pace_d_i(vdi_pace_s *p)
{
    std::lock_guard<std::mutex> lock(p->mu);
    return exp(p->x);
}

hipError_t note_use(vdi_s *v, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(v->mu);
    int k = -1;
    for (int i = 0; i < v->use_n; ++i)
        if (v->use_st[i] == stream) k = i;
    if (k < 0 && v->use_n < vdi_s::kUseSlots) k = v->use_n++;
    if (k < 0) {
        // More streams than slots: the least recently used one is waited for
        // and its slot taken over.
        k = 0;
        for (int i = 1; i < vdi_s::kUseSlots; ++i)
            if (v->use_tick[i] < v->use_tick[k]) k = i;
        const hipError_t e = hipEventSynchronize(v->use_ev[k]);
        if (e != hipSuccess) return e;
    }
    v->use_st[k] = stream;
    v->use_tick[k] = ++v->use_clock;
    return hipEventRecord(v->use_ev[k], stream);
}

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
int hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }
int check_render_args(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, const float *out)
{
    return ::check_args(v, cam, W, H, D_I, D_R, out);
}
void lowres_size(int32_t W, int32_t H, float D_I, int32_t *w, int32_t *h) { ::lowres_dims(W, H, D_I, w, h); }
hipError_t library_pool(int device, hipMemPool_t *out) { return ::scratch_pool(device, out); }
int make_frame(const VdiSet &S, const vdi_camera &cam, int w, int h, double aspect, Frame &f)
{
    return ::build_frame(S, cam, w, h, aspect, f);
}
VdiSet current(vdi_s *v)
{
    std::lock_guard<std::mutex> lock(v->mu);
    return v->cur;
}
}  // namespace vdi

extern "C" {

const char *vdi_last_error(void) { return g_err.c_str(); }

uint64_t vdi_plane_bytes(int32_t width, int32_t height, int32_t n_s, int32_t fmt)
{
    if (width < 1 || height < 1 || n_s < 1) return 0;
    const uint64_t plane = (uint64_t)width * height;
    const uint64_t colour = fmt == VDI_F32 ? 16 : 8;
    return plane + vdi::plane_elems(width, height, n_s) * (8 + colour);
}


int vdi_pace_create(float target_ms, float kp, float ki, float D_I_min, float D_I_max, float D_I_start,
                    vdi_pace_t *out)
{
    g_err.clear();
    if (!out) return fail(VDI_ERR_ARG, "null output");
    if (!isfinite(target_ms) || !(target_ms > 0.0f)) return fail(VDI_ERR_ARG, "target_ms must be > 0");
    if (!isfinite(kp) || !isfinite(ki) || kp < 0.0f || ki < 0.0f) return fail(VDI_ERR_ARG, "gains must be >= 0");
    if (!isfinite(D_I_min) || !isfinite(D_I_max) || !isfinite(D_I_start) || !(D_I_min >= 1.0f) ||
        !(D_I_min <= D_I_start) || !(D_I_start <= D_I_max))
        return fail(VDI_ERR_ARG, "need 1 <= D_I_min <= D_I_start <= D_I_max");
    vdi_pace_s *p = new (std::nothrow) vdi_pace_s();
    if (!p) return fail(VDI_ERR_OOM, "host allocation");
    p->target = target_ms;
    p->kp = kp;
    p->ki = ki;
    p->xmin = log((double)D_I_min);
    p->xmax = log((double)D_I_max);
    p->x = log((double)D_I_start);
    p->e_prev = 0.0;
    p->first = true;
    *out = p;
    return VDI_OK;
}

int vdi_pace_update(vdi_pace_t p, float frame_ms, float *next_D_I)
{
    g_err.clear();
    if (!p || !next_D_I) return fail(VDI_ERR_ARG, "null argument");
    if (!isfinite(frame_ms) || !(frame_ms > 0.0f)) return fail(VDI_ERR_ARG, "frame_ms must be > 0");
    *next_D_I = (float)vdi::pace_feed(p, frame_ms);
    return VDI_OK;
}

int vdi_pace_destroy(vdi_pace_t p)
{
    delete p;
    return VDI_OK;
}

int vdi_lowres_size(int32_t width, int32_t height, float D_I, int32_t *w, int32_t *h)
{
    if (!w || !h) return fail(VDI_ERR_ARG, "null output");
    if (width < 1 || height < 1 || !isfinite(D_I) || D_I < 1.0f) return fail(VDI_ERR_ARG, "invalid size or D_I");
    return lowres_dims(width, height, D_I, w, h);
}

int vdi_create(const vdi_desc *d, vdi_t *out)
{
    g_err.clear();
    if (!d || !out) return fail(VDI_ERR_ARG, "null argument");
    Basis ob;
    std::vector<float> gz;
    std::vector<uint8_t> count_copy;
    const uint8_t *counts = nullptr;
    int rc = check_desc(d, ob, gz, &counts, count_copy);
    if (rc) return rc;
    vdi_s *v = new (std::nothrow) vdi_s();
    if (!v) return fail(VDI_ERR_OOM, "host allocation");
    hipError_t e = hipGetDevice(&v->device);
    if (e != hipSuccess) {
        delete v;
        return hip_fail(e, "hipGetDevice");
    }
    const uint64_t plane = (uint64_t)d->width * d->height;
    const uint64_t stage_bytes = std::max<uint64_t>(256ull << 20, plane * 16);
    void *stage = nullptr;
    const char *what = "events";
    for (int i = 0; i < vdi_s::kUseSlots && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&v->use_ev[i], hipEventDisableTiming);
    // The upload runs on the VDI's own stream and only that stream is waited
    // for: work on the device's other streams (a server's batches, other
    // VDIs' renders) goes on meanwhile.  The staging buffer is stream-ordered
    // on it (hipFree would wait for the whole device).  The planes come from
    // hipMalloc: from the stream-ordered pool, growing it by a VDI's size
    // waited for the device's other work as well (measured).
    if (e == hipSuccess) what = "VDI stream", e = hipStreamCreateWithFlags(&v->copy, hipStreamNonBlocking);
    hipStream_t st = v->copy;
    if (e == hipSuccess) what = "staging", e = hipMallocAsync(&stage, stage_bytes, st);
    if (e == hipSuccess) e = upload_set(v->cur, d, counts, ob, gz, st, stage, stage_bytes, &what);
    if (stage) {
        const hipError_t ef = hipFreeAsync(stage, st);
        if (e == hipSuccess) e = ef;
    }
    if (st) {
        const hipError_t es = hipStreamSynchronize(st);
        if (e == hipSuccess) what = "upload", e = es;
    }
    if (e != hipSuccess) {
        rc = hip_fail(e, what);
        free_vdi(v);
        return rc;
    }
    v->set_bytes = set_bytes_of(d);
    vdi::g_mem_epoch.fetch_add(1);
    *out = v;
    return VDI_OK;
}

int vdi_replace_begin(vdi_t v, const vdi_desc *d, void *stream)
{
    g_err.clear();
    if (!v || !d) return fail(VDI_ERR_ARG, "null argument");
    // Device planes may still be being written on the caller's stream.
    if (d->planes_on_device) {
        const hipError_t es = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (es != hipSuccess) return hip_fail(es, "waiting for the caller's stream");
    }
    Basis ob;
    std::vector<float> gz;
    std::vector<uint8_t> count_copy;
    const uint8_t *counts = nullptr;
    int rc = check_desc(d, ob, gz, &counts, count_copy);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lock(v->mu);
        const vdi::DevVDI &C = v->cur.dev;
        if (d->width != C.WO || d->height != C.HO || d->max_supersegments != C.NS || d->rgba_fmt_store != C.fmt ||
            d->grid_k != C.gk || d->grid_nz != C.gnz)
            return fail(VDI_ERR_ARG, "the replacement must have the shape, N_S, colour format and grid of the VDI");
        if (v->pending) return fail(VDI_ERR_STATE, "a replacement is already pending");
        v->pending = true;
        v->enqueued = false;
        v->gz_host = gz;
    }
    // From here only this call touches the back set and the copy stream.
    const uint64_t plane = (uint64_t)d->width * d->height;
    const char *what = "replacement set-up";
    hipError_t e = hipSetDevice(v->device);
    if (e == hipSuccess && !v->start) {
        e = hipEventCreateWithFlags(&v->start, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&v->ready, hipEventDisableTiming);
        if (e == hipSuccess) {
            v->stage_bytes = std::max<uint64_t>(256ull << 20, plane * 16);
            e = hipMallocAsync(&v->stage, v->stage_bytes, v->copy);
        }
    }
    // The back set may be the one renders used before the last swap: the
    // upload waits for the work already enqueued on the caller's stream.
    if (e == hipSuccess) e = hipEventRecord(v->start, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamWaitEvent(v->copy, v->start, 0);
    if (e == hipSuccess) e = upload_set(v->back, d, counts, ob, v->gz_host, v->copy, v->stage, v->stage_bytes, &what);
    if (e == hipSuccess) what = "replacement", e = hipEventRecord(v->ready, v->copy);
    std::lock_guard<std::mutex> lock(v->mu);
    if (e != hipSuccess) {
        v->pending = false;
        return hip_fail(e, what);
    }
    v->enqueued = true;
    return VDI_OK;
}

int vdi_replace_poll(vdi_t v, int32_t *swapped)
{
    g_err.clear();
    if (!v || !swapped) return fail(VDI_ERR_ARG, "null argument");
    *swapped = 0;
    std::lock_guard<std::mutex> lock(v->mu);
    if (!v->pending || !v->enqueued) return VDI_OK;
    const hipError_t q = hipEventQuery(v->ready);
    if (q == hipErrorNotReady) return VDI_OK;
    v->pending = false;
    v->enqueued = false;
    if (q != hipSuccess) return hip_fail(q, "replacement upload");
    std::swap(v->cur, v->back);
    vdi::g_mem_epoch.fetch_add(1);
    *swapped = 1;
    return VDI_OK;
}

int vdi_render(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, float *out, void *stream)
{
    g_err.clear();
    return render_impl(v, cam, W, H, D_I, D_R, nullptr, out, static_cast<hipStream_t>(stream));
}

int vdi_render_noalloc(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, float *out,
                       void *stream)
{
    return render_impl(v, cam, W, H, D_I, D_R, nullptr, out, static_cast<hipStream_t>(stream), true);
}

int vdi_render_ex(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R,
                  const vdi_render_opts *opts, float *out, void *stream)
{
    g_err.clear();
    return render_impl(v, cam, W, H, D_I, D_R, opts, out, static_cast<hipStream_t>(stream));
}

int vdi_render_counters(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, const vdi_render_opts *opts,
                        float *out, uint8_t *touched_lists, uint8_t *touched_slots, int32_t *ray_stats, void *stream)
{
    g_err.clear();
    int rc = check_args(v, cam, W, H, 1.0f, 0.0f, out);
    if (rc) return rc;
    if (!touched_lists || !touched_slots) return fail(VDI_ERR_ARG, "null counter buffer");
    const vdi::VdiSet S = vdi::current(v);
    vdi::Frame f;
    rc = build_frame(S, *cam, W, H, (double)W / (double)H, f);
    if (rc) return rc;
    rc = check_opts(opts, f);
    if (rc) return rc;
    HIP_OR_FAIL(hipSetDevice(v->device), "hipSetDevice");
    f.out = reinterpret_cast<float4 *>(out);
    f.touched_lists = touched_lists;
    f.touched_slots = touched_slots;
    f.ray_stats = ray_stats;
    HIP_OR_FAIL(vdi::launch_render_exact(S.dev, f, true, static_cast<hipStream_t>(stream)), "counter render launch");
    HIP_OR_FAIL(vdi::note_use(v, static_cast<hipStream_t>(stream)), "render bookkeeping");
    return VDI_OK;
}

int vdi_preview_counters(vdi_t v, const vdi_camera *cam, int32_t W, int32_t H, float D_I, float D_R, float *lowres_out,
                         uint8_t *touched_lists, uint8_t *touched_slots, uint8_t *touched_cells, int32_t *ray_stats,
                         void *stream)
{
    g_err.clear();
    int rc = check_args(v, cam, W, H, D_I, D_R, lowres_out);
    if (rc) return rc;
    if (!(D_R > 0.0f)) return fail(VDI_ERR_ARG, "vdi_preview_counters needs D_R > 0");
    if (!touched_lists || !touched_slots || !touched_cells) return fail(VDI_ERR_ARG, "null counter buffer");
    int32_t w, h;
    lowres_dims(W, H, D_I, &w, &h);
    const vdi::VdiSet S = vdi::current(v);
    vdi::Frame f;
    rc = build_frame(S, *cam, w, h, (double)W / (double)H, f);
    if (rc) return rc;
    HIP_OR_FAIL(hipSetDevice(v->device), "hipSetDevice");
    f.out = reinterpret_cast<float4 *>(lowres_out);
    f.DR = D_R;
    f.touched_lists = touched_lists;
    f.touched_slots = touched_slots;
    f.touched_cells = touched_cells;
    f.ray_stats = ray_stats;
    HIP_OR_FAIL(vdi::launch_render_preview(S.dev, f, true, static_cast<hipStream_t>(stream)), "counter preview launch");
    HIP_OR_FAIL(vdi::note_use(v, static_cast<hipStream_t>(stream)), "render bookkeeping");
    return VDI_OK;
}

int vdi_get_grid(vdi_t v, uint32_t *host_out, size_t capacity)
{
    g_err.clear();
    if (!v || !host_out) return fail(VDI_ERR_ARG, "null argument");
    const vdi::VdiSet S = vdi::current(v);
    const size_t n = (size_t)S.dev.gnz * S.dev.GH * S.dev.GW;
    if (capacity < n) return fail(VDI_ERR_ARG, "grid needs %zu elements", n);
    HIP_OR_FAIL(hipSetDevice(v->device), "hipSetDevice");
    HIP_OR_FAIL(hipMemcpy(host_out, S.d_grid, n * sizeof(uint32_t), hipMemcpyDeviceToHost), "grid download");
    return VDI_OK;
}

int vdi_get_info(vdi_t v, vdi_info_t *info)
{
    g_err.clear();
    if (!v || !info) return fail(VDI_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lock(v->mu);
    const vdi::VdiSet &S = v->cur;
    info->width = S.dev.WO;
    info->height = S.dev.HO;
    info->max_supersegments = S.dev.NS;
    info->rgba_fmt = S.dev.fmt;
    info->grid_k = S.dev.gk;
    info->grid_nz = S.dev.gnz;
    info->grid_w = S.dev.GW;
    info->grid_h = S.dev.GH;
    info->device_bytes = v->set_bytes * (v->back.d_count ? 2 : 1) + (v->stage ? v->stage_bytes : 0);
    info->supersegments = S.supersegments;
    return VDI_OK;
}

int vdi_destroy(vdi_t v)
{
    g_err.clear();
    if (!v) return VDI_OK;
    hipError_t e = hipSetDevice(v->device);
    // Wait for what reads v's buffers: its renders (the last one on each
    // stream that rendered it), a replacement upload, and a server's requests.
    {
        std::lock_guard<std::mutex> lock(v->mu);
        for (int i = 0; i < v->use_n && e == hipSuccess; ++i) e = hipEventSynchronize(v->use_ev[i]);
    }
    if (e == hipSuccess && v->copy) e = hipStreamSynchronize(v->copy);
    for (int waited_ms = 0; e == hipSuccess && v->server_refs.load() > 0; ++waited_ms) {
        if (waited_ms >= 60000)
            return fail(VDI_ERR_STATE, "a server still holds %d requests on this VDI", v->server_refs.load());
        std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "waiting for work on the VDI before destroy");
        free_vdi(v);
        vdi::g_mem_epoch.fetch_add(1);
        return rc;
    }
    free_vdi(v);
    vdi::g_mem_epoch.fetch_add(1);
    return VDI_OK;
}

}  // extern "C"
