// Host replay of the exact walker's global loads, for measuring how much of
// a wavefront's memory traffic it could serve from storage of its own (the
// LDS, or its share of the L1).
//
// The per-ray code is the library's (vdi_trace.h), built for the host with
// its load hook defined to record, per ray, every global load: the 128-byte
// line it falls in, its stream (counts, occupancy bits, depth pairs,
// colours) and the main-loop iteration it belongs to.  The 64 rays of one
// exact tile are then replayed in the order a wavefront issues them: main-loop
// iteration by iteration, and within an iteration the k-th load of every lane
// as one load instruction, whose lanes that fall in one line make one request
// (the coalescing of a vector load).  The requests go through an LRU cache of
// a given capacity in lines, one per wavefront, counted by stack distance:
// a request hits a cache of C lines when fewer than C other lines were
// requested since the previous request of its line.
//
// The VDI is laid out in the library's device order (bricks) in host memory
// aligned like a device allocation, so lines are those of the device.
#include <stdint.h>

#include <hip/hip_runtime.h>

// Recorders of the load hook: they record on the host and do nothing in the
// device build of the same kernels.
__host__ __device__ void reuse_note(const void *p, int stream);
__host__ __device__ void reuse_step();
#define VDI_LOAD(p, stream) (reuse_note((const void *)(p), stream), *(p))
#define VDI_STEP() reuse_step()

#include "vdi_kernels.hip"
#include "vdi_api.hip"

#include <algorithm>
#include <cstdlib>
#include <unordered_map>
#include <vector>

namespace {

struct Load {
    int it;
    int stream;
    uint64_t line;
};
thread_local std::vector<Load> *g_rec = nullptr;
thread_local int g_it = 0;

// Fenwick tree over request times: a 1 marks the latest request of a line.
struct Fenwick {
    std::vector<int> t;
    void init(size_t n) { t.assign(n + 1, 0); }
    void add(size_t i, int v)
    {
        for (++i; i < t.size(); i += i & (~i + 1)) t[i] += v;
    }
    int prefix(size_t i) const  // sum over [0, i)
    {
        int s = 0;
        for (; i > 0; i -= i & (~i + 1)) s += t[i];
        return s;
    }
};

struct Layout {
    vdi::VdiSet v;
    vdi::Frame f;
    void *mem[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Layout()
    {
        for (void *p : mem) std::free(p);
    }
};

void *aligned(size_t bytes)
{
    return std::aligned_alloc(256, (bytes + 255) / 256 * 256);
}

int setup(const vdi_desc *d, const uint32_t *grid, const vdi_camera *cam, int W, int H, Layout &L)
{
    vdi::VdiSet &v = L.v;
    v.cam_o = d->camera_VO;
    memcpy(v.bmin, d->aabb_min, sizeof v.bmin);
    memcpy(v.bmax, d->aabb_max, sizeof v.bmax);
    vdi::DevVDI &D = v.dev;
    D.WO = d->width;
    D.HO = d->height;
    D.NS = d->max_supersegments;
    D.fmt = VDI_F32;
    D.plane = (uint64_t)d->width * d->height;
    D.sstride = vdi::kBrick ? (uint64_t)vdi::kBrick : D.plane;
    const uint64_t elems = vdi::plane_elems(D.WO, D.HO, D.NS);
    float2 *dep = (float2 *)aligned(elems * sizeof(float2));
    float4 *col = (float4 *)aligned(elems * sizeof(float4));
    uint8_t *cnt = (uint8_t *)aligned(D.plane);
    const uint32_t ncells =
        (uint32_t)d->grid_nz * ((d->height + d->grid_k - 1) / d->grid_k) * ((d->width + d->grid_k - 1) / d->grid_k);
    uint32_t *bits = (uint32_t *)aligned((ncells + 31) / 32 * sizeof(uint32_t));
    L.mem[0] = dep;
    L.mem[1] = col;
    L.mem[2] = cnt;
    L.mem[3] = bits;
    if (!dep || !col || !cnt || !bits) return VDI_ERR_OOM;
    for (uint64_t e = 0; e < elems; ++e) {
        dep[e] = make_float2(NAN, NAN);
        col[e] = make_float4(NAN, NAN, NAN, NAN);
    }
    for (int j = 0; j < D.NS; ++j)
        for (uint64_t li = 0; li < D.plane; ++li) {
            const uint64_t o = vdi::list_base(li, D.NS, D.WO) + (uint64_t)j * D.sstride;
            dep[o] = reinterpret_cast<const float2 *>(d->depth)[(uint64_t)j * D.plane + li];
            col[o] = static_cast<const float4 *>(d->rgba)[(uint64_t)j * D.plane + li];
        }
    memcpy(cnt, d->count, D.plane);
    memset(bits, 0, (ncells + 31) / 32 * sizeof(uint32_t));
    for (uint32_t c = 0; c < ncells; ++c)
        if (grid[c] != 0u) bits[c / 32] |= 1u << (c % 32);
    D.count = cnt;
    D.depth = dep;
    D.rgba = col;
    D.grid = grid;
    D.gbits = bits;
    D.gk = d->grid_k;
    D.gnz = d->grid_nz;
    D.GW = (d->width + d->grid_k - 1) / d->grid_k;
    D.GH = (d->height + d->grid_k - 1) / d->grid_k;
    D.gz = d->grid_z;
    Basis ob;
    int rc = make_basis(d->camera_VO, ob);
    if (rc) return rc;
    D.tx_o = (float)(ob.th * ((double)d->width / d->height));
    D.ty_o = (float)ob.th;
    D.dcx = 2.0 / d->width;
    D.dcy = 2.0 / d->height;
    D.inv_gk = nextafterf(1.0f / (float)d->grid_k, INFINITY);
    rc = build_frame(v, *cam, W, H, (double)W / H, L.f);
    if (rc) return rc;
    L.f.ess = 1;
    L.f.search = VDI_SEARCH_WINDOW;
    L.f.DR = 0;
    return VDI_OK;
}

// The requests of exact tile (tx, ty), in issue order: (line, stream) pairs.
void tile_requests(const Layout &L, int W, int H, int tx, int ty, std::vector<std::pair<uint64_t, int>> &req)
{
    std::vector<Load> rec[64];
    for (int l = 0; l < 64; ++l) {
        const int px = tx * vdi::kXTileW + l % vdi::kXTileW, py = ty * vdi::kXTileH + l / vdi::kXTileW;
        if (px >= W || py >= H) continue;
        g_rec = &rec[l];
        g_it = 0;
        vdi::Counters c = {0, 0};
        (void)vdi::trace_exact<VDI_F32, VDI_SEARCH_WINDOW, true, false>(L.v.dev, L.f, L.v.dev.gz, px, py, c);
        g_rec = nullptr;
    }
    req.clear();
    size_t pos[64] = {0};
    int last_it = 0;
    for (int l = 0; l < 64; ++l)
        if (!rec[l].empty()) last_it = std::max(last_it, rec[l].back().it);
    std::vector<std::pair<uint64_t, int>> group;
    for (int it = 0; it <= last_it; ++it) {
        size_t end[64];
        size_t kmax = 0;
        for (int l = 0; l < 64; ++l) {
            size_t q = pos[l];
            while (q < rec[l].size() && rec[l][q].it == it) ++q;
            end[l] = q;
            kmax = std::max(kmax, q - pos[l]);
        }
        for (size_t k = 0; k < kmax; ++k) {
            // One request per line, in the order of the first lane that
            // names it (an order that does not depend on where the buffers lie).
            group.clear();
            for (int l = 0; l < 64; ++l)
                if (pos[l] + k < end[l]) {
                    const std::pair<uint64_t, int> r = {rec[l][pos[l] + k].line, rec[l][pos[l] + k].stream};
                    if (std::find(group.begin(), group.end(), r) == group.end()) group.push_back(r);
                }
            req.insert(req.end(), group.begin(), group.end());
        }
        for (int l = 0; l < 64; ++l) pos[l] = end[l];
    }
}

}  // namespace

__host__ __device__ void reuse_note(const void *p, int stream)
{
#if !defined(__HIP_DEVICE_COMPILE__)
    if (g_rec) g_rec->push_back({g_it, stream, (uint64_t)(uintptr_t)p >> 7});
#else
    (void)p;
    (void)stream;
#endif
}
__host__ __device__ void reuse_step()
{
#if !defined(__HIP_DEVICE_COMPILE__)
    ++g_it;
#endif
}

extern "C" {

// Requests of exact tile (tx, ty) in issue order, as line numbers (address /
// 128) and streams.  Writes at most cap entries; returns the number of
// requests, or a negative error code.
long long reuse_tile_trace(const vdi_desc *d, const uint32_t *grid, const vdi_camera *cam, int W, int H, int tx,
                           int ty, uint64_t *lines, int32_t *streams, long long cap)
{
    Layout L;
    const int rc = setup(d, grid, cam, W, H, L);
    if (rc) return -rc;
    std::vector<std::pair<uint64_t, int>> req;
    tile_requests(L, W, H, tx, ty, req);
    for (long long i = 0; i < (long long)req.size() && i < cap; ++i) {
        lines[i] = req[i].first;
        streams[i] = req[i].second;
    }
    return (long long)req.size();
}

// Over the exact tiles of every row_step-th tile row: per stream s (0 counts,
// 1 occupancy bits, 2 depth pairs, 3 colours), stats[s * (2 + ncaps)] =
// requests, [+1] first requests of a line (cold), [+2 + c] hits in an LRU
// cache of caps[c] lines.
int reuse_exact(const vdi_desc *d, const uint32_t *grid, const vdi_camera *cam, int W, int H, int row_step,
                const int32_t *caps, int ncaps, double *stats)
{
    Layout L;
    const int rc = setup(d, grid, cam, W, H, L);
    if (rc) return rc;
    const int per = 2 + ncaps;
    const int tiles_x = (W + vdi::kXTileW - 1) / vdi::kXTileW, tiles_y = (H + vdi::kXTileH - 1) / vdi::kXTileH;
    std::vector<double> total(4 * per, 0.0);
#pragma omp parallel
    {
        std::vector<double> st(4 * per, 0.0);
        std::vector<std::pair<uint64_t, int>> req;
        std::unordered_map<uint64_t, size_t> last;
        Fenwick fw;
#pragma omp for schedule(dynamic, 4)
        for (int tile = 0; tile < tiles_x * tiles_y; ++tile) {
            const int ty = tile / tiles_x, tx = tile % tiles_x;
            if (ty % row_step) continue;
            tile_requests(L, W, H, tx, ty, req);
            fw.init(req.size());
            last.clear();
            for (size_t now = 0; now < req.size(); ++now) {
                double *S = &st[req[now].second * per];
                S[0] += 1;
                auto it = last.find(req[now].first);
                if (it == last.end()) {
                    S[1] += 1;
                } else {
                    // Distinct other lines requested since this line's previous request.
                    const int dist = fw.prefix(now) - fw.prefix(it->second + 1);
                    for (int c = 0; c < ncaps; ++c)
                        if (dist < caps[c]) S[2 + c] += 1;
                    fw.add(it->second, -1);
                }
                fw.add(now, 1);
                last[req[now].first] = now;
            }
        }
#pragma omp critical
        for (size_t i = 0; i < total.size(); ++i) total[i] += st[i];
    }
    for (size_t i = 0; i < total.size(); ++i) stats[i] = total[i];
    return VDI_OK;
}

}  // extern "C"
