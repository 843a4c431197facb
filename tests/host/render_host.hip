// Host build of the renderer's per-ray code: the same __host__ __device__
// functions the kernels run (ray set-up, list walk, searches, Eq. 2,
// compositing, preview sampling), one pixel at a time, with the VDI laid out
// in device order (bricks) in host memory.  Preview rays may be split into
// `parts` blocks of cells, combined in the order the kernel's lane shuffles
// use (pairs, then pairs of pairs).
#include "vdi_kernels.hip"
#include "vdi_api.hip"

#include <vector>

extern "C" int host_render(const vdi_desc *d, const uint32_t *grid, const vdi_camera *cam, int W, int H, int preview,
                           int search, int ess, float DR, int parts, float *out)
{
    vdi::VdiSet v;
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
    std::vector<float2> dep(elems, make_float2(NAN, NAN));
    std::vector<float4> col(elems, make_float4(NAN, NAN, NAN, NAN));
    for (int j = 0; j < D.NS; ++j)
        for (uint64_t li = 0; li < D.plane; ++li) {
            const uint64_t o = vdi::list_base(li, D.NS, D.WO) + (uint64_t)j * D.sstride;
            dep[o] = reinterpret_cast<const float2 *>(d->depth)[(uint64_t)j * D.plane + li];
            col[o] = static_cast<const float4 *>(d->rgba)[(uint64_t)j * D.plane + li];
        }
    D.count = d->count;
    D.depth = dep.data();
    D.rgba = col.data();
    D.grid = grid;
    const uint32_t ncells = (uint32_t)d->grid_nz * ((d->height + d->grid_k - 1) / d->grid_k) * ((d->width + d->grid_k - 1) / d->grid_k);
    std::vector<uint32_t> bits((ncells + 31) / 32, 0u);
    for (uint32_t c = 0; c < ncells; ++c)
        if (grid[c] != 0u) bits[c / 32] |= 1u << (c % 32);
    D.gbits = bits.data();
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
    vdi::Frame f;
    rc = build_frame(v, *cam, W, H, (double)W / H, f);
    if (rc) return rc;
    f.ess = ess;
    f.search = search;
    f.DR = DR;
    if (parts <= 0) parts = f.parts;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            float4 o;
            if (preview) {
                vdi::Accum a[8];
                for (int q = 0; q < parts; ++q) a[q] = vdi::trace_preview<VDI_F32>(D, f, d->grid_z, px, py, q, parts);
                for (int n = parts; n > 1; n /= 2)
                    for (int i = 0; i < n / 2; ++i) a[i] = vdi::over(a[2 * i], a[2 * i + 1]);
                o = vdi::to_rgba(a[0]);
            } else {
                vdi::Counters cnt = {0, 0};
                if (ess) {
                    switch (search) {
                    case VDI_SEARCH_WINDOW: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_WINDOW, true, false>(D, f, d->grid_z, px, py, cnt); break;
                    case VDI_SEARCH_BINARY: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_BINARY, true, false>(D, f, d->grid_z, px, py, cnt); break;
                    case VDI_SEARCH_LINEAR: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_LINEAR, true, false>(D, f, d->grid_z, px, py, cnt); break;
                    default: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_SEEDED, true, false>(D, f, d->grid_z, px, py, cnt);
                    }
                } else {
                    switch (search) {
                    case VDI_SEARCH_WINDOW: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_WINDOW, false, false>(D, f, d->grid_z, px, py, cnt); break;
                    case VDI_SEARCH_BINARY: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_BINARY, false, false>(D, f, d->grid_z, px, py, cnt); break;
                    case VDI_SEARCH_LINEAR: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_LINEAR, false, false>(D, f, d->grid_z, px, py, cnt); break;
                    default: o = vdi::trace_exact<VDI_F32, VDI_SEARCH_SEEDED, false, false>(D, f, d->grid_z, px, py, cnt);
                    }
                }
            }
            float *p = out + 4 * ((size_t)py * W + px);
            p[0] = o.x;
            p[1] = o.y;
            p[2] = o.z;
            p[3] = o.w;
        }
    return 0;
}
