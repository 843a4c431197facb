// Per-ray device code of libvdi, shared by the one-shot kernels
// (vdi_kernels.hip) and the persistent serving kernel (vdi_serve.hip):
// ray set-up and clipping, list-grid walking, first-supersegment search,
// opacity correction and compositing, preview sampling.  Every function is
// host-callable too, so a ray can be stepped through on the CPU.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "vdi_internal.h"

// Every global load of the per-ray code goes through VDI_LOAD(pointer,
// stream), with stream 0 for counts, 1 for occupancy bits, 2 for depth pairs
// and 3 for colours, and every main-loop iteration of an exact ray calls
// VDI_STEP().  In the library they are a plain load and nothing; a host build
// of the same code may define them to record what each ray reads, in order
// (tests/host/reuse_host.hip).
#ifndef VDI_LOAD
#define VDI_LOAD(p, stream) (*(p))
#endif
#ifndef VDI_STEP
#define VDI_STEP()
#endif

namespace vdi {

// Per-ray functions are host-callable too, so the traversal can be stepped
// through on the CPU with the same code.
#define VDI_HD __host__ __device__
// The per-ray walkers are inlined into every kernel: called out of line, a
// walker takes the frame and VDI constants through a pointer in vector
// registers and a stack frame of over 200 bytes per lane (the batched
// kernels lost half their speed that way once the persistent kernel added
// call sites and the inliner stopped inlining them).
#define VDI_HDI __host__ __device__ __forceinline__

// Arithmetic helpers: native gfx950 instructions on the device (overloaded
// on the compilation target), the plain formulas on the host.  The FP64
// reciprocal is refined by two Newton steps to full precision; the FP32 ones
// are within an ulp or two, far below the 1e-4 the renders are held to.
__device__ inline double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__host__ inline double rcp64(double x) { return 1.0 / x; }
__device__ inline float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }
__host__ inline float rcp32(float x) { return 1.0f / x; }
__device__ inline float rsqrt32(float x) { return __builtin_amdgcn_rsqf(x); }
__host__ inline float rsqrt32(float x) { return 1.0f / sqrtf(x); }
__device__ inline float exp2_32(float x) { return __builtin_amdgcn_exp2f(x); }
__host__ inline float exp2_32(float x) { return exp2f(x); }
__device__ inline float log2_32(float x) { return __builtin_amdgcn_logf(x); }
__host__ inline float log2_32(float x) { return log2f(x); }

constexpr int kBlock = kTileW * kTileH;

VDI_HD inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Tile of workgroup `bid`.  Workgroups are dealt to the 8 XCDs round-robin
// and each XCD has its own L2.  Tile rows are grouped into bands of
// `band_rows` tile rows (8 pixel rows); band b belongs to XCD b % 8, so each
// XCD renders whole bands (horizontal neighbours, whose rays cross the same
// V_O lists, share an L2) while the bands of every XCD are spread over the
// image (the work is balanced).  The map is a bijection from
// [0, tiles_x * tiles_y) onto itself.
#ifndef VDI_BAND_ROWS
#define VDI_BAND_ROWS 8
#endif
constexpr int kBandRows = VDI_BAND_ROWS / kTileH > 0 ? VDI_BAND_ROWS / kTileH : 1;     // rows of 64 x 1 tiles
constexpr int kXBandRows = VDI_BAND_ROWS / kXTileH > 0 ? VDI_BAND_ROWS / kXTileH : 1;  // rows of exact tiles

VDI_HD inline int xcd_tile(int bid, int tiles_x, int tiles_y, int band_rows = kBandRows)
{
    const int total = tiles_x * tiles_y;
    const int x = bid % kXcds, k = bid / kXcds;
    // Position of this block in the XCD-major order of all blocks.
    const int pos = x * (total / kXcds) + min(x, total % kXcds) + k;
    // Bands in XCD-group order: group g holds bands g, g + 8, g + 16, ...
    const int nb = (tiles_y + band_rows - 1) / band_rows;
    const int last_rows = tiles_y - (nb - 1) * band_rows;
    const int band_tiles = band_rows * tiles_x;
    int start = 0;
    for (int g = 0; g < kXcds; ++g) {
        const int nbg = g < nb ? (nb - 1 - g) / kXcds + 1 : 0;
        int size = nbg * band_tiles;
        if (nbg > 0 && (nb - 1) % kXcds == g) size -= (band_rows - last_rows) * tiles_x;
        if (pos < start + size) {
            const int local = pos - start;
            const int b = g + kXcds * (local / band_tiles);
            return b * band_tiles + local % band_tiles;
        }
        start += size;
    }
    return pos;  // not reached
}

// ---------------------------------------------------------------------------
// Colour planes
// ---------------------------------------------------------------------------
// Colour of slot idx.  FMT is the storage format, or kFmtRuntime to read it
// from `fmt` (one code path for kernels that serve VDIs of any format).
constexpr int kFmtRuntime = -1;

template <int FMT>
VDI_HD inline float4 load_rgba(const void *base, uint64_t idx, int fmt = FMT)
{
    const int f = FMT >= 0 ? FMT : fmt;
    if (FMT == VDI_F32 || (FMT < 0 && f == VDI_F32)) return VDI_LOAD(reinterpret_cast<const float4 *>(base) + idx, 3);
    const uint2 u = VDI_LOAD(reinterpret_cast<const uint2 *>(base) + idx, 3);
    if (f == VDI_F16) {
        const __half2 rg = *reinterpret_cast<const __half2 *>(&u.x);
        const __half2 ba = *reinterpret_cast<const __half2 *>(&u.y);
        const float2 a = __half22float2(rg), b = __half22float2(ba);
        return make_float4(a.x, a.y, b.x, b.y);
    }
    return make_float4(__builtin_bit_cast(float, u.x << 16), __builtin_bit_cast(float, u.x & 0xffff0000u),
                       __builtin_bit_cast(float, u.y << 16), __builtin_bit_cast(float, u.y & 0xffff0000u));
}

// ---------------------------------------------------------------------------
// Rays
// ---------------------------------------------------------------------------
struct Ray {
    double Xp, Yp, Zp;  // d/dt of (X, Y, Z) in V_O's frame; Z is V_O view depth
    double t0, t1;      // clipped parameter range (world distance from eye_N)
};

// Keep t with a + b t >= 0.
VDI_HD inline bool clip(double a, double b, double &lo, double &hi)
{
    if (b == 0.0) return a >= 0.0;
    const double t = -a / b;
    if (b > 0.0)
        lo = fmax(lo, t);
    else
        hi = fmin(hi, t);
    return true;
}

// Ray through NDC (xc, yc) of V_N, clipped to V_N's near plane, the AABB and
// V_O's frustum (Section 4.1: marching starts and ends where the ray meets
// the generating viewport and the volume's bounding box).
VDI_HD inline bool ray_setup(const Frame &F, double xc, double yc, Ray &r)
{
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = F.FN[a] + xc * F.tx_n * F.RN[a] + yc * F.ty_n * F.UN[a];
    const double inv = 1.0 / sqrt(dot3(d, d));
    for (int a = 0; a < 3; ++a) d[a] *= inv;
    r.Xp = dot3(F.RO, d) * F.sx_o;
    r.Yp = dot3(F.UO, d) * F.sy_o;
    r.Zp = dot3(F.FO, d);
    double lo = 0.0, hi = __builtin_huge_val();
    bool ok = clip(-F.near_n, dot3(F.FN, d), lo, hi);
    for (int a = 0; a < 3; ++a) {
        ok = ok && clip(F.eyeN[a] - F.bmin[a], d[a], lo, hi);
        ok = ok && clip(F.bmax[a] - F.eyeN[a], -d[a], lo, hi);
    }
    ok = ok && clip(F.Z0 - F.near_o, r.Zp, lo, hi);
    ok = ok && clip(F.Z0 - F.X0, r.Zp - r.Xp, lo, hi);
    ok = ok && clip(F.Z0 + F.X0, r.Zp + r.Xp, lo, hi);
    ok = ok && clip(F.Z0 - F.Y0, r.Zp - r.Yp, lo, hi);
    ok = ok && clip(F.Z0 + F.Y0, r.Zp + r.Yp, lo, hi);
    r.t0 = lo;
    r.t1 = hi;
    return ok && hi > lo;
}

// Parameter where the ray meets NDC line coord = -1 + 2 m / n (P = X or Y),
// or +inf if it never does.  coord(t) = P(t) / Z(t) is monotone where Z > 0
// but its asymptote is the ray's vanishing point: a line beyond it has its
// only root on the branch behind V_O (Z < 0), which is not a crossing.
VDI_HD inline double line_t(int m, double two_over_n, double P0, double Pp, double Z0, double Zp)
{
    const double c = fma((double)m, two_over_n, -1.0);
    const double den = Pp - c * Zp;
    if (den == 0.0) return __builtin_huge_val();
    const double t = (c * Z0 - P0) * rcp64(den);
    return Z0 + t * Zp > 0.0 ? t : __builtin_huge_val();
}

// Cell index of an NDC coordinate; a point exactly on a line belongs to the
// cell the ray is moving into.
VDI_HD inline int cell_of(double ndc, int n, int dir)
{
    const double f = (ndc + 1.0) * n / 2.0;
    const double fl = floor(f);
    int i = (int)fl;
    if (f == fl && dir < 0) i -= 1;
    return min(max(i, 0), n - 1);
}

// cos of the angle between list (ix, iy)'s generating ray and V_O's axis.
VDI_HD inline float list_cos(const DevVDI &V, int ix, int iy)
{
    const float x = (-1.0f + (2.0f * ix + 1.0f) / V.WO) * V.tx_o;
    const float y = (-1.0f + (2.0f * iy + 1.0f) / V.HO) * V.ty_o;
    return rsqrt32(1.0f + x * x + y * y);
}

// Depth slice holding depth z for a ray moving towards larger (fwd) or smaller z.
VDI_HD inline int slice_of(const float *gz, int gnz, double z, bool fwd)
{
    int lo = 0, hi = gnz - 1;  // answer in [0, gnz-1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const double b = gz[mid];
        if (fwd ? (b <= z) : (b < z))
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// First-supersegment search (Section 4.2, supplement Alg. S2)
// ---------------------------------------------------------------------------
// Smallest j in [0, n) with b_j > z (n if none).  Back depths increase with j
// because supersegments are sorted and disjoint.  Slot j of the list is
// dep[base + j * stride].
template <int SEARCH>
VDI_HD inline int first_back_above(const float2 *__restrict__ dep, uint64_t stride, uint64_t base, int n,
                                                double z, int p)
{
    if constexpr (SEARCH == VDI_SEARCH_LINEAR) {
        int j = 0;
        while (j < n && (double)VDI_LOAD(dep + ((uint64_t)j * stride + base), 2).y <= z) ++j;
        return j;
    }
    int lo = 0, hi = n;
    if constexpr (SEARCH == VDI_SEARCH_SEEDED) {
        if (p >= 0 && p < n) {
            // Both candidate back depths are fetched before either is compared.
            const float b1 = VDI_LOAD(dep + ((uint64_t)p * stride + base), 2).y;
            const float b0 = p > 0 ? VDI_LOAD(dep + ((uint64_t)(p - 1) * stride + base), 2).y : -__builtin_huge_valf();
            if ((double)b0 > z)
                hi = p - 1;  // the answer is at most p-1
            else if ((double)b1 > z)
                return p;    // the seed itself
            else
                lo = p + 1;
        }
    }
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((double)VDI_LOAD(dep + ((uint64_t)mid * stride + base), 2).y > z)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Largest j in [0, n) with f_j < z (-1 if none): the first supersegment met by
// a ray travelling towards smaller depth.
template <int SEARCH>
VDI_HD inline int last_front_below(const float2 *__restrict__ dep, uint64_t stride, uint64_t base, int n,
                                                double z, int p)
{
    if constexpr (SEARCH == VDI_SEARCH_LINEAR) {
        int j = n - 1;
        while (j >= 0 && (double)VDI_LOAD(dep + ((uint64_t)j * stride + base), 2).x >= z) --j;
        return j;
    }
    int lo = 0, hi = n;  // search the first j with f_j >= z
    if constexpr (SEARCH == VDI_SEARCH_SEEDED) {
        if (p >= 0 && p < n) {
            const float f1 = VDI_LOAD(dep + ((uint64_t)p * stride + base), 2).x;
            const float f2 = p + 1 < n ? VDI_LOAD(dep + ((uint64_t)(p + 1) * stride + base), 2).x : __builtin_huge_valf();
            if ((double)f1 >= z)
                hi = p;
            else if ((double)f2 >= z)
                return p;
            else
                lo = p + 2;
        }
    }
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((double)VDI_LOAD(dep + ((uint64_t)mid * stride + base), 2).x >= z)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo - 1;
}

// Window search (the default).  A ray's first supersegment in the next list
// is usually within a few slots of the one used in the previous list: on the
// 1080p workload the answer lies in [p-3, p+4] for 93% of list visits, and at
// p itself for only a third.  The back (forward rays) or front (backward rays)
// depths of kWin slots around the seed are therefore loaded together, in one
// round trip; being sorted, the number of them on the near side of z is the
// answer's offset in the window.  An answer outside the window is looked for
// in the windows next to it, and only then in the rest of the list (below).
// Every load is clamped into the list.  kWin = 4 with up to two further
// windows: a miss costs a round trip more, a hit fewer lines than a window
// of 8 (1080p benchmark step, 2 x 2 bricks, images bit-identical: 4 + 2
// further windows 8.89-8.92 ms; 4 + 3 8.93-8.96; 5 + 2 8.96; 3 + 3 8.99;
// 6 + 1 9.00-9.02; 8 + 1 9.35-9.42; 12 + 1 11.50).
#ifndef VDI_WIN
#define VDI_WIN 4
#endif
constexpr int kWin = VDI_WIN;

// For a float x and a double z: (double)x <= z exactly when x <= below(z),
// and (double)x < z exactly when x < above(z), where below(z) is the largest
// float <= z and above(z) the smallest float >= z.  The searches compare
// float depths against these bounds, with the same outcome as comparing in
// double precision.
VDI_HD inline float float_below(double z)
{
    const float f = (float)z;
    return (double)f > z ? nextafterf(f, -__builtin_huge_valf()) : f;
}
VDI_HD inline float float_above(double z)
{
    const float f = (float)z;
    return (double)f < z ? nextafterf(f, __builtin_huge_valf()) : f;
}

// A ray moving to larger depth usually finds its answer at or after the
// previous list's index p, one moving to smaller depth at or before it.
VDI_HD inline int win_start_fwd(int p) { return p - (kWin / 2 - 1); }
VDI_HD inline int win_start_bwd(int p) { return p - kWin / 2; }

// The first slot J of a list at which `below` turns false (below(slot j) is
// true exactly for j < J: sorted keys), searched from a window of kWin slots
// at `start`, moved inside the list.  Every round trip loads up to kWin keys
// from one base address and counts how many lie below.  When J lies outside
// the window, the rest is searched either by bisection (SPREAD = false) or
// (SPREAD = true) by kWin slots evenly spaced over what remains, which cuts
// it into kWin + 1 parts, then a window over the part holding J: at most
// three round trips for lists of up to about 80 slots, where bisection takes
// one per halving, but eight more lines read.  Preview samples, whose
// wavefronts wait on their slowest lane's search, gain from spreading (the
// 1080p D_I = 2 and 4 sweeps: 3.83 -> 3.70 ms, 1.81 -> 1.74 ms); exact rays,
// bound more by cache traffic, lose (9.75 -> 9.89 ms) and bisect.
// With `pair` (PICK = k: the pair of window slot J + k, k = 0 or -1): when
// the answer lies inside the first window, *pair gets that slot's depth
// pair from the window's registers and *have is set.  The exact walker takes
// its first supersegment's (f, b) from there instead of loading it again
// after the search: the window's lines hold both depths, the registers cost
// no occupancy, and the list's first piece waits one round trip less (1080p
// sweep 9.88 -> 9.80 ms, images bit-identical; VDI_WIN_PAIR=0 reloads it).
// An answer outside the first window is looked for next in VDI_WIN2 (without
// SPREAD) or VDI_WIN2_SPREAD (with it) further windows, each the kWin slots
// next to what is left on the answer's side, and only then bisected or
// spread over (the pair, if asked for, comes from the window that holds the
// answer).  Most answers a window misses lie just past its end, and a
// wavefront waits for the slowest lane's search: a round trip more for the
// lanes that missed instead of a bisection of up to six, or of up to three
// spread round trips.  With 8-slot windows, 1080p, images bit-identical:
// exact sweep 9.85 -> 9.61 ms with one further window (two: 10.15 ms);
// preview sweeps D_I = 2 3.78 -> 3.55 ms, D_I = 4 1.82 -> 1.75 ms (two:
// 3.57, 1.77 ms); benchmark step 9.70 -> 9.51 ms with the exact one, 9.51
// -> 9.35 ms with the preview's as well.  Smaller windows want more of them
// (kWin, above).  Zero restores the search straight after the first window.
#ifndef VDI_WIN_PAIR
#define VDI_WIN_PAIR 1
#endif
#ifndef VDI_WIN2
#define VDI_WIN2 2
#endif
#ifndef VDI_WIN2_SPREAD
#define VDI_WIN2_SPREAD 2
#endif
template <bool SPREAD, int PICK = 0, typename Below>
VDI_HD inline int window_search(const float2 *__restrict__ dep, uint64_t stride, uint64_t base, int n, int start,
                                Below below, float2 *pair = nullptr, bool *have = nullptr)
{
    int lo = 0, hi = n;  // J in [lo, hi]
    if (n >= kWin) {
        const int w0 = max(0, min(start, n - kWin));
        const float2 *w = dep + base + (uint64_t)w0 * stride;
        float2 b[kWin];
#pragma unroll
        for (int k = 0; k < kWin; ++k) b[k] = VDI_LOAD(w + k * stride, 2);
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < kWin; ++k) cnt += below(b[k]) ? 1 : 0;
        if (cnt == 0)
            hi = w0;
        else if (cnt == kWin)
            lo = w0 + kWin;
        else
            lo = hi = w0 + cnt;
        if (pair) {
            const int at = cnt + PICK;  // window slot of the answer
            float2 d = b[0];
#pragma unroll
            for (int k = 1; k < kWin; ++k) d = at == k ? b[k] : d;
            *pair = d;
            *have = cnt > 0 && cnt < kWin;
        }
        if constexpr ((SPREAD ? VDI_WIN2_SPREAD : VDI_WIN2) != 0) {
            const bool up = cnt == kWin;
#pragma unroll
            for (int e = 0; e < (SPREAD ? VDI_WIN2_SPREAD : VDI_WIN2); ++e) {
                if (lo >= hi) break;
                // One more window next to the bracket, on the answer's side.
                const int w1 = up ? min(lo, n - kWin) : max(0, hi - kWin);
                const float2 *v = dep + base + (uint64_t)w1 * stride;
                float2 c[kWin];
#pragma unroll
                for (int k = 0; k < kWin; ++k) c[k] = VDI_LOAD(v + k * stride, 2);
                int c2 = 0;
#pragma unroll
                for (int k = 0; k < kWin; ++k) c2 += below(c[k]) ? 1 : 0;
                if (c2 == 0)
                    hi = min(hi, w1);
                else if (c2 == kWin)
                    lo = max(lo, w1 + kWin);
                else
                    lo = hi = w1 + c2;
                if (pair && c2 > 0 && c2 < kWin) {
                    const int at = c2 + PICK;
                    float2 d = c[0];
#pragma unroll
                    for (int k = 1; k < kWin; ++k) d = at == k ? c[k] : d;
                    *pair = d;
                    *have = true;
                }
            }
        }
    }
    if constexpr (!SPREAD) {
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (below(VDI_LOAD(dep + base + (uint64_t)mid * stride, 2)))
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    }
    while (hi - lo > kWin) {
        // Slots lo + floor((k + 1)(hi - lo) / (kWin + 1)): distinct, inside [lo, hi).
        const int span = hi - lo;
        float2 b[kWin];
#pragma unroll
        for (int k = 0; k < kWin; ++k) b[k] = VDI_LOAD(dep + base + (uint64_t)(lo + ((k + 1) * span) / (kWin + 1)) * stride, 2);
        int m = 0;
#pragma unroll
        for (int k = 0; k < kWin; ++k) m += below(b[k]) ? 1 : 0;
        const int nlo = m > 0 ? lo + (m * span) / (kWin + 1) + 1 : lo;
        const int nhi = m < kWin ? lo + ((m + 1) * span) / (kWin + 1) : hi;
        lo = nlo;
        hi = nhi;
    }
    if (hi > lo) {
        // At most kWin candidate slots before hi: J is lo plus those below.
        const int len = hi - lo;
        const float2 *w = dep + base + (uint64_t)lo * stride;
        float2 b[kWin];
#pragma unroll
        for (int k = 0; k < kWin; ++k) b[k] = VDI_LOAD(w + (uint64_t)min(k, len - 1) * stride, 2);
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < kWin; ++k) cnt += (k < len && below(b[k])) ? 1 : 0;
        lo += cnt;
    }
    return lo;
}

// Smallest j in [0, n) with b_j > z (n if none); the window starts at slot
// `start`.
template <bool SPREAD = false>
VDI_HD inline int first_back_above_win(const float2 *__restrict__ dep, uint64_t stride, uint64_t base, int n, double z,
                                       int start, float2 *pair = nullptr, bool *have = nullptr)
{
    const float zb = float_below(z);  // b > z  <=>  b > zb
    return window_search<SPREAD, 0>(dep, stride, base, n, start, [zb](float2 d) { return d.y <= zb; }, pair, have);
}

// Largest j in [0, n) with f_j < z (-1 if none), window from `start`: one
// less than the first j with f_j >= z, found as above.
template <bool SPREAD = false>
VDI_HD inline int last_front_below_win(const float2 *__restrict__ dep, uint64_t stride, uint64_t base, int n, double z,
                                       int start, float2 *pair = nullptr, bool *have = nullptr)
{
    const float za = float_above(z);  // f < z  <=>  f < za
    return window_search<SPREAD, -1>(dep, stride, base, n, start, [za](float2 d) { return d.x < za; }, pair, have) - 1;
}

// ---------------------------------------------------------------------------
// Compositing
// ---------------------------------------------------------------------------
struct Accum {
    float r, g, b, T;
};

// Eq. 2 with exponent l = (world length in S) / (world length of the
// generating ray in S), then front-to-back "over".
VDI_HD inline void composite(Accum &A, float4 c, float l)
{
    const float at = c.w >= 1.0f ? 1.0f : 1.0f - exp2_32(l * log2_32(1.0f - c.w));
    const float w = A.T * at;
    A.r = fmaf(w, c.x, A.r);
    A.g = fmaf(w, c.y, A.g);
    A.b = fmaf(w, c.z, A.b);
    A.T *= 1.0f - at;
}

struct Counters {
    int32_t lists, pieces;
};

// With the window search, fetch the found slot's colour together with its
// depth pair (one round trip less when the ray composites it; a wasted load
// when the ray only crosses a gap of the list).
#ifndef VDI_WIN_COLOUR
#define VDI_WIN_COLOUR 0
#endif
constexpr bool kWinColour = VDI_WIN_COLOUR != 0;

// Element distance between slots j and j + 1 of a list: a compile-time
// constant with bricks, so slot addresses need no multiply.
VDI_HD inline uint64_t slot_stride(const DevVDI &V)
{
    if constexpr (kBrick != 0) return (uint64_t)kBrick;
    return V.sstride;
}

// Depth pair of slot j of the list whose storage starts at lb (list_base).
VDI_HD inline float2 depth_at(const DevVDI &V, int j, uint64_t lb) { return VDI_LOAD(V.depth + (uint64_t)j * slot_stride(V) + lb, 2); }

// Composite the part of list (ix, iy) that a ray with dz/dt = Zp crosses
// between parameters ta and tb (Sections 4.2, Eq. 2).  n is the list's count
// (fetched one step ahead by the caller).  The first supersegment comes from
// the configured search, seeded by p, the index used in the previous list
// (supplement Alg. S2: both candidate depth pairs are loaded before either is
// compared, and the one that hits is reused); the next ones by adjacency,
// each colour load overlapping the following depth load.  p is updated;
// returns true once the ray has terminated.
template <int FMT, int SEARCH, bool COUNT>
VDI_HDI bool do_list(const DevVDI &V, const Frame &F, int ix, int iy, int n, double ta, double tb, double Z0,
                    double Zp, double invZp, Accum &A, int &p, Counters &cnt)
{
    const uint64_t li = (uint64_t)iy * V.WO + ix;
    if constexpr (COUNT) {
        F.touched_lists[li] = 1;
        ++cnt.lists;
    }
    if (n == 0) return false;
    const double za = Z0 + ta * Zp, zb = Z0 + tb * Zp;
    const float cth = list_cos(V, ix, iy);
    const float2 *__restrict__ dep = V.depth;
    const uint64_t stride = slot_stride(V), lb = list_base_xy(ix, iy, V.NS, V.WO);
    auto piece = [&](int j, float2 d, float4 c, double zl, double zh, double inv) -> bool {
        composite(A, c, (float)((zh - zl) * inv) * cth * rcp32(d.y - d.x));
        if constexpr (COUNT) {
            F.touched_slots[(uint64_t)j * V.plane + li] = 1;
            ++cnt.pieces;
        }
        return A.T <= kTTerm;
    };
    if (Zp > kFlatZ) {
        const double inv = invZp;
        int j;
        bool have = false;
        float2 d = make_float2(0.0f, 0.0f);
        if constexpr (SEARCH == VDI_SEARCH_WINDOW) {
            if constexpr (VDI_WIN_PAIR != 0)
                j = first_back_above_win(dep, stride, lb, n, za, win_start_fwd(p), &d, &have);
            else
                j = first_back_above_win(dep, stride, lb, n, za, win_start_fwd(p));
        } else if (SEARCH == VDI_SEARCH_SEEDED && p >= 0 && p < n) {
            const float2 dp = depth_at(V, p, lb);
            const float2 dq = p > 0 ? depth_at(V, p - 1, lb) : make_float2(-__builtin_huge_valf(), -__builtin_huge_valf());
            if ((double)dq.y > za) {
                j = first_back_above<VDI_SEARCH_BINARY>(dep, stride, lb, p - 1, za, -1);
                if (j == p - 1) {
                    d = dq;
                    have = true;
                }
            } else if ((double)dp.y > za) {
                j = p;
                d = dp;
                have = true;
            } else {
                j = p + 1 + first_back_above<VDI_SEARCH_BINARY>(dep, stride, lb + (uint64_t)(p + 1) * stride, n - p - 1,
                                                                 za, -1);
            }
        } else {
            j = first_back_above<SEARCH>(dep, stride, lb, n, za, -1);
        }
        int last = -1;
        float4 c0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        bool have_c = false;
        if (j < n && !have) {
            d = depth_at(V, j, lb);
            if constexpr (kWinColour && SEARCH == VDI_SEARCH_WINDOW) {
                c0 = load_rgba<FMT>(V.rgba, (uint64_t)j * stride + lb, V.fmt);
                have_c = true;
            }
        }
        while (j < n) {
            if ((double)d.x >= zb) break;
            const float4 c = have_c ? c0 : load_rgba<FMT>(V.rgba, (uint64_t)j * stride + lb, V.fmt);
            have_c = false;
            const bool more = (double)d.y < zb && j + 1 < n;
            const float2 dn = more ? depth_at(V, j + 1, lb) : d;
            const double zl = fmax(za, (double)d.x), zh = fmin(zb, (double)d.y);
            if (zh > zl) {
                last = j;
                if (piece(j, d, c, zl, zh, inv)) {
                    p = last;
                    return true;
                }
            }
            if (!more) break;
            d = dn;
            ++j;
        }
        p = last >= 0 ? last : min(j, n - 1);
    } else if (Zp < -kFlatZ) {
        // Travelling towards smaller depth: mirror image of the above.
        const double inv = -invZp;
        int j;
        bool have = false;
        float2 d = make_float2(0.0f, 0.0f);
        if constexpr (SEARCH == VDI_SEARCH_WINDOW) {
            if constexpr (VDI_WIN_PAIR != 0)
                j = last_front_below_win(dep, stride, lb, n, za, win_start_bwd(p), &d, &have);
            else
                j = last_front_below_win(dep, stride, lb, n, za, win_start_bwd(p));
        } else if (SEARCH == VDI_SEARCH_SEEDED && p >= 0 && p < n) {
            const float2 dp = depth_at(V, p, lb);
            const float2 dq = p + 1 < n ? depth_at(V, p + 1, lb) : make_float2(__builtin_huge_valf(), __builtin_huge_valf());
            if ((double)dp.x >= za) {
                j = last_front_below<VDI_SEARCH_BINARY>(dep, stride, lb, p, za, -1);
            } else if ((double)dq.x >= za) {
                j = p;
                d = dp;
                have = true;
            } else {
                j = p + 2 + last_front_below<VDI_SEARCH_BINARY>(dep, stride, lb + (uint64_t)(p + 2) * stride, n - p - 2,
                                                                 za, -1);
            }
        } else {
            j = last_front_below<SEARCH>(dep, stride, lb, n, za, -1);
        }
        int last = -1;
        float4 c0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        bool have_c = false;
        if (j >= 0 && !have) {
            d = depth_at(V, j, lb);
            if constexpr (kWinColour && SEARCH == VDI_SEARCH_WINDOW) {
                c0 = load_rgba<FMT>(V.rgba, (uint64_t)j * stride + lb, V.fmt);
                have_c = true;
            }
        }
        while (j >= 0) {
            if ((double)d.y <= zb) break;
            const float4 c = have_c ? c0 : load_rgba<FMT>(V.rgba, (uint64_t)j * stride + lb, V.fmt);
            have_c = false;
            const bool more = (double)d.x > zb && j > 0;
            const float2 dn = more ? depth_at(V, j - 1, lb) : d;
            const double zl = fmax(zb, (double)d.x), zh = fmin(za, (double)d.y);
            if (zh > zl) {
                last = j;
                if (piece(j, d, c, zl, zh, inv)) {
                    p = last;
                    return true;
                }
            }
            if (!more) break;
            d = dn;
            --j;
        }
        p = last >= 0 ? last : max(j, 0);
    } else {
        // Constant depth: the supersegment holding za covers the whole piece.
        for (int j = 0; j < n; ++j) {
            const float2 d = depth_at(V, j, lb);
            if ((double)d.x <= za && za < (double)d.y) {
                const float4 c = load_rgba<FMT>(V.rgba, (uint64_t)j * stride + lb, V.fmt);
                p = j;
                composite(A, c, (float)(tb - ta) * cth * rcp32(d.y - d.x));
                if constexpr (COUNT) {
                    F.touched_slots[(uint64_t)j * V.plane + li] = 1;
                    ++cnt.pieces;
                }
                return A.T <= kTTerm;
            }
        }
    }
    return false;
}

// Whether grid cell `cell` holds any supersegment, from the occupancy bits
// (the exact walker needs no more than that from the count grid).
VDI_HD inline bool cell_occupied(const DevVDI &V, int cell)
{
    return (VDI_LOAD(V.gbits + ((uint32_t)cell >> 5), 1) >> ((uint32_t)cell & 31u)) & 1u;
}

// ---------------------------------------------------------------------------
// Exact render (Sections 4.1-4.3)
// ---------------------------------------------------------------------------
// One exact ray through V_N pixel (px, py); s_gz = slice boundaries (LDS copy).
// The ray steps through the list grid (voxel stepping in V_O NDC, Section
// 4.1), fetching the count of the list it enters next while it composites the
// current one; with ESS on it crosses grid cells of count 0 in one step
// (Section 4.3), keeping the current cell and depth slice from step to step.
template <int FMT, int SEARCH, bool ESS, bool COUNT>
VDI_HDI float4 trace_exact(const DevVDI &V, const Frame &F, const float *s_gz, int px, int py, Counters &cnt)
{
    Accum A = {0.0f, 0.0f, 0.0f, 1.0f};
    Ray r;
    const double xc = -1.0 + (2.0 * px + 1.0) / F.W, yc = -1.0 + (2.0 * py + 1.0) / F.H;
    if (!ray_setup(F, xc, yc, r)) return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int WO = V.WO, HO = V.HO, gk = V.gk;
    // Direction of travel across the list grid: d/dt (X/Z) has the sign of Kx.
    const double Kx = r.Xp * F.Z0 - F.X0 * r.Zp, Ky = r.Yp * F.Z0 - F.Y0 * r.Zp;
    const int sx = (Kx > 0.0) - (Kx < 0.0), sy = (Ky > 0.0) - (Ky < 0.0);
    const bool fwd = r.Zp >= 0.0, flat = fabs(r.Zp) < kFlatZ;
    const double inf = __builtin_huge_val();
    const double invZp = flat ? 0.0 : rcp64(r.Zp);
    double t = r.t0, tx = inf, ty = inf, tz = inf;
    // (ix, iy): current list; the next x (y) grid line crossed is ix + (sx > 0).
    int ix = 0, iy = 0, cz = 0;
    const int ox = sx > 0, oy = sy > 0;
    int ccell = -1;  // grid cell whose occupancy cg holds (fewer than 2^31 cells)
    bool cg = false;  // whether grid cell ccell is occupied
    auto slice_t = [&](int c) -> double {
        if (flat) return inf;
        if (fwd) return c + 1 < V.gnz ? ((double)s_gz[c + 1] - F.Z0) * invZp : inf;
        return c > 0 ? ((double)s_gz[c] - F.Z0) * invZp : inf;
    };
    auto locate = [&](double tt) {
        const double z = F.Z0 + tt * r.Zp;
        const double iz = rcp64(z);
        ix = cell_of((F.X0 + tt * r.Xp) * iz, WO, sx);
        iy = cell_of((F.Y0 + tt * r.Yp) * iz, HO, sy);
        const int mx = ix + ox, my = iy + oy;
        tx = (sx != 0 && mx > 0 && mx < WO) ? line_t(mx, V.dcx, F.X0, r.Xp, F.Z0, r.Zp) : inf;
        ty = (sy != 0 && my > 0 && my < HO) ? line_t(my, V.dcy, F.Y0, r.Yp, F.Z0, r.Zp) : inf;
        if constexpr (ESS) {
            cz = slice_of(s_gz, V.gnz, z, fwd);
            tz = slice_t(cz);
        }
    };
    locate(t);
    int p = -1;
    int n = VDI_LOAD(V.count + (uint64_t)iy * WO + ix, 0);
    // Every iteration moves one list or jumps a grid cell; the cap only
    // guards against a loop that does not advance.
    const int max_iter = 4 * (WO + HO) + 4 * V.gnz + 64;
    // Crossing of the next cell boundary in x (y) for a ray in cell column c.
    auto cell_tx = [&](int c) -> double {
        if (sx == 0) return inf;
        const int m = sx > 0 ? min((c + 1) * gk, WO) : c * gk;
        return (m > 0 && m < WO) ? line_t(m, V.dcx, F.X0, r.Xp, F.Z0, r.Zp) : inf;
    };
    auto cell_ty = [&](int c) -> double {
        if (sy == 0) return inf;
        const int m = sy > 0 ? min((c + 1) * gk, HO) : c * gk;
        return (m > 0 && m < HO) ? line_t(m, V.dcy, F.Y0, r.Yp, F.Z0, r.Zp) : inf;
    };
    // Cell mode (empty-space skipping): one empty grid cell per iteration, a
    // crossing and a grid load, no division; lanes in cell mode and in list
    // mode advance together.  Where a non-empty cell is entered the ray is
    // located again and walks lists.
    bool cellmode = false;
    for (int it = 0; it < max_iter; ++it) {
        VDI_STEP();
        if constexpr (ESS) {
            if (cellmode) {
                const double te = fmin(fmin(tx, ty), fmin(tz, r.t1));
                if (te >= r.t1) break;
                // One crossing solve per step whichever face the lanes leave by.
                const bool ax = tx <= ty && tx <= tz, ay = !ax && ty <= tz, az = !ax && !ay;
                ix += ax ? sx : 0;
                iy += ay ? sy : 0;
                cz += az ? (fwd ? 1 : -1) : 0;
                const int cc = ax ? ix : iy, sc = ax ? sx : sy, lim = ax ? WO : HO;
                const int m = sc > 0 ? min((cc + 1) * gk, lim) : cc * gk;
                const double tl = (sc != 0 && m > 0 && m < lim && !az)
                                      ? line_t(m, ax ? V.dcx : V.dcy, ax ? F.X0 : F.Y0, ax ? r.Xp : r.Yp, F.Z0, r.Zp)
                                      : inf;
                const double tzn = az ? slice_t(cz) : tz;
                tx = ax ? tl : tx;
                ty = ay ? tl : ty;
                tz = tzn;
                if ((unsigned)ix >= (unsigned)V.GW || (unsigned)iy >= (unsigned)V.GH || (unsigned)cz >= (unsigned)V.gnz)
                    break;
                t = fmax(t, te);
                const int cell = (cz * V.GH + iy) * V.GW + ix;
                if (cell_occupied(V, cell)) {
                    cellmode = false;
                    locate(t);
                    n = VDI_LOAD(V.count + (uint64_t)iy * WO + ix, 0);
                    ccell = -1;
                }
                continue;
            }
        }
        const double tn = fmin(fmin(tx, ty), r.t1);
        if constexpr (ESS) {
            while (tz <= t) {
                cz += fwd ? 1 : -1;
                tz = slice_t(cz);
            }
            const int cx = (int)((float)ix * V.inv_gk), cy = (int)((float)iy * V.inv_gk);
            const int cell = (cz * V.GH + cy) * V.GW + cx;
            if (cell != ccell) {
                cg = cell_occupied(V, cell);
                ccell = cell;
            }
            if (!cg) {
                // Empty-space skipping: switch to walking cells (ix, iy become
                // the cell indices, tx, ty the crossings of cell boundaries)
                // when that skips a list, i.e. the ray leaves its list before
                // the cell: otherwise the list step below reaches the list's
                // exit in one step where cells would take one per depth
                // slice.  Not either when the ray sits on the cell's exit (a
                // located position rounded onto a cell boundary): then the
                // list step moves it across.
                const double ctx = cell_tx(cx), cty = cell_ty(cy);
                const double te = fmin(fmin(ctx, cty), fmin(tz, r.t1));
                if (te > t && tn < te) {
                    ix = cx;
                    iy = cy;
                    tx = ctx;
                    ty = cty;
                    cellmode = true;
                    continue;
                }
            }
        }
        // The list entered next, and its count, are known before this one is composited.
        const bool stepx = tx <= ty;
        const int nx = stepx ? ix + sx : ix, ny = stepx ? iy : iy + sy;
        const bool more = tn < r.t1 && (unsigned)nx < (unsigned)WO && (unsigned)ny < (unsigned)HO;
        const int n_next = more ? VDI_LOAD(V.count + (uint64_t)ny * WO + nx, 0) : 0;
        if (tn > t && do_list<FMT, SEARCH, COUNT>(V, F, ix, iy, n, t, tn, F.Z0, r.Zp, invZp, A, p, cnt)) break;
        if (!more) break;
        {
            // One crossing solve per step, for the axis the ray stepped in.
            const int mm = stepx ? nx + ox : ny + oy, lim = stepx ? WO : HO;
            const double tl = (mm > 0 && mm < lim)
                                  ? line_t(mm, stepx ? V.dcx : V.dcy, stepx ? F.X0 : F.Y0, stepx ? r.Xp : r.Yp, F.Z0, r.Zp)
                                  : inf;
            tx = stepx ? tl : tx;
            ty = stepx ? ty : tl;
        }
        ix = nx;
        iy = ny;
        n = n_next;
        t = fmax(t, tn);
    }
    return make_float4(A.r, A.g, A.b, 1.0f - A.T);
}

// ---------------------------------------------------------------------------
// Preview: adaptive along-ray subsampling (Section 4.4)
// ---------------------------------------------------------------------------
// Shift, in V_O pixels, added to a preview sample's list coordinates: far
// above the FP64 rounding of a coordinate (about 1e-12 pixel at 16384
// lists) and far below any distance that decides a sample off a tie.
constexpr double kTieShift = 1e-9;

// Part `part` of `parts` of the preview ray through V_N pixel (px, py) of
// the (low-res) grid: the samples of a contiguous block of the grid cells the
// ray crosses, composited front to back from full transmittance.  The blocks
// cut the ray's parameter range into equal parts, each cut moved back to the
// entry of the cell it falls in; a part starts at its first cell and stops
// where the next part starts, so together the parts take exactly the samples
// of the whole ray (parts = 1).
// With COUNT, also marks what the part read: every grid cell whose count
// it read (touched_cells), the list of every sample (touched_lists) and every
// supersegment it composited (touched_slots), counted in cnt as samples
// (lists) and pieces.
template <int FMT, bool COUNT = false>
VDI_HDI Accum trace_preview(const DevVDI &V, const Frame &F, const float *s_gz, int px, int py, int part = 0,
                           int parts = 1, Counters *cnt = nullptr)
{
    Accum A = {0.0f, 0.0f, 0.0f, 1.0f};
    Ray r;
    const double xc = -1.0 + (2.0 * px + 1.0) / F.W, yc = -1.0 + (2.0 * py + 1.0) / F.H;
    if (ray_setup(F, xc, yc, r)) {
        const int WO = V.WO, HO = V.HO, k = V.gk;
        const double Kx = r.Xp * F.Z0 - F.X0 * r.Zp, Ky = r.Yp * F.Z0 - F.Y0 * r.Zp;
        const int sx = (Kx > 0.0) - (Kx < 0.0), sy = (Ky > 0.0) - (Ky < 0.0);
        const bool fwd = r.Zp >= 0.0;
        const bool flat = fabs(r.Zp) < kFlatZ;
        const double inf = __builtin_huge_val();
        const double invZp = flat ? 0.0 : rcp64(r.Zp);
        const double inv_k2 = 1.0 / (double)(k * k);
        const float2 *__restrict__ dep = V.depth;
        const uint64_t stride = slot_stride(V);
        double t = r.t0;
        int cx, cy, cz, mx, my;
        double tx, ty, tz;
        // Cell of the point at parameter tt (point location).
        auto cell_at = [&](double tt) {
            const double z = F.Z0 + tt * r.Zp;
            cx = (int)((float)cell_of((F.X0 + tt * r.Xp) / z, WO, sx) * V.inv_gk);
            cy = (int)((float)cell_of((F.Y0 + tt * r.Yp) / z, HO, sy) * V.inv_gk);
            cz = slice_of(s_gz, V.gnz, z, fwd);
        };
        auto locate = [&](double tt) {
            cell_at(tt);
            mx = sx > 0 ? min((cx + 1) * k, WO) : cx * k;
            my = sy > 0 ? min((cy + 1) * k, HO) : cy * k;
            tx = (sx != 0 && mx > 0 && mx < WO) ? line_t(mx, V.dcx, F.X0, r.Xp, F.Z0, r.Zp) : inf;
            ty = (sy != 0 && my > 0 && my < HO) ? line_t(my, V.dcy, F.Y0, r.Yp, F.Z0, r.Zp) : inf;
            if (flat)
                tz = inf;
            else if (fwd)
                tz = cz + 1 < V.gnz ? ((double)s_gz[cz + 1] - F.Z0) * invZp : inf;
            else
                tz = cz > 0 ? ((double)s_gz[cz] - F.Z0) * invZp : inf;
        };
        // The cell the walk is in at parameter u, and the parameter at which
        // the walk enters it.  The walk moves between cells at face crossings
        // computed by line_t (list-grid lines) and from the slice depths, so
        // its cell at u is, axis by axis, the one whose entry face is crossed
        // at or before u and whose exit face after u, with those crossings.
        // Point location (which divides a position instead) gives the first
        // guess, right but for a rounding error near a face; each axis is then
        // moved until its faces bracket u.  The entry is the latest of the
        // three entry crossings.  A face the walk never crosses (no grid line
        // there, or a line beyond the vanishing point: +inf from the crossing
        // functions) counts as crossed at -inf where it is the entry.
        auto x_face = [&](int m) -> double {
            return (m > 0 && m < WO) ? line_t(m, V.dcx, F.X0, r.Xp, F.Z0, r.Zp) : inf;
        };
        auto y_face = [&](int m) -> double {
            return (m > 0 && m < HO) ? line_t(m, V.dcy, F.Y0, r.Yp, F.Z0, r.Zp) : inf;
        };
        auto z_face = [&](int c) -> double {  // slice boundary c, 0 < c < gnz
            return (c > 0 && c < V.gnz) ? ((double)s_gz[c] - F.Z0) * invZp : inf;
        };
        auto enter = [&](double tf) -> double { return tf == inf ? -inf : tf; };
        auto entry_at = [&](double u) -> double {
            cell_at(u);
            double te = r.t0;
            // Each crossing is solved once: moving on, a cell's exit face is
            // the next cell's entry face, and moving back the other way round.
            if (sx != 0) {
                auto in_m = [&](int c) { return sx > 0 ? c * k : (c + 1) * k; };
                auto out_m = [&](int c) { return sx > 0 ? min((c + 1) * k, WO) : c * k; };
                double ti = enter(x_face(in_m(cx))), to = x_face(out_m(cx));
#pragma nounroll
                for (int g = 0; g < 4; ++g) {
                    if (to <= u && (unsigned)(cx + sx) < (unsigned)V.GW) {
                        cx += sx;
                        ti = to;
                        to = x_face(out_m(cx));
                    } else if (ti > u && (unsigned)(cx - sx) < (unsigned)V.GW) {
                        cx -= sx;
                        to = ti;
                        ti = enter(x_face(in_m(cx)));
                    } else {
                        break;
                    }
                }
                te = fmax(te, ti);
                mx = out_m(cx);
                tx = to;
            } else {
                tx = inf;
            }
            if (sy != 0) {
                auto in_m = [&](int c) { return sy > 0 ? c * k : (c + 1) * k; };
                auto out_m = [&](int c) { return sy > 0 ? min((c + 1) * k, HO) : c * k; };
                double ti = enter(y_face(in_m(cy))), to = y_face(out_m(cy));
#pragma nounroll
                for (int g = 0; g < 4; ++g) {
                    if (to <= u && (unsigned)(cy + sy) < (unsigned)V.GH) {
                        cy += sy;
                        ti = to;
                        to = y_face(out_m(cy));
                    } else if (ti > u && (unsigned)(cy - sy) < (unsigned)V.GH) {
                        cy -= sy;
                        to = ti;
                        ti = enter(y_face(in_m(cy)));
                    } else {
                        break;
                    }
                }
                te = fmax(te, ti);
                my = out_m(cy);
                ty = to;
            } else {
                ty = inf;
            }
            if (!flat) {
                const int dz = fwd ? 1 : -1;
                auto in_c = [&](int c) { return fwd ? c : c + 1; };
                auto out_c = [&](int c) { return fwd ? c + 1 : c; };
                double ti = enter(z_face(in_c(cz))), to = z_face(out_c(cz));
#pragma nounroll
                for (int g = 0; g < 4; ++g) {
                    if (to <= u && (unsigned)(cz + dz) < (unsigned)V.gnz) {
                        cz += dz;
                        ti = to;
                        to = z_face(out_c(cz));
                    } else if (ti > u && (unsigned)(cz - dz) < (unsigned)V.gnz) {
                        cz -= dz;
                        to = ti;
                        ti = enter(z_face(in_c(cz)));
                    } else {
                        break;
                    }
                }
                te = fmax(te, ti);
                tz = to;
            } else {
                tz = inf;
            }
            return te;
        };
        // Lane `part` takes the cells the walk enters in [its start, t_stop):
        // the ray's parameter range cut into equal parts, each cut moved back
        // to the entry of the cell it falls in, so the lanes need not walk the
        // cells before their own.
        double t_stop = inf;
        if (parts > 1 && part > 0) {
            // One call site for both cuts (the next lane's start, where this
            // lane stops, then this lane's own start), so the code is inlined once.
            const double span = r.t1 - r.t0;
#pragma nounroll
            for (int w = part + 1 < parts ? 0 : 1; w < 2; ++w) {
                const double te = entry_at(r.t0 + span * (w == 0 ? part + 1 : part) / parts);
                if (w == 0) t_stop = te;
                else t = te;
            }
        } else {
            if (parts > 1) t_stop = entry_at(r.t0 + (r.t1 - r.t0) / parts);
            locate(t);
        }
        int p = -1;
        const int max_iter = 4 * (WO + HO) / k + 4 * V.gnz + 64;
        // List of sample q of the current cell (its count is fetched one sample ahead).
        // A sample on a list edge belongs to the list on its +x (+y) side,
        // the half-open cell rule; the shift of kTieShift pixel keeps that
        // decision the same for every such sample of a ray, where rounding
        // alone would put them on either side (a ray lying in an edge plane,
        // e.g. a downsampled view from the generating viewpoint).
        double h = 0.0;
        auto sample_list = [&](int q, double &u, double &z, int &lx, int &ly) {
            u = t + (q + 0.5) * h;
            z = F.Z0 + u * r.Zp;
            const double iz = rcp64(z);
            const double fx = ((F.X0 + u * r.Xp) * iz + 1.0) * (0.5 * WO) + kTieShift;
            const double fy = ((F.Y0 + u * r.Yp) * iz + 1.0) * (0.5 * HO) + kTieShift;
            lx = min(max((int)floor(fx), 0), WO - 1);
            ly = min(max((int)floor(fy), 0), HO - 1);
        };
        // One flat loop: every step either enters the current grid cell (and,
        // when the cell is non-empty, sets up its samples) or takes one
        // sample.  Lanes of a wavefront that are crossing empty cells and
        // lanes that are sampling thus advance together, instead of a cell
        // step waiting for the wavefront's longest run of samples in a cell.
        int it = 0;        // cells entered
        int q = 0, n = 0;  // sample q of n in the current cell; n == 0 between cells
        double tn = 0.0, u = 0.0, z = 0.0;
        int lx = 0, ly = 0;
        int nl = 0;
        for (;;) {
            bool advance = true;
            if (n == 0) {
                if (it >= max_iter || t >= t_stop) break;
                tn = fmin(fmin(fmin(tx, ty), tz), r.t1);
                if (tn > t) {
                    const uint64_t cell = ((uint64_t)cz * V.GH + cy) * V.GW + cx;
                    const uint32_t G = VDI_LOAD(V.grid + (cell), 1);
                    if constexpr (COUNT) F.touched_cells[cell] = 1;
                    if (G != 0u) {
                        const double dz = (double)s_gz[cz + 1] - (double)s_gz[cz];
                        const double x = ((tn - t) / dz) * ((double)G * inv_k2) / F.DR;
                        // D_R >= 1e-4 keeps x far below this bound; it only caps the loop.
                        n = (int)fmin(fmax(ceil(x), 1.0), 16777216.0);
                        h = (tn - t) / n;
                        q = 0;
                        sample_list(0, u, z, lx, ly);
                        nl = VDI_LOAD(V.count + ((uint64_t)ly * WO + lx), 0);
                        advance = false;
                    }
                }
            } else {
                double un = 0.0, zn = 0.0;
                int lxn = lx, lyn = ly;
                if (q + 1 < n) sample_list(q + 1, un, zn, lxn, lyn);
                const int nln = q + 1 < n ? (int)VDI_LOAD(V.count + ((uint64_t)lyn * WO + lxn), 0) : 0;
                if constexpr (COUNT) {
                    F.touched_lists[(uint64_t)ly * WO + lx] = 1;
                    ++cnt->lists;
                }
                if (nl > 0) {
                    // Point location: the supersegment with f <= z < b.
                    const uint64_t lb = list_base_xy(lx, ly, V.NS, WO);
                    const int j = first_back_above_win<true>(dep, stride, lb, nl, z, fwd ? win_start_fwd(p) : win_start_bwd(p));
                    if (j < nl) {
                        const float2 fb = VDI_LOAD(dep + ((uint64_t)j * stride + lb), 2);
                        p = j;
                        if ((double)fb.x <= z) {
                            const float4 c = load_rgba<FMT>(V.rgba, (uint64_t)j * stride + lb, V.fmt);
                            composite(A, c, (float)h * list_cos(V, lx, ly) * rcp32(fb.y - fb.x));
                            if constexpr (COUNT) {
                                F.touched_slots[(uint64_t)j * V.plane + (uint64_t)ly * WO + lx] = 1;
                                ++cnt->pieces;
                            }
                            if (A.T <= kTTerm) break;
                        }
                    }
                }
                lx = lxn;
                ly = lyn;
                nl = nln;
                u = un;
                z = zn;
                ++q;
                advance = q == n;
                if (advance) n = 0;
            }
            if (!advance) continue;
            if (tn >= r.t1) break;
            if (tx <= ty && tx <= tz) {
                cx += sx;
                mx = sx > 0 ? min((cx + 1) * k, WO) : cx * k;
                tx = (mx > 0 && mx < WO) ? line_t(mx, V.dcx, F.X0, r.Xp, F.Z0, r.Zp) : inf;
            } else if (ty <= tz) {
                cy += sy;
                my = sy > 0 ? min((cy + 1) * k, HO) : cy * k;
                ty = (my > 0 && my < HO) ? line_t(my, V.dcy, F.Y0, r.Yp, F.Z0, r.Zp) : inf;
            } else {
                cz += fwd ? 1 : -1;
                if (fwd)
                    tz = cz + 1 < V.gnz ? ((double)s_gz[cz + 1] - F.Z0) * invZp : inf;
                else
                    tz = cz > 0 ? ((double)s_gz[cz] - F.Z0) * invZp : inf;
            }
            t = fmax(t, tn);
            ++it;
            if ((unsigned)cx >= (unsigned)V.GW || (unsigned)cy >= (unsigned)V.GH || (unsigned)cz >= (unsigned)V.gnz)
                break;
        }
    }
    return A;
}

// "over" of a front and a back partial result of one ray.
VDI_HD inline Accum over(const Accum &f, const Accum &b)
{
    return {fmaf(f.T, b.r, f.r), fmaf(f.T, b.g, f.g), fmaf(f.T, b.b, f.b), f.T * b.T};
}

// Combine the partial results of the `parts` lanes of each ray (adjacent
// lanes, part = lane % parts, parts a power of two) in ray order: pairs, then
// pairs of pairs.  Every lane of the group ends with the same result.
__device__ inline Accum combine_parts(Accum a, int parts, int lane)
{
    for (int m = 1; m < parts; m <<= 1) {
        const Accum o = {__shfl_xor(a.r, m), __shfl_xor(a.g, m), __shfl_xor(a.b, m), __shfl_xor(a.T, m)};
        a = (lane & m) ? over(o, a) : over(a, o);
    }
    return a;
}

VDI_HD inline float4 to_rgba(const Accum &A) { return make_float4(A.r, A.g, A.b, 1.0f - A.T); }


// ---------------------------------------------------------------------------
// Bilinear upsampling of one output pixel (x, y) of a W x H image from a
// w x h image, half-pixel centres, clamped (Section 4.4, Fig. 7 caption).
// ---------------------------------------------------------------------------
// `texel(i)` gives texel i of the low-res image (row-major).
template <typename Texel>
VDI_HD inline float4 upsample_px_by(const Texel &texel, int w, int h, int W, int H, int x, int y)
{
    double sx = (x + 0.5) * (double)w / W - 0.5, sy = (y + 0.5) * (double)h / H - 0.5;
    sx = fmin(fmax(sx, 0.0), (double)(w - 1));
    sy = fmin(fmax(sy, 0.0), (double)(h - 1));
    const int x0 = (int)sx, y0 = (int)sy;
    const int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    const float fx = (float)(sx - x0), fy = (float)(sy - y0);
    const float4 a = texel((uint64_t)y0 * w + x0), b = texel((uint64_t)y0 * w + x1);
    const float4 c = texel((uint64_t)y1 * w + x0), d = texel((uint64_t)y1 * w + x1);
    // Explicit fused multiply-adds: the result does not depend on how a
    // compiler contracts the expression in the kernel it is inlined into.
    auto mix = [&](float pa, float pb, float pc, float pd) {
        const float top = fmaf(fx, pb - pa, pa), bot = fmaf(fx, pd - pc, pc);
        return fmaf(fy, bot - top, top);
    };
    return make_float4(mix(a.x, b.x, c.x, d.x), mix(a.y, b.y, c.y, d.y), mix(a.z, b.z, c.z, d.z),
                       mix(a.w, b.w, c.w, d.w));
}

VDI_HD inline float4 upsample_px(const float4 *__restrict__ lo, int w, int h, int W, int H, int x, int y)
{
    return upsample_px_by([lo](uint64_t i) { return lo[i]; }, w, h, W, H, x, y);
}

}  // namespace vdi
